// Internal launchers of the warm-start network kernels (nn_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace elwh {
namespace nn {

void gemm(hipStream_t s, bool ta, bool tb, int M, int N, int K, const unsigned short* A, int lda,
          const unsigned short* B, int ldb, float* C, int ldc, int splits, float* part, int accumulate);
void to_bf16(hipStream_t s, const float* x, unsigned short* y, int64_t n);
void im2col(hipStream_t s, const float* X, unsigned short* col, int B, int H, int W, int C);
void col2im(hipStream_t s, const float* dcol, float* dX, int B, int H, int W, int C);
void bias_act(hipStream_t s, float* Z, float* A, const float* bias, int64_t npix, int C, int act);
void act_back(hipStream_t s, float* dA, const float* Z, int64_t n, int act);
void channel_sum(hipStream_t s, const float* X, int64_t npix, int C, float* part, int nchunks, float* out,
                 int accumulate);
void avgpool(hipStream_t s, const float* X, float* Y, int B, int H, int W, int C);
void avgpool_back(hipStream_t s, const float* dY, float* dX, int B, int H, int W, int C, int accumulate);
void upsample(hipStream_t s, const float* X, float* Y, int B, int H, int W, int C, int Cy, int coff);
void upsample_back(hipStream_t s, const float* dY, float* dX, int B, int H, int W, int C, int Cy, int coff);
void copy_channels(hipStream_t s, const float* X, int Cx, int xoff, float* Y, int Cy, int yoff, int64_t npix, int C,
                   int accumulate);
void loss(hipStream_t s, const float* yh, const float* y, const float* w, int B, int64_t npix_per, int C, float* dyh,
          float* loss_per);
void adam(hipStream_t s, float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
          float eps, int step);

}  // namespace nn
}  // namespace elwh
