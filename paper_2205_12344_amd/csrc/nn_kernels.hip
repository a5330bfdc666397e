// Kernels of the warm-start network: BF16 MFMA GEMM with FP32 accumulation
// (the convolutions, as GEMMs over an im2col matrix), im2col / col2im, SiLU, pooling,
// upsampling, channel copies, loss and Adam.  Activations are NHWC FP32;
// GEMM operands are BF16.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "nn_internal.h"

namespace elwh {
namespace nn {

// ---- BF16 helpers (round to nearest even) ----------------------------------
__device__ __forceinline__ unsigned short f2bf(float f) {
    unsigned int u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)((u >> 16) | ((u & 0xffff) ? 0x40 : 0));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short b) { return __uint_as_float(((unsigned int)b) << 16); }

// ---- GEMM ------------------------------------------------------------------
// C[z][m][n] = sum_{k in split z} A(m,k) B(k,n);  A(m,k) = TA ? A[k*lda+m] : A[m*lda+k],
// B(k,n) = TB ? B[n*ldb+k] : B[k*ldb+n].  Block: 256 threads = 4 wavefronts in a
// 2x2 arrangement of 32x32 output tiles (64x64 per block); K in chunks of 32
// staged through LDS with k contiguous; gfx950's v_mfma_f32_32x32x16_bf16 per
// 16 k (lane l holds A(row l mod 32, k 8 (l / 32) .. + 7) and the same slice
// of B; twice the k of the older 32x32x8 instruction per issue).
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float float16_t __attribute__((ext_vector_type(16)));

constexpr int GT = 64, GK = 32, GKP = GK + 8;   // tile, k chunk, padded LDS row

template <bool TA, bool TB>
__global__ __launch_bounds__(256) void gemm_bf16_kernel(int M, int N, int K, int kchunk, const unsigned short* __restrict__ A,
                                                        int lda, const unsigned short* __restrict__ B, int ldb,
                                                        float* __restrict__ C, int ldc, int64_t zstride) {
    __shared__ unsigned short As[GT][GKP];
    __shared__ unsigned short Bs[GT][GKP];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
    const int kbeg = blockIdx.z * kchunk, kend = min(K, kbeg + kchunk);
    const int wm = w >> 1, wn = w & 1;
    float16_t acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.f;

    for (int k0 = kbeg; k0 < kend; k0 += GK) {
        // A tile: 64 (m) x 32 (k)
        if (!TA) {
            const int m = t >> 2, k8 = (t & 3) * 8;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int gm = m0 + m, gk = k0 + k8 + e;
                As[m][k8 + e] = (gm < M && gk < kend) ? A[(int64_t)gm * lda + gk] : (unsigned short)0;
            }
        } else {
            const int m8 = (t & 7) * 8, k = t >> 3;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int gm = m0 + m8 + e, gk = k0 + k;
                As[m8 + e][k] = (gm < M && gk < kend) ? A[(int64_t)gk * lda + gm] : (unsigned short)0;
            }
        }
        // B tile: 32 (k) x 64 (n), stored [n][k]
        if (!TB) {
            const int n8 = (t & 7) * 8, k = t >> 3;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int gn = n0 + n8 + e, gk = k0 + k;
                Bs[n8 + e][k] = (gn < N && gk < kend) ? B[(int64_t)gk * ldb + gn] : (unsigned short)0;
            }
        } else {
            const int n = t >> 2, k8 = (t & 3) * 8;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int gn = n0 + n, gk = k0 + k8 + e;
                Bs[n][k8 + e] = (gn < N && gk < kend) ? B[(int64_t)gn * ldb + gk] : (unsigned short)0;
            }
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < GK; ks += 16) {
            const int kk = ks + (lane >> 5) * 8;   // <= 31 < GKP
            const unsigned short* ap = &As[wm * 32 + (lane & 31)][kk];
            const unsigned short* bp = &Bs[wn * 32 + (lane & 31)][kk];
            bf16x8_t a, b;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                a[e] = __builtin_bit_cast(__bf16, ap[e]);
                b[e] = __builtin_bit_cast(__bf16, bp[e]);
            }
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
        }
        __syncthreads();
    }
    float* Cz = C + (int64_t)blockIdx.z * zstride;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int gm = m0 + wm * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int gn = n0 + wn * 32 + (lane & 31);
        if (gm < M && gn < N) Cz[(int64_t)gm * ldc + gn] = acc[r];
    }
}

__global__ void sum_splits_kernel(const float* __restrict__ part, int splits, int64_t n, float* __restrict__ out,
                                  int accumulate) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        float s = 0.f;
        for (int z = 0; z < splits; ++z) s += part[(int64_t)z * n + e];
        out[e] = accumulate ? out[e] + s : s;
    }
}

// ---- conversions, im2col, col2im -------------------------------------------
__global__ void to_bf16_kernel(const float* __restrict__ x, unsigned short* __restrict__ y, int64_t n) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        y[e] = f2bf(x[e]);
}

// col[(b,y,x)][(ky*3+kx)*C + c] = X[b, y+ky-1, x+kx-1, c] (zero outside)
__global__ void im2col_kernel(const float* __restrict__ X, unsigned short* __restrict__ col, int B, int H, int W,
                              int C) {
    const int64_t K = 9LL * C;
    const int64_t total = (int64_t)B * H * W * K;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t pix = e / K;
        const int kidx = (int)(e - pix * K);
        const int tap = kidx / C, c = kidx - tap * C;
        const int ky = tap / 3, kx = tap - ky * 3;
        const int x = (int)(pix % W);
        const int64_t r = pix / W;
        const int y = (int)(r % H);
        const int b = (int)(r / H);
        const int yy = y + ky - 1, xx = x + kx - 1;
        float v = 0.f;
        if (yy >= 0 && yy < H && xx >= 0 && xx < W) v = X[(((int64_t)b * H + yy) * W + xx) * C + c];
        col[e] = f2bf(v);
    }
}

// dX[b,y,x,c] = sum over taps of dcol[(b, y-ky+1, x-kx+1)][(ky*3+kx)*C + c]
__global__ void col2im_kernel(const float* __restrict__ dcol, float* __restrict__ dX, int B, int H, int W, int C) {
    const int64_t total = (int64_t)B * H * W * C;
    const int64_t K = 9LL * C;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(e % C);
        const int64_t pix = e / C;
        const int x = (int)(pix % W);
        const int64_t r = pix / W;
        const int y = (int)(r % H);
        const int b = (int)(r / H);
        float s = 0.f;
#pragma unroll
        for (int ky = 0; ky < 3; ++ky)
#pragma unroll
            for (int kx = 0; kx < 3; ++kx) {
                const int yy = y - ky + 1, xx = x - kx + 1;
                if (yy >= 0 && yy < H && xx >= 0 && xx < W)
                    s += dcol[(((int64_t)b * H + yy) * W + xx) * K + (ky * 3 + kx) * C + c];
            }
        dX[e] = s;
    }
}

// ---- elementwise -------------------------------------------------------------
__device__ __forceinline__ float sigm(float z) { return 1.f / (1.f + __expf(-z)); }

// Z = Y + bias (in place), A = silu(Z) (or A = Z when act == 0)
__global__ void bias_act_kernel(float* __restrict__ Z, float* __restrict__ A, const float* __restrict__ bias,
                                int64_t npix, int C, int act) {
    const int64_t n = npix * C;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const float z = Z[e] + bias[e % C];
        Z[e] = z;
        A[e] = act ? z * sigm(z) : z;
    }
}

// dZ = dA * silu'(Z) (in place on dA) when act; identity otherwise
__global__ void act_back_kernel(float* __restrict__ dA, const float* __restrict__ Z, int64_t n, int act) {
    if (!act) return;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const float z = Z[e], s = sigm(z);
        dA[e] *= s * (1.f + z * (1.f - s));
    }
}

// per-channel partial sums over pixel chunks: part[chunk][c]
__global__ void channel_sum_partial_kernel(const float* __restrict__ X, int64_t npix, int C, int chunk,
                                           float* __restrict__ part) {
    const int c = threadIdx.x + blockIdx.y * blockDim.x;
    if (c >= C) return;
    const int64_t p0 = (int64_t)blockIdx.x * chunk, p1 = min(npix, p0 + chunk);
    float s = 0.f;
    for (int64_t p = p0; p < p1; ++p) s += X[p * C + c];
    part[(int64_t)blockIdx.x * C + c] = s;
}

__global__ void avgpool_kernel(const float* __restrict__ X, float* __restrict__ Y, int B, int H, int W, int C) {
    const int Ho = H / 2, Wo = W / 2;
    const int64_t n = (int64_t)B * Ho * Wo * C;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(e % C);
        int64_t r = e / C;
        const int x = (int)(r % Wo);
        r /= Wo;
        const int y = (int)(r % Ho);
        const int b = (int)(r / Ho);
        const float* p = X + (((int64_t)b * H + 2 * y) * W + 2 * x) * C + c;
        Y[e] = 0.25f * (p[0] + p[C] + p[(int64_t)W * C] + p[(int64_t)W * C + C]);
    }
}

__global__ void avgpool_back_kernel(const float* __restrict__ dY, float* __restrict__ dX, int B, int H, int W, int C,
                                    int accumulate) {
    const int Ho = H / 2, Wo = W / 2;
    const int64_t n = (int64_t)B * H * W * C;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(e % C);
        int64_t r = e / C;
        const int x = (int)(r % W);
        r /= W;
        const int y = (int)(r % H);
        const int b = (int)(r / H);
        const float g = 0.25f * dY[(((int64_t)b * Ho + y / 2) * Wo + x / 2) * C + c];
        dX[e] = accumulate ? dX[e] + g : g;
    }
}

// nearest upsampling by 2 of X (B,H,W,C) into channels [coff, coff+C) of Y (B,2H,2W,Cy)
__global__ void upsample_kernel(const float* __restrict__ X, float* __restrict__ Y, int B, int H, int W, int C,
                                int Cy, int coff) {
    const int64_t n = (int64_t)B * 4 * H * W * C;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(e % C);
        int64_t r = e / C;
        const int x = (int)(r % (2 * W));
        r /= 2 * W;
        const int y = (int)(r % (2 * H));
        const int b = (int)(r / (2 * H));
        Y[(((int64_t)b * 2 * H + y) * 2 * W + x) * Cy + coff + c] = X[(((int64_t)b * H + y / 2) * W + x / 2) * C + c];
    }
}

// dX (B,H,W,C) = sum of the 4 children of dY channels [coff, coff+C)
__global__ void upsample_back_kernel(const float* __restrict__ dY, float* __restrict__ dX, int B, int H, int W, int C,
                                     int Cy, int coff) {
    const int64_t n = (int64_t)B * H * W * C;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(e % C);
        int64_t r = e / C;
        const int x = (int)(r % W);
        r /= W;
        const int y = (int)(r % H);
        const int b = (int)(r / H);
        const int64_t W2 = 2 * W;
        const float* p = dY + (((int64_t)b * 2 * H + 2 * y) * W2 + 2 * x) * Cy + coff + c;
        dX[e] = p[0] + p[Cy] + p[W2 * Cy] + p[W2 * Cy + Cy];
    }
}

// copy channels: Y[..., yoff + c] = X[..., xoff + c], c < C  (npix pixels)
__global__ void copy_channels_kernel(const float* __restrict__ X, int Cx, int xoff, float* __restrict__ Y, int Cy,
                                     int yoff, int64_t npix, int C, int accumulate) {
    const int64_t n = npix * C;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(e % C);
        const int64_t p = e / C;
        const float v = X[p * Cx + xoff + c];
        float& d = Y[p * Cy + yoff + c];
        d = accumulate ? d + v : v;
    }
}

// Relative error in the weighted norm, per sample b:
//   L = (1/B) sum_b sum w (yh - y)^2 / sum w y^2 ;  dyh = (2/B) w (yh - y) / den_b
__global__ __launch_bounds__(256) void loss_kernel(const float* __restrict__ yh, const float* __restrict__ y,
                                                   const float* __restrict__ w, int B, int64_t npix_per, int C,
                                                   float* __restrict__ dyh, float* __restrict__ loss_per) {
    const int b = blockIdx.x;
    __shared__ float sn[256], sd[256];
    float num = 0.f, den = 0.f;
    const int64_t n = npix_per * C;
    const float* yb = y + (int64_t)b * n;
    const float* yhb = yh + (int64_t)b * n;
    const float* wb = w + (int64_t)b * npix_per;
    for (int64_t e = threadIdx.x; e < n; e += 256) {
        const float ww = wb[e / C], d = yhb[e] - yb[e];
        num += ww * d * d;
        den += ww * yb[e] * yb[e];
    }
    sn[threadIdx.x] = num;
    sd[threadIdx.x] = den;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            sn[threadIdx.x] += sn[threadIdx.x + s];
            sd[threadIdx.x] += sd[threadIdx.x + s];
        }
        __syncthreads();
    }
    const float D = sd[0] > 0.f ? sd[0] : 1.f;
    if (threadIdx.x == 0) loss_per[b] = sn[0] / D / B;
    if (dyh)
        for (int64_t e = threadIdx.x; e < n; e += 256)
            dyh[(int64_t)b * n + e] = 2.f / B * wb[e / C] * (yhb[e] - yb[e]) / D;
}

__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float c1,
                            float c2) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const float gg = g[e];
        const float mm = b1 * m[e] + (1.f - b1) * gg;
        const float vv = b2 * v[e] + (1.f - b2) * gg * gg;
        m[e] = mm;
        v[e] = vv;
        p[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
    }
}

unsigned grid1(int64_t n) {
    const int64_t g = (n + 255) / 256;
    return (unsigned)(g < 1 ? 1 : (g > 65536 ? 65536 : g));
}

}  // namespace nn

// ---- launchers ----------------------------------------------------------------
namespace nn {

void gemm(hipStream_t s, bool ta, bool tb, int M, int N, int K, const unsigned short* A, int lda,
          const unsigned short* B, int ldb, float* C, int ldc, int splits, float* part, int accumulate) {
    splits = splits < 1 ? 1 : splits;
    int kchunk = (K + splits - 1) / splits;
    kchunk = (kchunk + GK - 1) / GK * GK;
    splits = (K + kchunk - 1) / kchunk;
    dim3 g((unsigned)((N + GT - 1) / GT), (unsigned)((M + GT - 1) / GT), (unsigned)splits);
    float* dst = (splits > 1 || accumulate) ? part : C;
    const int ldd = (splits > 1 || accumulate) ? N : ldc;
    const int64_t zs = (int64_t)M * N;
#define GL(TA_, TB_) hipLaunchKernelGGL((gemm_bf16_kernel<TA_, TB_>), g, dim3(256), 0, s, M, N, K, kchunk, A, lda, B, ldb, dst, ldd, zs)
    if (!ta && !tb) GL(false, false);
    else if (!ta && tb) GL(false, true);
    else if (ta && !tb) GL(true, false);
    else GL(true, true);
#undef GL
    if (splits > 1 || accumulate) {
        // ldc == N for the split path (callers use dense C)
        hipLaunchKernelGGL(sum_splits_kernel, dim3(grid1(zs)), dim3(256), 0, s, part, splits, zs, C, accumulate);
    }
}

void to_bf16(hipStream_t s, const float* x, unsigned short* y, int64_t n) {
    hipLaunchKernelGGL(to_bf16_kernel, dim3(grid1(n)), dim3(256), 0, s, x, y, n);
}
void im2col(hipStream_t s, const float* X, unsigned short* col, int B, int H, int W, int C) {
    hipLaunchKernelGGL(im2col_kernel, dim3(grid1((int64_t)B * H * W * 9 * C)), dim3(256), 0, s, X, col, B, H, W, C);
}
void col2im(hipStream_t s, const float* dcol, float* dX, int B, int H, int W, int C) {
    hipLaunchKernelGGL(col2im_kernel, dim3(grid1((int64_t)B * H * W * C)), dim3(256), 0, s, dcol, dX, B, H, W, C);
}
void bias_act(hipStream_t s, float* Z, float* A, const float* bias, int64_t npix, int C, int act) {
    hipLaunchKernelGGL(bias_act_kernel, dim3(grid1(npix * C)), dim3(256), 0, s, Z, A, bias, npix, C, act);
}
void act_back(hipStream_t s, float* dA, const float* Z, int64_t n, int act) {
    hipLaunchKernelGGL(act_back_kernel, dim3(grid1(n)), dim3(256), 0, s, dA, Z, n, act);
}
void channel_sum(hipStream_t s, const float* X, int64_t npix, int C, float* part, int nchunks, float* out,
                 int accumulate) {
    const int chunk = (int)((npix + nchunks - 1) / nchunks);
    nchunks = (int)((npix + chunk - 1) / chunk);
    dim3 g((unsigned)nchunks, (unsigned)((C + 63) / 64));
    hipLaunchKernelGGL(channel_sum_partial_kernel, g, dim3(64), 0, s, X, npix, C, chunk, part);
    hipLaunchKernelGGL(sum_splits_kernel, dim3(grid1(C)), dim3(256), 0, s, part, nchunks, (int64_t)C, out, accumulate);
}
void avgpool(hipStream_t s, const float* X, float* Y, int B, int H, int W, int C) {
    hipLaunchKernelGGL(avgpool_kernel, dim3(grid1((int64_t)B * H * W * C / 4)), dim3(256), 0, s, X, Y, B, H, W, C);
}
void avgpool_back(hipStream_t s, const float* dY, float* dX, int B, int H, int W, int C, int accumulate) {
    hipLaunchKernelGGL(avgpool_back_kernel, dim3(grid1((int64_t)B * H * W * C)), dim3(256), 0, s, dY, dX, B, H, W, C,
                       accumulate);
}
void upsample(hipStream_t s, const float* X, float* Y, int B, int H, int W, int C, int Cy, int coff) {
    hipLaunchKernelGGL(upsample_kernel, dim3(grid1((int64_t)B * 4 * H * W * C)), dim3(256), 0, s, X, Y, B, H, W, C, Cy,
                       coff);
}
void upsample_back(hipStream_t s, const float* dY, float* dX, int B, int H, int W, int C, int Cy, int coff) {
    hipLaunchKernelGGL(upsample_back_kernel, dim3(grid1((int64_t)B * H * W * C)), dim3(256), 0, s, dY, dX, B, H, W, C,
                       Cy, coff);
}
void copy_channels(hipStream_t s, const float* X, int Cx, int xoff, float* Y, int Cy, int yoff, int64_t npix, int C,
                   int accumulate) {
    hipLaunchKernelGGL(copy_channels_kernel, dim3(grid1(npix * C)), dim3(256), 0, s, X, Cx, xoff, Y, Cy, yoff, npix, C,
                       accumulate);
}
void loss(hipStream_t s, const float* yh, const float* y, const float* w, int B, int64_t npix_per, int C, float* dyh,
          float* loss_per) {
    hipLaunchKernelGGL(loss_kernel, dim3(B), dim3(256), 0, s, yh, y, w, B, npix_per, C, dyh, loss_per);
}
void adam(hipStream_t s, float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
          float eps, int step) {
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(adam_kernel, dim3(grid1(n)), dim3(256), 0, s, p, g, m, v, n, lr, b1, b2, eps, c1, c2);
}

}  // namespace nn
}  // namespace elwh
