// Learned warm start for the Krylov solve (C ABI elwh_ws_* in include/elwh.h).
//
// A convolutional encoder-decoder (U-Net, five resolution levels, 3x3
// convolutions with bias and SiLU, 2x2 average pooling, nearest upsampling,
// skip concatenation; 1 644 578 parameters) maps the problem data on the node
// grid -- log rho, log mu, log(lambda/mu), the forcing normalised by its
// maximum, omega h and omega -- to the displacement, and its output seeds the
// solve (x0).  Convolutions are GEMMs on MFMA over a BF16 im2col matrix
// with FP32 accumulation; master weights, activations, gradients and Adam
// state are FP32.  Training minimises the relative error in the M-weighted
// norm against solutions computed by the solver itself.
#include <cmath>
#include <cstring>
#include <new>
#include <random>
#include <string>
#include <vector>

#include "elwh_internal.h"
#include "nn_internal.h"

using namespace elwh;

namespace {

struct Conv {
    int cin, cout, act;
    int64_t woff, boff;   // offsets of W [9 cin][cout] and bias [cout] in the flat parameter vector
};

// Layer table, in parameter order.
const int kLayers[][3] = {
    {7, 32, 1},    {32, 32, 1},   // e0
    {32, 64, 1},   {64, 64, 1},   // e1
    {64, 96, 1},   {96, 96, 1},   // e2
    {96, 128, 1},  {128, 128, 1}, // e3
    {128, 128, 1}, {128, 128, 1}, // e4 (bottleneck)
    {256, 128, 1}, {128, 128, 1}, // d3
    {224, 96, 1},  {96, 96, 1},   // d2
    {160, 64, 1},  {64, 64, 1},   // d1
    {96, 32, 1},   {32, 32, 1},   // d0
    {32, 2, 0},                   // head
};
constexpr int NL = sizeof(kLayers) / sizeof(kLayers[0]);
constexpr int NOUT = 2, NLEV = 5;
const int kWidth[NLEV] = {32, 64, 96, 128, 128};

}  // namespace

struct elwh_ws {
    int maxB = 0, H = 0, W = 0;
    hipStream_t stream = nullptr;
    std::string err;
    std::vector<Conv> L;
    int64_t nparam = 0;
    float *P = nullptr, *G = nullptr, *Mo = nullptr, *Vo = nullptr;   // params, grads, Adam moments
    unsigned short* Pb = nullptr;                                       // BF16 copy of the params
    int step = 0;
    double out_scale = 1.0;
    // activations
    std::vector<float*> Z, A;          // per conv layer: pre-activation, activation
    std::vector<float*> dA;            // per conv layer: gradient w.r.t. activation
    float* pool[NLEV - 1] = {};        // pooled tensors (input of level l+1)
    float* cat[NLEV - 1] = {};         // concat inputs of the decoder levels 0..3
    float* dpool[NLEV - 1] = {};
    float* dcat[NLEV - 1] = {};
    float* dout = nullptr;
    unsigned short* col = nullptr;     // im2col scratch (BF16)
    float* dcol = nullptr;             // col2im scratch (FP32)
    unsigned short* gbf = nullptr;     // BF16 copy of a layer's output gradient
    float* part = nullptr;             // split-K / channel-sum partials
    int64_t part_elems = 0;
    float* lossb = nullptr;            // per-sample loss
    float* hloss = nullptr;            // pinned
    // feature scratch
    double* fmax = nullptr;
    const double** dptr = nullptr;     // device pointer tables
};

namespace {

thread_local std::string g_ws_err;

#define WCK(expr)                                                               \
    do {                                                                        \
        hipError_t e_ = (expr);                                                 \
        if (e_ != hipSuccess) {                                                 \
            ws->err = std::string(#expr) + ": " + hipGetErrorString(e_);        \
            return ELWH_ERR_HIP;                                                \
        }                                                                       \
    } while (0)

// input of conv layer l given the network's buffers
struct LayerIO {
    const float* X;
    int H, W;
};

int level_of(int l) {
    // e0..e4: layers 0..9 -> level l/2; d3..d0: layers 10..17 -> 3 - (l-10)/2; head: 0
    if (l < 10) return l / 2;
    if (l < 18) return 3 - (l - 10) / 2;
    return 0;
}

LayerIO layer_input(const elwh_ws* ws, int l, const float* x) {
    const int lev = level_of(l);
    LayerIO io;
    io.H = ws->H >> lev;
    io.W = ws->W >> lev;
    if (l == 0) io.X = x;
    else if (l < 10 && (l % 2 == 0)) io.X = ws->pool[lev - 1];   // first conv of encoder level lev > 0
    else if (l >= 10 && l < 18 && ((l - 10) % 2 == 0)) io.X = ws->cat[lev];
    else io.X = ws->A[l - 1];
    return io;
}

void conv_forward(elwh_ws* ws, int l, int B, const float* x) {
    const Conv& c = ws->L[l];
    const LayerIO io = layer_input(ws, l, x);
    const int64_t M = (int64_t)B * io.H * io.W;
    nn::im2col(ws->stream, io.X, ws->col, B, io.H, io.W, c.cin);
    nn::gemm(ws->stream, false, false, (int)M, c.cout, 9 * c.cin, ws->col, 9 * c.cin, ws->Pb + c.woff, c.cout, ws->Z[l],
             c.cout, 1, ws->part, 0);
    nn::bias_act(ws->stream, ws->Z[l], ws->A[l], ws->P + c.boff, M, c.cout, c.act);
}

// dA[l] holds dL/dA on entry; accumulates dW, db; writes dX (if dX != null).
void conv_backward(elwh_ws* ws, int l, int B, const float* x, float* dX) {
    const Conv& c = ws->L[l];
    const LayerIO io = layer_input(ws, l, x);
    const int64_t M = (int64_t)B * io.H * io.W;
    const int K = 9 * c.cin;
    float* dZ = ws->dA[l];
    nn::act_back(ws->stream, dZ, ws->Z[l], M * c.cout, c.act);
    nn::channel_sum(ws->stream, dZ, M, c.cout, ws->part, 256, ws->G + c.boff, 0);
    nn::to_bf16(ws->stream, dZ, ws->gbf, M * c.cout);
    nn::im2col(ws->stream, io.X, ws->col, B, io.H, io.W, c.cin);
    // dW[K][cout] = col^T dZ  (reduction over the M pixels, split for parallelism)
    int splits = (int)std::min<int64_t>(256, std::max<int64_t>(1, M / 1024));
    const int64_t need = (int64_t)splits * K * c.cout;
    if (need > ws->part_elems) splits = (int)std::max<int64_t>(1, ws->part_elems / ((int64_t)K * c.cout));
    nn::gemm(ws->stream, true, false, K, c.cout, (int)M, ws->col, K, ws->gbf, c.cout, ws->G + c.woff, c.cout, splits,
             ws->part, 0);
    if (dX) {
        // dcol[M][K] = dZ W^T, then the gather back to pixels
        nn::gemm(ws->stream, false, true, (int)M, K, c.cout, ws->gbf, c.cout, ws->Pb + c.woff, c.cout, ws->dcol, K, 1,
                 ws->part, 0);
        nn::col2im(ws->stream, ws->dcol, dX, B, io.H, io.W, c.cin);
    }
}

void forward(elwh_ws* ws, int B, const float* x) {
    const int H = ws->H, W = ws->W;
    for (int lev = 0; lev < NLEV; ++lev) {
        conv_forward(ws, 2 * lev, B, x);
        conv_forward(ws, 2 * lev + 1, B, x);
        if (lev < NLEV - 1)
            nn::avgpool(ws->stream, ws->A[2 * lev + 1], ws->pool[lev], B, H >> lev, W >> lev, kWidth[lev]);
    }
    // decoder: level 3 down to 0
    for (int lev = NLEV - 2; lev >= 0; --lev) {
        const int deeper = lev == NLEV - 2 ? 9 : 10 + 2 * (NLEV - 3 - lev) + 1;   // last conv of the level below
        const int cup = ws->L[deeper].cout;
        const int cskip = kWidth[lev];
        const int Hl = H >> lev, Wl = W >> lev;
        nn::upsample(ws->stream, ws->A[deeper], ws->cat[lev], B, Hl / 2, Wl / 2, cup, cup + cskip, 0);
        nn::copy_channels(ws->stream, ws->A[2 * lev + 1], cskip, 0, ws->cat[lev], cup + cskip, cup,
                          (int64_t)B * Hl * Wl, cskip, 0);
        const int la = 10 + 2 * (NLEV - 2 - lev);
        conv_forward(ws, la, B, x);
        conv_forward(ws, la + 1, B, x);
    }
    conv_forward(ws, NL - 1, B, x);
}

void backward(elwh_ws* ws, int B, const float* x) {
    const int H = ws->H, W = ws->W;
    // head: dA[head] = dout
    (void)hipMemcpyAsync(ws->dA[NL - 1], ws->dout, sizeof(float) * (size_t)B * H * W * NOUT, hipMemcpyDeviceToDevice,
                         ws->stream);
    conv_backward(ws, NL - 1, B, x, ws->dA[NL - 2]);
    for (int lev = 0; lev <= NLEV - 2; ++lev) {
        const int la = 10 + 2 * (NLEV - 2 - lev);
        const int deeper = lev == NLEV - 2 ? 9 : la - 1;
        const int cup = ws->L[deeper].cout;
        const int cskip = kWidth[lev];
        const int Hl = H >> lev, Wl = W >> lev;
        conv_backward(ws, la + 1, B, x, ws->dA[la]);
        conv_backward(ws, la, B, x, ws->dcat[lev]);
        nn::upsample_back(ws->stream, ws->dcat[lev], ws->dA[deeper], B, Hl / 2, Wl / 2, cup, cup + cskip, 0);
        nn::copy_channels(ws->stream, ws->dcat[lev], cup + cskip, cup, ws->dA[2 * lev + 1], cskip, 0,
                          (int64_t)B * Hl * Wl, cskip, 0);
    }
    // encoder, deepest first; each level's input gradient flows back through the pooling
    for (int lev = NLEV - 1; lev >= 0; --lev) {
        conv_backward(ws, 2 * lev + 1, B, x, ws->dA[2 * lev]);
        if (lev == 0) {
            conv_backward(ws, 0, B, x, nullptr);
        } else {
            conv_backward(ws, 2 * lev, B, x, ws->dpool[lev - 1]);
            nn::avgpool_back(ws->stream, ws->dpool[lev - 1], ws->dA[2 * lev - 1], B, H >> (lev - 1), W >> (lev - 1),
                             kWidth[lev - 1], 1);
        }
    }
}

elwh_status alloc(elwh_ws* ws, void** p, size_t bytes) {
    if (hipMalloc(p, bytes) != hipSuccess) {
        *p = nullptr;
        ws->err = "device allocation failed (" + std::to_string(bytes) + " bytes)";
        return ELWH_ERR_ALLOC;
    }
    (void)hipMemsetAsync(*p, 0, bytes, ws->stream);
    return ELWH_OK;
}

void free_ws(elwh_ws* ws) {
    auto f = [](void* p) {
        if (p) (void)hipFree(p);
    };
    f(ws->P); f(ws->G); f(ws->Mo); f(ws->Vo); f(ws->Pb);
    for (auto* p : ws->Z) f(p);
    for (auto* p : ws->A) f(p);
    for (auto* p : ws->dA) f(p);
    for (int k = 0; k < NLEV - 1; ++k) { f(ws->pool[k]); f(ws->cat[k]); f(ws->dpool[k]); f(ws->dcat[k]); }
    f(ws->dout); f(ws->col); f(ws->dcol); f(ws->gbf); f(ws->part); f(ws->lossb); f(ws->fmax); f(ws->dptr);
    if (ws->hloss) (void)hipHostFree(ws->hloss);
}

// ---- problem data <-> network tensors ----------------------------------------
// Network pixel (py, px) <-> node (i = px, j = py + 1) of an n x n-cell grid
// (H = W = n), i.e. the unknown rows 1..n of a Dirichlet-bottom / free-top
// square plus the Dirichlet column i = 0.

__global__ void fmax_kernel(const double* const* __restrict__ f, int nn, double* __restrict__ out) {
    const double* fb = f[blockIdx.x];
    double m = 0.0;
    for (int e = threadIdx.x; e < 2 * nn; e += blockDim.x) m = fmax(m, fabs(fb[e]));
    __shared__ double red[256];
    red[threadIdx.x] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0] > 0 ? red[0] : 1.0;
}

// Per-sample target normalisation: y[b] /= sqrt(sum w y^2 / (2 sum w)), the
// w-weighted RMS over both components (one block per sample, FP64 sums;
// samples with no weight or a zero target are left as they are).
__global__ void normalize_kernel(float* __restrict__ y, const float* __restrict__ w, int npix) {
    float* yb = y + (int64_t)blockIdx.x * npix * 2;
    const float* wb = w + (int64_t)blockIdx.x * npix;
    double sy = 0.0, sw = 0.0;
    for (int p = threadIdx.x; p < npix; p += blockDim.x) {
        const double wp = wb[p], a = yb[2 * p], c = yb[2 * p + 1];
        sy += wp * (a * a + c * c);
        sw += wp;
    }
    __shared__ double r1[256], r2[256];
    __shared__ float scale;
    r1[threadIdx.x] = sy;
    r2[threadIdx.x] = sw;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            r1[threadIdx.x] += r1[threadIdx.x + st];
            r2[threadIdx.x] += r2[threadIdx.x + st];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double rms = r2[0] > 0 ? sqrt(r1[0] / (2.0 * r2[0])) : 0.0;
        scale = rms > 0 ? (float)(1.0 / rms) : 1.0f;
    }
    __syncthreads();
    for (int p = threadIdx.x; p < 2 * npix; p += blockDim.x) yb[p] *= scale;
}

// x[b,py,px,:] = (log rho/0.2, log mu/0.2, log(lam/mu)/0.5, fx/fmax, fy/fmax, 5 omega h, omega/60)
// w[b,py,px] = M weight of the node (trapezoid weight * rho), 0 on Dirichlet nodes
__global__ void features_kernel(const double* const* __restrict__ rho, const double* const* __restrict__ lam,
                                const double* const* __restrict__ mu, const double* const* __restrict__ f,
                                const double* __restrict__ omega, const double* __restrict__ fmx, int n,
                                float* __restrict__ x, float* __restrict__ w, int B) {
    const int64_t npix = (int64_t)n * n;
    const int64_t total = npix * B;
    const int nn1 = n + 1;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int b = (int)(e / npix);
        const int64_t pix = e - (int64_t)b * npix;
        const int py = (int)(pix / n), px = (int)(pix - (int64_t)py * n);
        const int i = px, j = py + 1;
        const int64_t node = (int64_t)j * nn1 + i;
        const double r = rho[b][node], l = lam[b][node], m = mu[b][node];
        const double s = 1.0 / fmx[b];
        float* xo = x + e * 7;
        xo[0] = (float)(log(r) / 0.2);
        xo[1] = (float)(log(m) / 0.2);
        xo[2] = (float)(log(l / m) / 0.5);
        xo[3] = (float)(f[b][node] * s);
        xo[4] = (float)(f[b][node + (int64_t)nn1 * nn1] * s);
        xo[5] = (float)(5.0 * omega[b] / n);
        xo[6] = (float)(omega[b] / 60.0);
        const bool unknown = i >= 1 && i <= n - 1;
        const double wt = (j == n) ? 0.5 : 1.0;   // free top row carries trapezoid weight 1/2
        w[e] = unknown ? (float)(wt * r) : 0.f;
    }
}

// y[b,py,px,c] = v_c(i,j) * omega^2 / (fmax * k)   (targets from solutions)
__global__ void from_field_kernel(const double* const* __restrict__ v, const double* __restrict__ omega,
                                  const double* __restrict__ fmx, double k, int n, float* __restrict__ y, int B) {
    const int64_t npix = (int64_t)n * n;
    const int nn1 = n + 1;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < npix * B; e += (int64_t)gridDim.x * blockDim.x) {
        const int b = (int)(e / npix);
        const int64_t pix = e - (int64_t)b * npix;
        const int py = (int)(pix / n), px = (int)(pix - (int64_t)py * n);
        const int64_t node = (int64_t)(py + 1) * nn1 + px;
        const double s = omega[b] * omega[b] / (fmx[b] * k);
        y[e * 2] = (float)(v[b][node] * s);
        y[e * 2 + 1] = (float)(v[b][node + (int64_t)nn1 * nn1] * s);
    }
}

// x0_c(i,j) = y[b,py,px,c] * fmax * k / omega^2 on unknown nodes, 0 elsewhere
__global__ void to_field_kernel(const float* __restrict__ y, const double* __restrict__ omega,
                                const double* __restrict__ fmx, double k, int n, double* const* __restrict__ x0, int B) {
    const int nn1 = n + 1;
    const int64_t nodes = (int64_t)nn1 * nn1;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nodes * B; e += (int64_t)gridDim.x * blockDim.x) {
        const int b = (int)(e / nodes);
        const int64_t node = e - (int64_t)b * nodes;
        const int j = (int)(node / nn1), i = (int)(node - (int64_t)j * nn1);
        double u = 0.0, v = 0.0;
        if (i >= 1 && i <= n - 1 && j >= 1) {
            const int64_t pix = ((int64_t)b * n + (j - 1)) * n + i;
            const double s = fmx[b] * k / (omega[b] * omega[b]);
            u = y[pix * 2] * s;
            v = y[pix * 2 + 1] * s;
        }
        x0[b][node] = u;
        x0[b][node + nodes] = v;
    }
}

unsigned g1(int64_t n) {
    const int64_t g = (n + 255) / 256;
    return (unsigned)(g < 1 ? 1 : (g > 65536 ? 65536 : g));
}

elwh_status upload_ptrs(elwh_ws* ws, int B, const double* const* a, int slot) {
    WCK(hipMemcpyAsync(ws->dptr + (size_t)slot * ws->maxB, a, sizeof(double*) * B, hipMemcpyHostToDevice, ws->stream));
    return ELWH_OK;
}

}  // namespace

extern "C" {

elwh_status elwh_ws_create(int max_batch, int H, int W, unsigned long long seed, void* stream, elwh_ws** out) {
    if (!out) return ELWH_ERR_ARG;
    *out = nullptr;
    if (max_batch < 1 || H < 16 || W < 16 || H % 16 || W % 16 || (int64_t)H * W * max_batch > (1LL << 26)) {
        g_ws_err = "network: H, W must be multiples of 16 (>= 16); batch x H x W <= 2^26";
        return ELWH_ERR_ARG;
    }
    elwh_ws* ws = new (std::nothrow) elwh_ws();
    if (!ws) return ELWH_ERR_ALLOC;
    ws->maxB = max_batch;
    ws->H = H;
    ws->W = W;
    ws->stream = reinterpret_cast<hipStream_t>(stream);
    auto fail = [&](elwh_status s) {
        g_ws_err = ws->err;
        free_ws(ws);
        delete ws;
        return s;
    };
    int64_t off = 0;
    for (int l = 0; l < NL; ++l) {
        Conv c{kLayers[l][0], kLayers[l][1], kLayers[l][2], 0, 0};
        c.woff = off;
        off += 9LL * c.cin * c.cout;
        c.boff = off;
        off += c.cout;
        ws->L.push_back(c);
    }
    ws->nparam = off;
    elwh_status st;
    const size_t np = (size_t)off;
    if ((st = alloc(ws, (void**)&ws->P, np * 4)) || (st = alloc(ws, (void**)&ws->G, np * 4)) ||
        (st = alloc(ws, (void**)&ws->Mo, np * 4)) || (st = alloc(ws, (void**)&ws->Vo, np * 4)) ||
        (st = alloc(ws, (void**)&ws->Pb, np * 2)))
        return fail(st);
    const int64_t B = max_batch;
    int64_t max_col = 0, max_act = 0;
    ws->Z.resize(NL);
    ws->A.resize(NL);
    ws->dA.resize(NL);
    for (int l = 0; l < NL; ++l) {
        const int lev = level_of(l);
        const int64_t npix = B * (H >> lev) * (W >> lev);
        const size_t bytes = (size_t)npix * ws->L[l].cout * 4;
        if ((st = alloc(ws, (void**)&ws->Z[l], bytes)) || (st = alloc(ws, (void**)&ws->A[l], bytes)) ||
            (st = alloc(ws, (void**)&ws->dA[l], bytes)))
            return fail(st);
        max_col = std::max(max_col, npix * 9 * ws->L[l].cin);
        max_act = std::max(max_act, npix * ws->L[l].cout);
    }
    for (int lev = 0; lev < NLEV - 1; ++lev) {
        const int64_t npix1 = B * (H >> (lev + 1)) * (W >> (lev + 1));
        const int64_t npix = B * (H >> lev) * (W >> lev);
        const int ccat = kWidth[lev] + (lev == NLEV - 2 ? kWidth[NLEV - 1] : kWidth[lev + 1]);
        if ((st = alloc(ws, (void**)&ws->pool[lev], (size_t)npix1 * kWidth[lev] * 4)) ||
            (st = alloc(ws, (void**)&ws->dpool[lev], (size_t)npix1 * kWidth[lev] * 4)) ||
            (st = alloc(ws, (void**)&ws->cat[lev], (size_t)npix * ccat * 4)) ||
            (st = alloc(ws, (void**)&ws->dcat[lev], (size_t)npix * ccat * 4)))
            return fail(st);
    }
    ws->part_elems = std::max<int64_t>(std::max<int64_t>(max_act, 256LL * 256), 256LL * 9 * 256 * 128);
    if ((st = alloc(ws, (void**)&ws->dout, (size_t)B * H * W * NOUT * 4)) ||
        (st = alloc(ws, (void**)&ws->col, (size_t)max_col * 2)) ||
        (st = alloc(ws, (void**)&ws->dcol, (size_t)max_col * 4)) ||
        (st = alloc(ws, (void**)&ws->gbf, (size_t)max_act * 2)) ||
        (st = alloc(ws, (void**)&ws->part, (size_t)ws->part_elems * 4)) ||
        (st = alloc(ws, (void**)&ws->lossb, (size_t)B * 4)) || (st = alloc(ws, (void**)&ws->fmax, (size_t)B * 8)) ||
        (st = alloc(ws, (void**)&ws->dptr, (size_t)B * 8 * sizeof(double*))))
        return fail(st);
    if (hipHostMalloc((void**)&ws->hloss, (size_t)B * 4, hipHostMallocDefault) != hipSuccess) return fail(ELWH_ERR_ALLOC);
    // He-style initialisation (seeded), zero biases; the head starts small
    std::vector<float> hp(np, 0.f);
    std::mt19937_64 rng(seed);
    for (int l = 0; l < NL; ++l) {
        const Conv& c = ws->L[l];
        const double sd = std::sqrt(2.0 / (9.0 * c.cin)) * (l == NL - 1 ? 0.1 : 1.0);
        std::normal_distribution<double> nd(0.0, sd);
        for (int64_t k = 0; k < 9LL * c.cin * c.cout; ++k) hp[c.woff + k] = (float)nd(rng);
    }
    if (hipMemcpyAsync(ws->P, hp.data(), np * 4, hipMemcpyHostToDevice, ws->stream) != hipSuccess)
        return fail(ELWH_ERR_HIP);
    nn::to_bf16(ws->stream, ws->P, ws->Pb, ws->nparam);
    if (hipStreamSynchronize(ws->stream) != hipSuccess) return fail(ELWH_ERR_HIP);
    *out = ws;
    return ELWH_OK;
}

void elwh_ws_destroy(elwh_ws* ws) {
    if (!ws) return;
    (void)hipStreamSynchronize(ws->stream);
    free_ws(ws);
    delete ws;
}

const char* elwh_ws_last_error(const elwh_ws* ws) { return ws ? ws->err.c_str() : g_ws_err.c_str(); }

long long elwh_ws_num_params(const elwh_ws* ws) { return ws ? ws->nparam : -1; }

elwh_status elwh_ws_params(elwh_ws* ws, float* get, const float* set, double* out_scale_get, const double* out_scale_set) {
    if (!ws) return ELWH_ERR_ARG;
    if (set) {
        WCK(hipMemcpyAsync(ws->P, set, ws->nparam * 4, hipMemcpyHostToDevice, ws->stream));
        nn::to_bf16(ws->stream, ws->P, ws->Pb, ws->nparam);
        WCK(hipMemsetAsync(ws->Mo, 0, ws->nparam * 4, ws->stream));
        WCK(hipMemsetAsync(ws->Vo, 0, ws->nparam * 4, ws->stream));
        ws->step = 0;
    }
    if (out_scale_set) ws->out_scale = *out_scale_set;
    if (out_scale_get) *out_scale_get = ws->out_scale;
    if (get) WCK(hipMemcpyAsync(get, ws->P, ws->nparam * 4, hipMemcpyDeviceToHost, ws->stream));
    WCK(hipStreamSynchronize(ws->stream));
    return ELWH_OK;
}

elwh_status elwh_ws_forward(elwh_ws* ws, int B, const float* x, float* y) {
    if (!ws || !x || !y || B < 1 || B > ws->maxB) return ELWH_ERR_ARG;
    forward(ws, B, x);
    WCK(hipMemcpyAsync(y, ws->A[NL - 1], sizeof(float) * (size_t)B * ws->H * ws->W * NOUT, hipMemcpyDeviceToDevice,
                       ws->stream));
    WCK(hipGetLastError());
    return ELWH_OK;
}

elwh_status elwh_ws_loss_grad(elwh_ws* ws, int B, const float* x, const float* y, const float* w, float* loss,
                              float* grad_host) {
    if (!ws || !x || !y || !w || B < 1 || B > ws->maxB) return ELWH_ERR_ARG;
    forward(ws, B, x);
    nn::loss(ws->stream, ws->A[NL - 1], y, w, B, (int64_t)ws->H * ws->W, NOUT, ws->dout, ws->lossb);
    backward(ws, B, x);
    WCK(hipMemcpyAsync(ws->hloss, ws->lossb, sizeof(float) * B, hipMemcpyDeviceToHost, ws->stream));
    if (grad_host) WCK(hipMemcpyAsync(grad_host, ws->G, ws->nparam * 4, hipMemcpyDeviceToHost, ws->stream));
    WCK(hipStreamSynchronize(ws->stream));
    if (loss) {
        double s = 0;
        for (int b = 0; b < B; ++b) s += ws->hloss[b];
        *loss = (float)s;
    }
    return ELWH_OK;
}

elwh_status elwh_ws_train_step(elwh_ws* ws, int B, const float* x, const float* y, const float* w, float lr,
                               float* loss) {
    if (!ws || !x || !y || !w || B < 1 || B > ws->maxB || !(lr > 0)) return ELWH_ERR_ARG;
    forward(ws, B, x);
    nn::loss(ws->stream, ws->A[NL - 1], y, w, B, (int64_t)ws->H * ws->W, NOUT, ws->dout, ws->lossb);
    backward(ws, B, x);
    ws->step++;
    nn::adam(ws->stream, ws->P, ws->G, ws->Mo, ws->Vo, ws->nparam, lr, 0.9f, 0.999f, 1e-8f, ws->step);
    nn::to_bf16(ws->stream, ws->P, ws->Pb, ws->nparam);
    if (loss) {
        WCK(hipMemcpyAsync(ws->hloss, ws->lossb, sizeof(float) * B, hipMemcpyDeviceToHost, ws->stream));
        WCK(hipStreamSynchronize(ws->stream));
        double s = 0;
        for (int b = 0; b < B; ++b) s += ws->hloss[b];
        *loss = (float)s;
    }
    WCK(hipGetLastError());
    return ELWH_OK;
}

elwh_status elwh_ws_features(elwh_ws* ws, int B, int n, const double* const* rho, const double* const* lam,
                             const double* const* mu, const double* const* f, const double* omega_dev, float* x,
                             float* w) {
    if (!ws || B < 1 || B > ws->maxB || n != ws->H || n != ws->W || !rho || !lam || !mu || !f || !omega_dev || !x ||
        !w)
        return ELWH_ERR_ARG;
    elwh_status st;
    if ((st = upload_ptrs(ws, B, rho, 0)) || (st = upload_ptrs(ws, B, lam, 1)) || (st = upload_ptrs(ws, B, mu, 2)) ||
        (st = upload_ptrs(ws, B, f, 3)))
        return st;
    const double** d = ws->dptr;
    const int M = ws->maxB;
    hipLaunchKernelGGL(fmax_kernel, dim3(B), dim3(256), 0, ws->stream, d + 3 * M, (n + 1) * (n + 1), ws->fmax);
    hipLaunchKernelGGL(features_kernel, dim3(g1((int64_t)B * n * n)), dim3(256), 0, ws->stream, d, d + M, d + 2 * M,
                       d + 3 * M, omega_dev, ws->fmax, n, x, w, B);
    WCK(hipStreamSynchronize(ws->stream));   // the pointer tables are reused by the next call
    WCK(hipGetLastError());
    return ELWH_OK;
}

elwh_status elwh_ws_from_field(elwh_ws* ws, int B, int n, const double* const* f, const double* const* v,
                               const double* omega_dev, float* y) {
    if (!ws || B < 1 || B > ws->maxB || n != ws->H || !f || !v || !omega_dev || !y) return ELWH_ERR_ARG;
    elwh_status st;
    if ((st = upload_ptrs(ws, B, f, 3)) || (st = upload_ptrs(ws, B, v, 4))) return st;
    const double** d = ws->dptr;
    const int M = ws->maxB;
    hipLaunchKernelGGL(fmax_kernel, dim3(B), dim3(256), 0, ws->stream, d + 3 * M, (n + 1) * (n + 1), ws->fmax);
    hipLaunchKernelGGL(from_field_kernel, dim3(g1((int64_t)B * n * n)), dim3(256), 0, ws->stream, d + 4 * M,
                       omega_dev, ws->fmax, ws->out_scale, n, y, B);
    WCK(hipStreamSynchronize(ws->stream));
    WCK(hipGetLastError());
    return ELWH_OK;
}

elwh_status elwh_ws_normalize(elwh_ws* ws, int B, float* y, const float* w) {
    if (!ws || B < 1 || B > ws->maxB || !y || !w) return ELWH_ERR_ARG;
    hipLaunchKernelGGL(normalize_kernel, dim3(B), dim3(256), 0, ws->stream, y, w, ws->H * ws->W);
    WCK(hipGetLastError());
    return ELWH_OK;
}

elwh_status elwh_ws_predict(elwh_ws* ws, int B, int n, const float* x, const double* const* f, const double* omega_dev,
                            double* const* x0) {
    if (!ws || B < 1 || B > ws->maxB || n != ws->H || !x || !f || !omega_dev || !x0) return ELWH_ERR_ARG;
    forward(ws, B, x);
    elwh_status st;
    if ((st = upload_ptrs(ws, B, f, 3)) ||
        (st = upload_ptrs(ws, B, reinterpret_cast<const double* const*>(x0), 5)))
        return st;
    const double** d = ws->dptr;
    const int M = ws->maxB;
    hipLaunchKernelGGL(fmax_kernel, dim3(B), dim3(256), 0, ws->stream, d + 3 * M, (n + 1) * (n + 1), ws->fmax);
    hipLaunchKernelGGL(to_field_kernel, dim3(g1((int64_t)B * (n + 1) * (n + 1))), dim3(256), 0, ws->stream,
                       ws->A[NL - 1], omega_dev, ws->fmax, ws->out_scale, n,
                       reinterpret_cast<double* const*>(const_cast<double**>(d + 5 * M)), B);
    WCK(hipStreamSynchronize(ws->stream));
    WCK(hipGetLastError());
    return ELWH_OK;
}

}  // extern "C"
