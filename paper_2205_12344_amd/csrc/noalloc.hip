// elwh_dot_M_noalloc: the M inner product of elwh_dot_M (Sec. 4.5) for
// callers that cannot allocate device memory.  It needs no context: the node
// weights of M (rho times 1/2 per traction-type face the node lies on, 0 on
// Dirichlet faces) are formed on the fly from the grid, the faces and rho, and
// the fields are read in the caller's layout.  Its two reduction passes keep
// their partial sums and the result in the file-scope array `scratch` below
// (a fixed size, independent of the grid), so the call makes no hipMalloc,
// hipFree or other allocating call.
//
// Each GPU holds its own copy of `scratch`; the host finds that copy's
// address once per device with hipGetSymbolAddress and passes it to the
// kernels.  Every call on one GPU shares the array, so calls that overlap on
// one GPU (two streams, two host threads) race.
#include <cmath>
#include <cstdint>
#include <mutex>
#include <string>

#include "elwh_internal.h"

namespace {

constexpr int kNaBlocks = 512;           // blocks of the first pass = partial sums
constexpr int kNaThreads = 256;
constexpr int kNaSlots = kNaBlocks + 64;  // partials, then the result at kNaBlocks
constexpr int64_t kNaMaxNodes = (int64_t)1 << 31;   // per component
constexpr int kNaMaxDevices = 64;

static __device__ __align__(256) double scratch[kNaSlots];

std::mutex g_na_mu;
double* g_na_ptr[kNaMaxDevices] = {};    // per device: the device address of scratch

struct NaGrid {
    int dim, nx, ny, nz;
    int dir[6];    // 1: that face is Dirichlet (its nodes are not unknowns)
};

// Weight of node (i, j, k) in M / rho: 0 on a Dirichlet face, else 1/2 per
// traction-type face (free or impedance) the node lies on.
__device__ __forceinline__ double node_weight(const NaGrid& g, int i, int j, int k) {
    double w = 1.0;
    const int c[3] = {i, j, k};
    const int m[3] = {g.nx, g.ny, g.nz};
    for (int a = 0; a < g.dim; ++a) {
        if (c[a] == 0) {
            if (g.dir[2 * a]) return 0.0;
            w *= 0.5;
        }
        if (c[a] == m[a]) {
            if (g.dir[2 * a + 1]) return 0.0;
            w *= 0.5;
        }
    }
    return w;
}

// First pass: block b sums w_e rho_e sum_c x_ce y_ce over a grid-stride share
// of the nodes and writes its partial to part[b].
__global__ __launch_bounds__(kNaThreads) void na_dot_partial(NaGrid g, int64_t nodes, const double* __restrict__ rho,
                                                             const double* __restrict__ x,
                                                             const double* __restrict__ y,
                                                             double* __restrict__ part) {
    double s = 0.0;
    const int64_t rowlen = g.nx + 1, plane = rowlen * (g.ny + 1);
    for (int64_t e = (int64_t)blockIdx.x * kNaThreads + threadIdx.x; e < nodes;
         e += (int64_t)gridDim.x * kNaThreads) {
        const int k = (int)(e / plane);
        const int64_t r = e - (int64_t)k * plane;
        const int j = (int)(r / rowlen);
        const int i = (int)(r - (int64_t)j * rowlen);
        const double w = node_weight(g, i, j, k);
        if (w == 0.0) continue;
        double t = 0.0;
        for (int c = 0; c < g.dim; ++c) t += x[c * nodes + e] * y[c * nodes + e];
        s += w * rho[e] * t;
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    __shared__ double red[kNaThreads / 64];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = 0.0;
        for (int q = 0; q < kNaThreads / 64; ++q) b += red[q];
        part[blockIdx.x] = b;
    }
}

// Second pass: the kNaBlocks partials in a fixed order (deterministic result).
__global__ __launch_bounds__(kNaThreads) void na_dot_final(const double* __restrict__ part, double* __restrict__ out) {
    __shared__ double buf[kNaThreads];
    double v = 0.0;
    for (int k = threadIdx.x; k < kNaBlocks; k += kNaThreads) v += part[k];
    buf[threadIdx.x] = v;
    __syncthreads();
    for (int w = kNaThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) buf[threadIdx.x] += buf[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = buf[0];
}

// The device address of scratch on the current device, looked up once per
// device with that device current.
elwh_status scratch_on_current_device(double** out, std::string* err) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kNaMaxDevices) {
        *err = "elwh_dot_M_noalloc: no current HIP device (or device index beyond 63)";
        return ELWH_ERR_HIP;
    }
    std::lock_guard<std::mutex> lock(g_na_mu);
    if (!g_na_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            *err = std::string("elwh_dot_M_noalloc: hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e);
            return ELWH_ERR_HIP;
        }
        g_na_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_na_ptr[dev];
    return ELWH_OK;
}

}  // namespace

extern "C" elwh_status elwh_dot_M_noalloc(const elwh_grid* grid, const double* rho, const int bc[6], const double* x,
                                          const double* y, void* stream, double* out) {
    std::string err;
    auto fail = [&](elwh_status st, const char* msg) {
        elwh::set_create_error(msg);
        return st;
    };
    if (!grid || !rho || !bc || !x || !y || !out) return fail(ELWH_ERR_ARG, "elwh_dot_M_noalloc: null argument");
    if (grid->dim != 2 && grid->dim != 3) return fail(ELWH_ERR_ARG, "elwh_dot_M_noalloc: dim must be 2 or 3");
    NaGrid g{};
    g.dim = grid->dim;
    g.nx = grid->n[0];
    g.ny = grid->n[1];
    g.nz = grid->dim == 3 ? grid->n[2] : 0;
    for (int a = 0; a < grid->dim; ++a)
        if (grid->n[a] < 2) return fail(ELWH_ERR_ARG, "elwh_dot_M_noalloc: every axis needs at least 2 cells");
    for (int f = 0; f < 6; ++f) {
        if (f < 2 * grid->dim && (bc[f] < ELWH_BC_DIRICHLET || bc[f] > ELWH_BC_IMPEDANCE))
            return fail(ELWH_ERR_ARG, "elwh_dot_M_noalloc: unknown face type");
        g.dir[f] = f < 2 * grid->dim && bc[f] == ELWH_BC_DIRICHLET;
    }
    const int64_t nodes = (int64_t)(g.nx + 1) * (g.ny + 1) * (g.dim == 3 ? (g.nz + 1) : 1);
    if (nodes > kNaMaxNodes)
        return fail(ELWH_ERR_ARG, "elwh_dot_M_noalloc: more than 2^31 nodes per component");
    double* sp = nullptr;
    const elwh_status st = scratch_on_current_device(&sp, &err);
    if (st != ELWH_OK) {
        elwh::set_create_error(err);
        return st;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(na_dot_partial, dim3(kNaBlocks), dim3(kNaThreads), 0, s, g, nodes, rho, x, y, sp);
    hipLaunchKernelGGL(na_dot_final, dim3(1), dim3(kNaThreads), 0, s, sp, sp + kNaBlocks);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(out, sp + kNaBlocks, sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        elwh::set_create_error(std::string("elwh_dot_M_noalloc: ") + hipGetErrorString(e));
        return ELWH_ERR_HIP;
    }
    return ELWH_OK;
}
