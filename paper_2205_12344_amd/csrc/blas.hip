// Layout conversion, FP64 Krylov reductions and vector updates for libelwh.
//
// Inner products are (x, y)_M = sum_i m_i x_i y_i over the unknown dofs,
// m = trapezoid weight * rho (the M of Sec. 4.1 / 4.5).  They are reduced
// deterministically in two passes: every block of a fixed-size grid sums a
// grid-strided slice (wavefront shuffles, then LDS across the block's
// wavefronts) into one partial; a single block then adds the partials in a
// fixed tree order.  Reruns on the same data are bit-identical.
#include "elwh_internal.h"

namespace elwh {

namespace {

constexpr int RB = 256;  // threads per reduction block

struct PackArgs {
    int dim, nx, ny, nz;
    int64_t P, PS, CS;
    int mask;            // zero Dirichlet nodes
    int bc[6];
};

__device__ __forceinline__ bool node_unknown(const PackArgs& a, int x, int y, int z) {
    if (x == 0 && a.bc[0] == ELWH_BC_DIRICHLET) return false;
    if (x == a.nx && a.bc[1] == ELWH_BC_DIRICHLET) return false;
    if (y == 0 && a.bc[2] == ELWH_BC_DIRICHLET) return false;
    if (y == a.ny && a.bc[3] == ELWH_BC_DIRICHLET) return false;
    if (a.dim == 3) {
        if (z == 0 && a.bc[4] == ELWH_BC_DIRICHLET) return false;
        if (z == a.nz && a.bc[5] == ELWH_BC_DIRICHLET) return false;
    }
    return true;
}

template <typename D>
__global__ void pack_kernel(const double* __restrict__ src, D* __restrict__ dst, int ncomp, PackArgs a) {
    const int64_t total = a.CS * ncomp;
    const int64_t nxn = a.nx + 1, nyn = a.ny + 1;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = e / a.CS;
        const int64_t r = e - c * a.CS;
        const int z = (int)(r / a.PS);
        const int64_t r2 = r - (int64_t)z * a.PS;
        const int y = (int)(r2 / a.P);
        const int x = (int)(r2 - (int64_t)y * a.P);
        double v = 0.0;
        if (x <= a.nx && (!a.mask || node_unknown(a, x, y, z)))
            v = src[((c * (a.dim == 3 ? a.nz + 1 : 1) + z) * nyn + y) * nxn + x];
        dst[e] = (D)v;
    }
}

__global__ void unpack_kernel(const double* __restrict__ src, double* __restrict__ dst, int ncomp, PackArgs a) {
    const int64_t nxn = a.nx + 1, nyn = a.ny + 1, nzn = a.dim == 3 ? a.nz + 1 : 1;
    const int64_t total = nxn * nyn * nzn * ncomp;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        int64_t r = e;
        const int x = (int)(r % nxn);
        r /= nxn;
        const int y = (int)(r % nyn);
        r /= nyn;
        const int z = (int)(r % nzn);
        const int64_t c = r / nzn;
        double v = 0.0;
        if (node_unknown(a, x, y, z)) v = src[c * a.CS + (int64_t)z * a.PS + (int64_t)y * a.P + x];
        dst[e] = v;
    }
}

__global__ void convert_kernel(const double* __restrict__ src, float* __restrict__ dst, int64_t n) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        dst[e] = (float)src[e];
}

// dst[e] *= w[e mod cs] over ncomp components of cs elements each.
__global__ void scale_field_kernel(double* __restrict__ dst, const double* __restrict__ w, int64_t cs, int64_t n) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        dst[e] *= w[e % cs];
}

PackArgs pack_args(const Layout& L, const int bc[6], int mask) {
    PackArgs a;
    a.dim = L.dim;
    a.nx = L.nx;
    a.ny = L.ny;
    a.nz = L.nz;
    a.P = L.P;
    a.PS = L.PS;
    a.CS = L.CS;
    a.mask = mask;
    for (int f = 0; f < 6; ++f) a.bc[f] = f < 2 * L.dim ? bc[f] : ELWH_BC_DIRICHLET;
    return a;
}

unsigned grid_for(int64_t n, int bs = 256) {
    int64_t g = (n + bs - 1) / bs;
    return (unsigned)std::min<int64_t>(std::max<int64_t>(g, 1), 65536);
}

// ---- reductions -------------------------------------------------------------

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

__device__ __forceinline__ double block_sum(double v) {
    __shared__ double red[RB / 64];
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < RB / 64; ++k) s += red[k];
    }
    return s;  // valid in thread 0
}

__global__ __launch_bounds__(RB) void dotm_partial_kernel(const double* __restrict__ x, const double* __restrict__ y,
                                                          const double* __restrict__ m, int ncomp, int64_t CS,
                                                          double* __restrict__ partials) {
    double s = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * RB + threadIdx.x; e < CS; e += (int64_t)gridDim.x * RB) {
        const double me = m[e];
        double t = 0.0;
        for (int c = 0; c < ncomp; ++c) t += x[e + c * CS] * y[e + c * CS];
        s += me * t;
    }
    s = block_sum(s);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// (p, q)_M into partials[0, gridDim) and (p, p)_M into partials[gridDim, 2 gridDim).
__global__ __launch_bounds__(RB) void dot_pq_pp_partial_kernel(const double* __restrict__ p,
                                                               const double* __restrict__ q,
                                                               const double* __restrict__ m, int ncomp, int64_t CS,
                                                               double* __restrict__ partials) {
    double s = 0.0, s2 = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * RB + threadIdx.x; e < CS; e += (int64_t)gridDim.x * RB) {
        const double me = m[e];
        double t = 0.0, t2 = 0.0;
        for (int c = 0; c < ncomp; ++c) {
            const double pv = p[e + c * CS];
            t += pv * q[e + c * CS];
            t2 += pv * pv;
        }
        s += me * t;
        s2 += me * t2;
    }
    s = block_sum(s);
    s2 = block_sum(s2);
    if (threadIdx.x == 0) {
        partials[blockIdx.x] = s;
        partials[gridDim.x + blockIdx.x] = s2;
    }
}

// RED_PQ reduces two partial arrays: (p, q)_M from partials[0, n) and
// (p, p)_M from partials[n, 2n).
__global__ __launch_bounds__(1024) void reduce_final_kernel(const double* __restrict__ partials, int n,
                                                             double* __restrict__ sc, int mode, int slot) {
    __shared__ double buf[1024], buf2[1024];
    double v = 0.0, v2 = 0.0;
    for (int k = threadIdx.x; k < n; k += 1024) {
        v += partials[k];
        if (mode == RED_PQ) v2 += partials[n + k];
    }
    buf[threadIdx.x] = v;
    buf2[threadIdx.x] = v2;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            buf[threadIdx.x] += buf[threadIdx.x + w];
            buf2[threadIdx.x] += buf2[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double s = buf[0];
        if (mode == RED_SUM) {
            sc[slot] = s;
        } else if (mode == RED_PQ) {
            const double pp = buf2[0];
            sc[S_PQ] = s;
            sc[S_PP] = pp;
            if (!(s <= kStableRayleighHi * pp && s >= kStableRayleighLo * pp)) {
                sc[S_ALPHA] = 0.0;
                sc[S_FLAG] = 2.0;  // Rayleigh quotient beyond a stable step's spectrum
            } else if (s > 0.0) {
                sc[S_ALPHA] = sc[S_RR] / s;
            } else {
                sc[S_ALPHA] = 0.0;
                sc[S_FLAG] = 1.0;  // breakdown: (p, A p)_M <= 0
            }
        } else {  // RED_RR
            sc[S_RRNEW] = s;
            sc[S_BETA] = s / sc[S_RR];
            sc[S_RR] = s;
        }
    }
}

__global__ __launch_bounds__(RB) void cg_xr_kernel(double* __restrict__ x, double* __restrict__ r,
                                                   const double* __restrict__ p, const double* __restrict__ q,
                                                   const double* __restrict__ m, int ncomp, int64_t CS,
                                                   const double* __restrict__ sc, double* __restrict__ partials) {
    const double alpha = sc[S_ALPHA];
    double s = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * RB + threadIdx.x; e < CS; e += (int64_t)gridDim.x * RB) {
        double t = 0.0;
        for (int c = 0; c < ncomp; ++c) {
            const int64_t o = e + c * CS;
            x[o] += alpha * p[o];
            const double rn = r[o] - alpha * q[o];
            r[o] = rn;
            t += rn * rn;
        }
        s += m[e] * t;
    }
    s = block_sum(s);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ void cg_p_kernel(double* __restrict__ p, const double* __restrict__ r, int64_t n,
                            const double* __restrict__ sc) {
    const double beta = sc[S_BETA];
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        p[e] = r[e] + beta * p[e];
}

__global__ void axpby_kernel(double a, const double* __restrict__ x, double b, double* __restrict__ y, int64_t n) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        y[e] = a * x[e] + b * y[e];
}

// Orthogonalisation of GMRES with the coefficients on the device: a Krylov
// vector is H fields, V[H i .. H i + H - 1] (H = 2 for the two-field
// operator, 1 otherwise).  Block (b, i) of multidot adds the M-weighted
// products of vector i with w over its grid-stride share into
// partials[i nb + b]; multireduce sums the nb partials of each i in a fixed
// order.
template <int H>
__global__ __launch_bounds__(RB) void multidot_kernel(const double* const* __restrict__ V,
                                                      const double* __restrict__ wa,
                                                      const double* __restrict__ wb,
                                                      const double* __restrict__ m, int ncomp, int64_t CS,
                                                      double* __restrict__ partials) {
    const int i = blockIdx.y, nb = gridDim.x;
    const double* __restrict__ va = V[H * i];
    const double* __restrict__ vb = V[H * i + H - 1];
    double s = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * RB + threadIdx.x; e < CS; e += (int64_t)nb * RB) {
        double t = 0.0;
        for (int c = 0; c < ncomp; ++c) {
            const int64_t o = e + c * CS;
            t += va[o] * wa[o];
            if (H == 2) t += vb[o] * wb[o];
        }
        s += m[e] * t;
    }
    s = block_sum(s);
    if (threadIdx.x == 0) partials[(int64_t)i * nb + blockIdx.x] = s;
}

__global__ __launch_bounds__(RB) void multireduce_kernel(const double* __restrict__ partials, int nb,
                                                         double* __restrict__ out) {
    double v = 0.0;
    for (int k = threadIdx.x; k < nb; k += RB) v += partials[(int64_t)blockIdx.x * nb + k];
    v = block_sum(v);
    if (threadIdx.x == 0) out[blockIdx.x] = v;
}

// w -= sum_i h[i] V_i over n elements of each field.
template <int H>
__global__ __launch_bounds__(RB) void multiaxpy_kernel(const double* const* __restrict__ V, int k,
                                                       const double* __restrict__ h, double* __restrict__ wa,
                                                       double* __restrict__ wb, int64_t n) {
    for (int64_t e = (int64_t)blockIdx.x * RB + threadIdx.x; e < n; e += (int64_t)gridDim.x * RB) {
        double a = wa[e], b = H == 2 ? wb[e] : 0.0;
        for (int i = 0; i < k; ++i) {
            const double hi = h[i];
            a -= hi * V[H * i][e];
            if (H == 2) b -= hi * V[H * i + 1][e];
        }
        wa[e] = a;
        if (H == 2) wb[e] = b;
    }
}

__global__ void copy_kernel(const double* __restrict__ x, double* __restrict__ y, int64_t n) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        y[e] = x[e];
}

}  // namespace

void launch_pack(const Layout& L, const int bc[6], const double* src, double* dst, int ncomp, hipStream_t s) {
    PackArgs a = pack_args(L, bc, ncomp > 1 ? 1 : 0);
    hipLaunchKernelGGL(pack_kernel<double>, dim3(grid_for(L.CS * ncomp)), dim3(256), 0, s, src, dst, ncomp, a);
}

void launch_pack_f32(const Layout& L, const int bc[6], const double* src, float* dst, int ncomp, hipStream_t s) {
    PackArgs a = pack_args(L, bc, ncomp > 1 ? 1 : 0);
    hipLaunchKernelGGL(pack_kernel<float>, dim3(grid_for(L.CS * ncomp)), dim3(256), 0, s, src, dst, ncomp, a);
}

void launch_unpack(const Layout& L, const int bc[6], const double* src, double* dst, int ncomp, hipStream_t s) {
    PackArgs a = pack_args(L, bc, 1);
    hipLaunchKernelGGL(unpack_kernel, dim3(grid_for(L.nodes_caller() * ncomp)), dim3(256), 0, s, src, dst, ncomp, a);
}

void launch_convert_f32(const Layout& L, const double* src, float* dst, int ncomp, hipStream_t s) {
    const int64_t n = L.CS * ncomp;
    hipLaunchKernelGGL(convert_kernel, dim3(grid_for(n)), dim3(256), 0, s, src, dst, n);
}

void launch_scale_field(const Layout& L, double* dst, const double* w, int ncomp, hipStream_t s) {
    const int64_t n = L.CS * ncomp;
    hipLaunchKernelGGL(scale_field_kernel, dim3(grid_for(n)), dim3(256), 0, s, dst, w, L.CS, n);
}

void launch_dot_M_partial(const elwh_ctx* c, const double* x, const double* y, hipStream_t s) {
    hipLaunchKernelGGL(dotm_partial_kernel, dim3(c->red_blocks), dim3(RB), 0, s, x, y, c->mw, c->L.dim, c->L.CS,
                       c->partials);
}

void launch_dot_pq_pp_partial(const elwh_ctx* c, const double* p, const double* q, hipStream_t s) {
    hipLaunchKernelGGL(dot_pq_pp_partial_kernel, dim3(c->red_blocks), dim3(RB), 0, s, p, q, c->mw, c->L.dim,
                       c->L.CS, c->partials);
}

void launch_reduce_final(const elwh_ctx* c, int mode, int slot, hipStream_t s) {
    hipLaunchKernelGGL(reduce_final_kernel, dim3(1), dim3(1024), 0, s, c->partials, c->red_blocks, c->dscal, mode,
                       slot);
}

void launch_cg_update_xr(const elwh_ctx* c, double* x, double* r, const double* p, const double* q,
                         hipStream_t s) {
    hipLaunchKernelGGL(cg_xr_kernel, dim3(c->red_blocks), dim3(RB), 0, s, x, r, p, q, c->mw, c->L.dim, c->L.CS,
                       c->dscal, c->partials);
}

void launch_cg_update_p(const elwh_ctx* c, double* p, const double* r, hipStream_t s) {
    const int64_t n = c->L.field_elems();
    hipLaunchKernelGGL(cg_p_kernel, dim3(grid_for(n)), dim3(256), 0, s, p, r, n, c->dscal);
}

void launch_axpby(const elwh_ctx* c, double a, const double* x, double b, double* y, hipStream_t s) {
    const int64_t n = c->L.field_elems();
    hipLaunchKernelGGL(axpby_kernel, dim3(grid_for(n)), dim3(256), 0, s, a, x, b, y, n);
}

int multidot2_blocks(const elwh_ctx* c) { return (int)std::min<int64_t>(256, grid_for(c->L.CS, RB)); }

void launch_multidot2(const elwh_ctx* c, const double* const* V, int k, const double* wa, const double* wb,
                      double* partials, double* out, hipStream_t s) {
    const int nb = multidot2_blocks(c);
    if (wb)
        hipLaunchKernelGGL(multidot_kernel<2>, dim3(nb, k), dim3(RB), 0, s, V, wa, wb, c->mw, c->L.dim, c->L.CS,
                           partials);
    else
        hipLaunchKernelGGL(multidot_kernel<1>, dim3(nb, k), dim3(RB), 0, s, V, wa, wa, c->mw, c->L.dim, c->L.CS,
                           partials);
    hipLaunchKernelGGL(multireduce_kernel, dim3(k), dim3(RB), 0, s, partials, nb, out);
}

void launch_multiaxpy2(const elwh_ctx* c, const double* const* V, int k, const double* h, double* wa, double* wb,
                       hipStream_t s) {
    const int64_t n = c->L.field_elems();
    if (wb)
        hipLaunchKernelGGL(multiaxpy_kernel<2>, dim3(grid_for(n, RB)), dim3(RB), 0, s, V, k, h, wa, wb, n);
    else
        hipLaunchKernelGGL(multiaxpy_kernel<1>, dim3(grid_for(n, RB)), dim3(RB), 0, s, V, k, h, wa, wa, n);
}

void launch_copy(const elwh_ctx* c, const double* x, double* y, hipStream_t s) {
    const int64_t n = c->L.field_elems();
    hipLaunchKernelGGL(copy_kernel, dim3(grid_for(n)), dim3(256), 0, s, x, y, n);
}

}  // namespace elwh

// ---- HBM ceiling probe ---------------------------------------------------------
// STREAM triad a = b + s c over n doubles: each thread moves one 32-byte
// vector of each array (three 16-byte vector accesses per array half), the
// grid covers the arrays once, so every byte crosses HBM exactly once when
// the arrays exceed the 256 MiB Infinity Cache.
namespace {
__global__ __launch_bounds__(256) void triad_kernel(double* __restrict__ a, const double* __restrict__ b,
                                                    const double* __restrict__ c, double s, int64_t n4) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= n4) return;
    const double4 bv = reinterpret_cast<const double4*>(b)[t];
    const double4 cv = reinterpret_cast<const double4*>(c)[t];
    double4 r;
    r.x = bv.x + s * cv.x;
    r.y = bv.y + s * cv.y;
    r.z = bv.z + s * cv.z;
    r.w = bv.w + s * cv.w;
    reinterpret_cast<double4*>(a)[t] = r;
}
}  // namespace

extern "C" elwh_status elwh_stream_triad(double* a, const double* b, const double* c, double s, long long n,
                                         void* stream) {
    if (!a || !b || !c || n <= 0 || n % 4 != 0 || ((uintptr_t)a | (uintptr_t)b | (uintptr_t)c) % 32 != 0)
        return ELWH_ERR_ARG;
    const int64_t n4 = n / 4;
    const int64_t blocks = (n4 + 255) / 256;
    if (blocks > 0x7fffffffLL) return ELWH_ERR_ARG;
    hipLaunchKernelGGL(triad_kernel, dim3((unsigned)blocks), dim3(256), 0, static_cast<hipStream_t>(stream), a, b, c,
                       s, n4);
    return hipGetLastError() == hipSuccess ? ELWH_OK : ELWH_ERR_HIP;
}
