// Bookkeeping and Krylov kernels of the ragged batch of 2-D problems: the
// per-tick advance of every problem's step counter and state-buffer roles,
// the CG updates in the M inner product (Sec. 3.2: alpha from (p, A p)_M,
// x and r updates with (r, r)_M, the new direction) of the problems that
// finished an application in the tick, and the per-problem linear
// combinations and M inner products of the set-up and fallback phases.
#include "step2d_common.h"   // the buffer-role rules shared with the step kernels

namespace elwh {

// Advance the step counters and the roles of the state buffers after a tick
// (the same rules the step kernels applied).  single: the phase is one
// application per problem (deactivate when it completes).  After the half
// step u^{n-1} = u^0 is src in FP64 and s[0] in FP32.
__global__ void batch_advance_kernel(const BProb2D* __restrict__ pr, BState* __restrict__ st, int np, int single,
                                     int kb, int fp32) {
    const int p = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (p >= np || !st[p].active) return;
    BState& s = st[p];
    const int neff = s.end ? 0 : s.n;
    int steps = 1;
    if (neff == 0) {
        s.ip = fp32 ? 0 : -1;
        s.ic = 1;
    } else if (batch_multi_step(neff, pr[p].nsteps, kb)) {
        // u^{n+kb-1} and u^{n+kb} went to the two free buffers
        int x1, x2;
        batch_free_two(s.ic, s.ip, x1, x2);
        s.ip = x1;
        s.ic = x2;
        steps = kb;
    } else {
        const int nxt = batch_single_target(s.ic, s.ip);
        s.ip = s.ic;
        s.ic = nxt;
    }
    s.n = neff + steps;
    s.end = s.n == pr[p].nsteps;
    if (single && s.end) s.active = 0;
}

constexpr int BRB = 64;   // reduction blocks per problem

template <int MODE>
__device__ __forceinline__ void batch_cg_finish(BState& b, double s, double s2, int* __restrict__ n_active);

// mode 0: partials (p, q)_M (partials[p BRB + k]) and (p, p)_M (partials[(np + p) BRB + k]);
// mode 1: x += alpha p, r -= alpha q, partial (r, r)_M; mode 2: p = r + beta p.
// Only problems that finished an application this tick.  BRB blocks per
// listed problem: block b works for problem plist[b / BRB] (the problems
// still active when the launch was set up; nplist of them).  In modes 0
// and 1 the last of a problem's BRB blocks to finish (arrive[p] counts
// them and is reset to zero by that block) adds up the BRB partials in a
// fixed order and finishes the CG update of the problem.
template <int MODE>
__global__ __launch_bounds__(256) void batch_cg_kernel(const BProb2D* __restrict__ pr, BState* __restrict__ st,
                                                       int np, const int* __restrict__ plist, int nplist,
                                                       double* __restrict__ partials, int* __restrict__ arrive,
                                                       int* __restrict__ n_active) {
    const int slot = (int)blockIdx.x / BRB, k = (int)blockIdx.x % BRB;
    if (slot >= nplist) return;
    const int p = plist[slot];
    if (p < 0 || p >= np || !st[p].active || !st[p].end) return;
    const BProb2D& q = pr[p];
    const int64_t CS = q.A.CS;
    double s = 0.0, s2 = 0.0;
    const double alpha = st[p].alpha, beta = st[p].beta;
    for (int64_t e = (int64_t)k * 256 + threadIdx.x; e < CS; e += (int64_t)BRB * 256) {
        const double me = q.m[e];
        double t = 0.0, t2 = 0.0;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int64_t o = e + c * CS;
            if (MODE == 0) {
                const double pv = q.cp[o];
                t += pv * q.out[o];
                t2 += pv * pv;
            } else if (MODE == 1) {
                q.cx[o] += alpha * q.cp[o];
                const double rn = q.cr[o] - alpha * q.out[o];
                q.cr[o] = rn;
                t += rn * rn;
            } else {
                q.cp[o] = q.cr[o] + beta * q.cp[o];
            }
        }
        s += me * t;
        s2 += me * t2;
    }
    if (MODE == 2) return;
    // wavefront then block reduction
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        s += __shfl_down(s, off, 64);
        s2 += __shfl_down(s2, off, 64);
    }
    __shared__ double red[4], red2[4];
    __shared__ int last;
    if ((threadIdx.x & 63) == 0) {
        red[threadIdx.x >> 6] = s;
        red2[threadIdx.x >> 6] = s2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        partials[p * BRB + k] = red[0] + red[1] + red[2] + red[3];
        if (MODE == 0) partials[(np + p) * BRB + k] = red2[0] + red2[1] + red2[2] + red2[3];
        __threadfence();
        last = atomicAdd(&arrive[p], 1) == BRB - 1;
        if (last) __threadfence();
    }
    __syncthreads();
    if (!last || threadIdx.x >= 64) return;
    // the last block: the BRB partials of problem p, read from L2, in order
    double t = __hip_atomic_load(&partials[p * BRB + threadIdx.x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    double t2 = MODE == 0 ? __hip_atomic_load(&partials[(np + p) * BRB + threadIdx.x], __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT)
                          : 0.0;   // BRB == 64: one partial per lane of the first wavefront
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        t += __shfl_down(t, off, 64);
        t2 += __shfl_down(t2, off, 64);
    }
    if (threadIdx.x == 0) {
        batch_cg_finish<MODE>(st[p], t, t2, n_active);
        arrive[p] = 0;
    }
}

// Finish the reduction of an ending problem (sums s of (p, q)_M or (r, r)_M
// and s2 of (p, p)_M): mode 0: alpha = rr / pq with the stability and
// breakdown tests; mode 1: rr, beta, iteration count and the stopping tests.
template <int MODE>
__device__ __forceinline__ void batch_cg_finish(BState& b, double s, double s2, int* __restrict__ n_active) {
    if (MODE == 0) {
        b.pq = s;
        if (!(s <= kStableRayleighHi * s2 && s >= kStableRayleighLo * s2)) {
            b.status = ELWH_ERR_UNSTABLE;   // Rayleigh quotient beyond a stable step's spectrum
            b.active = 0;
            atomicSub(n_active, 1);
        } else if (s > 0.0 && isfinite(s)) {
            b.alpha = b.rr / s;
        } else {
            b.status = isfinite(s) ? ELWH_ERR_BREAKDOWN : ELWH_ERR_UNSTABLE;
            b.active = 0;
            atomicSub(n_active, 1);
        }
    } else {
        b.beta = s / b.rr;
        b.rr = s;
        b.iters++;
        if (!isfinite(s)) {
            b.status = ELWH_ERR_UNSTABLE;
        } else if (s <= b.tol2 * b.bb) {
            b.status = ELWH_OK;
        } else if (b.iters >= b.maxit) {
            b.status = ELWH_ERR_NOT_CONVERGED;
        } else {
            return;
        }
        b.active = 0;
        atomicSub(n_active, 1);
    }
}

// dst = alpha a + beta b over the whole padded field of every selected problem
// (vector indices into BProb2D::vec; ib < 0: no b; betav != null: beta is
// betav[p], one per problem).  sel: problems with a non-zero flag in mask.
__global__ __launch_bounds__(256) void batch_lincomb_kernel(const BProb2D* __restrict__ pr, int np,
                                                            const int* __restrict__ mask, int idst, int ia,
                                                            double alpha, int ib, double beta,
                                                            const double* __restrict__ betav) {
    const int p = (int)blockIdx.x / BRB, k = (int)blockIdx.x % BRB;
    if (p >= np || (mask && !mask[p])) return;
    if (betav) beta = betav[p];
    const BProb2D& q = pr[p];
    double* d = q.vec[idst];
    const double* a = q.vec[ia];
    const double* bb = ib >= 0 ? q.vec[ib] : nullptr;
    const int64_t n = 2 * q.A.CS;
    for (int64_t e = (int64_t)k * 256 + threadIdx.x; e < n; e += (int64_t)BRB * 256)
        d[e] = alpha * a[e] + (bb ? beta * bb[e] : 0.0);
}

// Per-problem (a, b)_M into out[p] (two passes: partials, then one block).
__global__ __launch_bounds__(256) void batch_dot_partial_kernel(const BProb2D* __restrict__ pr, int np,
                                                                const int* __restrict__ mask, int ia, int ib,
                                                                double* __restrict__ partials) {
    const int p = (int)blockIdx.x / BRB, k = (int)blockIdx.x % BRB;
    if (p >= np || (mask && !mask[p])) return;
    const BProb2D& q = pr[p];
    const double* a = q.vec[ia];
    const double* b = q.vec[ib];
    const int64_t CS = q.A.CS;
    double s = 0.0;
    for (int64_t e = (int64_t)k * 256 + threadIdx.x; e < CS; e += (int64_t)BRB * 256)
        s += q.m[e] * (a[e] * b[e] + a[e + CS] * b[e + CS]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    __shared__ double red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) partials[p * BRB + k] = red[0] + red[1] + red[2] + red[3];
}

__global__ __launch_bounds__(64) void batch_dot_final_kernel(int np, const int* __restrict__ mask,
                                                             const double* __restrict__ partials,
                                                             double* __restrict__ out) {
    const int p = (int)blockIdx.x;
    if (p >= np || (mask && !mask[p])) return;
    double s = partials[p * BRB + threadIdx.x];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if (threadIdx.x == 0) out[p] = s;
}

void launch_batch_advance(hipStream_t s, const BProb2D* pr, BState* st, int np, int single, int kb, int fp32) {
    hipLaunchKernelGGL(batch_advance_kernel, dim3((np + 63) / 64), dim3(64), 0, s, pr, st, np, single, kb, fp32);
}

void launch_batch_cg(hipStream_t s, int mode, const BProb2D* pr, BState* st, int np, const int* plist, int nplist,
                     double* partials, int* arrive, int* n_active) {
    if (nplist < 1) return;
    const dim3 g((unsigned)(nplist * BRB));
    if (mode == 0)
        hipLaunchKernelGGL(batch_cg_kernel<0>, g, dim3(256), 0, s, pr, st, np, plist, nplist, partials, arrive,
                           n_active);
    else if (mode == 1)
        hipLaunchKernelGGL(batch_cg_kernel<1>, g, dim3(256), 0, s, pr, st, np, plist, nplist, partials, arrive,
                           n_active);
    else
        hipLaunchKernelGGL(batch_cg_kernel<2>, g, dim3(256), 0, s, pr, st, np, plist, nplist, partials, arrive,
                           n_active);
}

void launch_batch_lincomb(hipStream_t s, const BProb2D* pr, int np, const int* mask, int idst, int ia, double alpha,
                          int ib, double beta, const double* betav) {
    hipLaunchKernelGGL(batch_lincomb_kernel, dim3((unsigned)(np * BRB)), dim3(256), 0, s, pr, np, mask, idst, ia,
                       alpha, ib, beta, betav);
}

void launch_batch_dot(hipStream_t s, const BProb2D* pr, int np, const int* mask, int ia, int ib, double* partials,
                      double* out) {
    hipLaunchKernelGGL(batch_dot_partial_kernel, dim3((unsigned)(np * BRB)), dim3(256), 0, s, pr, np, mask, ia, ib,
                       partials);
    hipLaunchKernelGGL(batch_dot_final_kernel, dim3(np), dim3(64), 0, s, np, mask, partials, out);
}

}  // namespace elwh
