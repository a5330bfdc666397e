// Fused El-WaveHoltz step on a mapped 3-D grid (Sec. 4.1 in three
// dimensions; the partial toroidal shell of Sec. 5.11).
//
// The unit cube (q, r, s) is mapped to the domain; with G_a = J grad a and
// the 3x3 blocks K^{ab} = (1/J) [lam G_a G_b^T + mu (G_a . G_b) I +
// mu G_b G_a^T], L_h is minus the gradient of the discrete energy
//   E_h = 1/2 sum_a sum_{a-edges} w_e (D+a U)^T Kbar^aa (D+a U)
//       + sum_{a != b} sum_{unknown n} w_n (Dh_a U)_n^T K^ab_n (Dh_b U)_n / 2
// (Kbar the mean over the edge's two nodes, Dh central, one-sided into the
// domain on a free s face, w the trapezoid weights: 1/2 on a free s face).
// Row p of L_h is gathered directly:
//   L_p = sum_a sum_{+-} w_e Kbar^aa (U_{p +- e_a} - U_p) / h_a^2
//       - sum_{a != b} sum_n (Dh_a)_{n,p} w_n K^ab_n (Dh_b U)_n,
// where K^ab v = (lam/J) G_a (G_b . v) + (mu/J) (G_b (G_a . v) + (G_a . G_b) v)
// is formed from lam/J, mu/J and the nine metric values at the node (no 3x3
// block is stored).  The step is the corrected leapfrog of Sec. 4.3 with mass
// rho J (a = c dt^2 / (rho J), forcing J f) and the trapezoid accumulation
// of eq. el_WHI_OP fused in, as in the Cartesian kernels.
//
// Mapping: one thread per node, 64 consecutive q nodes per wavefront, one
// (r, s) row per workgroup, XCD-banded; every neighbour value is loaded
// (the 19-point footprint and the coefficients of the six face neighbours
// are served by the caches), one time step per launch.
#include "elwh_internal.h"
#include "xcd.h"

namespace elwh {

struct ArgsC3 {
    int nq, nr, ns;
    int64_t P, PS, CS;
    int klo, khi, free_lo, free_hi;
    double hq, hr, hs;
    double w, w0, fc;
    int final_;
};

template <typename T>
struct Metric3 {
    const T* g[9];   // G_q, G_r, G_s by component
};

__device__ __forceinline__ void acc_add_c3(double& hi, double& lo, double x, bool comp) {
    if (comp) {
        const double t = hi + x;
        const double z = t - hi;
        const double e = (hi - (t - z)) + (x - z);
        hi = t;
        lo += e;
    } else {
        hi += x;
    }
}

// Dh along one axis at index t (0..N): central inside, one-sided into the
// domain on a free face, nothing on a Dirichlet face.
__device__ __forceinline__ int dh_coef(int t, int N, double h, bool flo, bool fhi, int off[2], double cf[2]) {
    if (t >= 1 && t <= N - 1) {
        off[0] = 1; cf[0] = 0.5 / h;
        off[1] = -1; cf[1] = -0.5 / h;
        return 2;
    }
    if (t == 0 && flo) {
        off[0] = 1; cf[0] = 1.0 / h;
        off[1] = 0; cf[1] = -1.0 / h;
        return 2;
    }
    if (t == N && fhi) {
        off[0] = 0; cf[0] = 1.0 / h;
        off[1] = -1; cf[1] = -1.0 / h;
        return 2;
    }
    return 0;
}

template <typename T, typename U, int MODE, bool FORCE, bool COMP>
__global__ __launch_bounds__(64) void curv3d_kernel(const U* __restrict__ u, const T* uprev, T* unext,
                                                   const double* __restrict__ xbase, T* __restrict__ u0out,
                                                   double* __restrict__ acc, double* __restrict__ acclo,
                                                   const T* __restrict__ ca, const T* __restrict__ cl,
                                                   const T* __restrict__ cm, Metric3<T> G, const T* __restrict__ f,
                                                   ArgsC3 A) {
    const int nbx = (A.nq - 1 + 63) / 64, nrr = A.nr - 1, npl = A.khi - A.klo + 1;
    int t;
    if (!xcd_tile((int)blockIdx.x, nbx * nrr * npl, t)) return;
    const int i = 1 + 64 * (t % nbx) + (int)threadIdx.x;
    const int j = 1 + (t / nbx) % nrr;
    const int k = A.klo + t / (nbx * nrr);
    if (i > A.nq - 1) return;
    const int64_t P = A.P, PS = A.PS, CS = A.CS;
    const int64_t st[3] = {1, P, PS};
    const int N[3] = {A.nq, A.nr, A.ns};
    const double h[3] = {A.hq, A.hr, A.hs};
    const int tp[3] = {i, j, k};
    const int64_t o = (int64_t)k * PS + (int64_t)j * P + i;

    auto load3 = [&](int64_t q, T v[3]) {
#pragma unroll
        for (int c = 0; c < 3; ++c) v[c] = (T)u[q + c * CS];
    };
    // out = K^ab_n v
    auto kv = [&](int64_t n, int a, int b, const T v[3], T out[3]) {
        const T l = cl[n], m = cm[n];
        T ga[3], gb[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            ga[c] = G.g[3 * a + c][n];
            gb[c] = G.g[3 * b + c][n];
        }
        const T gbv = gb[0] * v[0] + gb[1] * v[1] + gb[2] * v[2];
        const T gav = ga[0] * v[0] + ga[1] * v[1] + ga[2] * v[2];
        const T gab = ga[0] * gb[0] + ga[1] * gb[1] + ga[2] * gb[2];
#pragma unroll
        for (int c = 0; c < 3; ++c) out[c] = l * ga[c] * gbv + m * (gb[c] * gav + gab * v[c]);
    };
    auto unknown = [&](int ti, int tj, int tk) {
        return ti >= 1 && ti <= A.nq - 1 && tj >= 1 && tj <= A.nr - 1 && tk >= A.klo && tk <= A.khi;
    };
    auto wnode = [&](int tk) {
        return ((A.free_lo && tk == 0) || (A.free_hi && tk == A.ns)) ? (T)0.5 : (T)1;
    };

    T uc[3];
    load3(o, uc);
    T L[3] = {(T)0, (T)0, (T)0};
    // edge terms
    const bool in_free_s = (A.free_lo && k == 0) || (A.free_hi && k == A.ns);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const T we = (a < 2 && in_free_s) ? (T)0.5 : (T)1;
        const T ih2 = (T)(1.0 / (h[a] * h[a]));
#pragma unroll
        for (int sg = -1; sg <= 1; sg += 2) {
            const int tn = tp[a] + sg;
            if (tn < 0 || tn > N[a]) continue;
            const int64_t n = o + sg * st[a];
            T un[3], d[3], k0[3], k1[3];
            load3(n, un);
#pragma unroll
            for (int c = 0; c < 3; ++c) d[c] = un[c] - uc[c];
            kv(o, a, a, d, k0);
            kv(n, a, a, d, k1);
#pragma unroll
            for (int c = 0; c < 3; ++c) L[c] += we * (T)0.5 * ih2 * (k0[c] + k1[c]);
        }
    }
    // node terms over the ordered axis pairs
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            if (a == b) continue;
            for (int da = -1; da <= 1; ++da) {
                int tn[3] = {i, j, k};
                tn[a] += da;
                if (!unknown(tn[0], tn[1], tn[2])) continue;
                int oa[2], ob[2];
                double cfa[2], cfb[2];
                const int na = dh_coef(tn[a], N[a], h[a], a == 2 && A.free_lo, a == 2 && A.free_hi, oa, cfa);
                double cpa = 0.0;
                for (int q = 0; q < na; ++q)
                    if (tn[a] + oa[q] == tp[a]) cpa += cfa[q];
                if (cpa == 0.0) continue;
                const int64_t n = o + da * st[a];
                const int nb = dh_coef(tn[b], N[b], h[b], b == 2 && A.free_lo, b == 2 && A.free_hi, ob, cfb);
                T dbu[3] = {(T)0, (T)0, (T)0};
                for (int q = 0; q < nb; ++q) {
                    T um[3];
                    load3(n + ob[q] * st[b], um);
#pragma unroll
                    for (int c = 0; c < 3; ++c) dbu[c] += (T)cfb[q] * um[c];
                }
                T F[3];
                kv(n, a, b, dbu, F);
                const T s = (T)cpa * wnode(tn[2]);
#pragma unroll
                for (int c = 0; c < 3; ++c) L[c] -= s * F[c];
            }
        }
    }

    // L_h / w_p, then the corrected leapfrog with the trapezoid accumulation
    const T iw = (T)1 / wnode(k);
    const T a_ = ca[o];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const int64_t oq = o + q * CS;
        T Lq = L[q] * iw;
        if constexpr (FORCE) Lq -= (T)A.fc * f[oq];
        double hq = 0.0, lq = 0.0;
        T nq;
        if constexpr (MODE == 0) {
            hq = acc[oq];
            if constexpr (COMP) lq = acclo[oq];
            nq = (T)2 * uc[q] - uprev[oq] + a_ * Lq;
        } else {
            hq = xbase ? xbase[oq] : 0.0;
            nq = uc[q] + (T)0.5 * a_ * Lq;
            acc_add_c3(hq, lq, A.w0 * (double)uc[q], COMP);
            if (u0out) u0out[oq] = uc[q];
        }
        unext[oq] = nq;
        acc_add_c3(hq, lq, A.w * (double)nq, COMP);
        if (COMP && A.final_) {
            acc[oq] = hq + lq;
        } else {
            acc[oq] = hq;
            if constexpr (COMP) acclo[oq] = lq;
        }
    }
}

bool tile_valid_curv3(bool fp32, int V, int TY) {
    (void)fp32;
    return V == 1 && TY == 4;
}

template <typename T, typename U, int MODE>
static void launch_c3(bool force, bool comp, const ArgsC3& A, hipStream_t s, const U* u, const T* uprev, T* unext,
                      const double* xbase, T* u0out, double* acc, double* acclo, const T* ca, const T* cl,
                      const T* cm, const Metric3<T>& G, const T* f) {
    const int nbx = (A.nq - 1 + 63) / 64;
    const dim3 grid((unsigned)xcd_grid(nbx * (A.nr - 1) * (A.khi - A.klo + 1)));
#define ELWH_LC3(F, CMP)                                                                                        \
    hipLaunchKernelGGL((curv3d_kernel<T, U, MODE, F, CMP>), grid, dim3(64), 0, s, u, uprev, unext, xbase, u0out, \
                       acc, acclo, ca, cl, cm, G, f, A)
    if (force) {
        if (comp) ELWH_LC3(true, true); else ELWH_LC3(true, false);
    } else {
        if (comp) ELWH_LC3(false, true); else ELWH_LC3(false, false);
    }
#undef ELWH_LC3
}

void run_filter_curv3d(elwh_ctx* c, const double* x, bool with_force, bool amode, bool fp32, double* out) {
    hipStream_t s = c->stream;
    ArgsC3 A;
    A.nq = c->L.nx;
    A.nr = c->L.ny;
    A.ns = c->L.nz;
    A.P = c->L.P;
    A.PS = c->L.PS;
    A.CS = c->L.CS;
    A.klo = c->mr.lo;
    A.khi = c->mr.hi;
    A.free_lo = c->mr.free_lo;
    A.free_hi = c->mr.free_hi;
    A.hq = 1.0 / c->L.nx;
    A.hr = 1.0 / c->L.ny;
    A.hs = 1.0 / c->L.nz;
    A.final_ = 0;
    const int nsteps = c->plan.nt * c->opts.periods;
    const double sgn = amode ? -1.0 : 1.0;
    const bool comp = fp32 && c->opts.compensated;
    double* acc = out;
    double* lo = c->acc_lo;
    A.w0 = sgn * c->w[0];
    A.w = sgn * c->w[1];
    A.fc = c->cosn[0];
    if (!fp32) {
        Metric3<double> G;
        for (int q = 0; q < 9; ++q) G.g[q] = c->cg[q];
        double *b0 = c->s64[0], *b1 = c->s64[1];
        prof_mark(c, 0);
        launch_c3<double, double, 1>(with_force, false, A, s, x, nullptr, b1, amode ? x : nullptr, nullptr, acc, lo,
                                     c->ca, c->cl, c->cm, G, c->f64);
        prof_mark(c, 1);
        const double* prev = x;
        double* cur = b1;
        for (int n = 1; n < nsteps; ++n) {
            double* nxt = (n == 1) ? b0 : const_cast<double*>(prev);
            A.w = sgn * c->w[n + 1];
            A.fc = c->cosn[n];
            launch_c3<double, double, 0>(with_force, false, A, s, cur, prev, nxt, nullptr, nullptr, acc, lo, c->ca,
                                         c->cl, c->cm, G, c->f64);
            prev = cur;
            cur = nxt;
        }
    } else {
        Metric3<float> G;
        for (int q = 0; q < 9; ++q) G.g[q] = c->fg[q];
        float *b0 = c->s32[0], *b1 = c->s32[1];
        prof_mark(c, 0);
        launch_c3<float, double, 1>(with_force, comp, A, s, x, nullptr, b1, amode ? x : nullptr, b0, acc, lo, c->fa,
                                    c->fl, c->fm, G, c->f32);
        prof_mark(c, 1);
        float* prev = b0;
        float* cur = b1;
        for (int n = 1; n < nsteps; ++n) {
            A.w = sgn * c->w[n + 1];
            A.fc = c->cosn[n];
            A.final_ = (n == nsteps - 1);
            launch_c3<float, float, 0>(with_force, comp, A, s, cur, prev, prev, nullptr, nullptr, acc, lo, c->fa,
                                       c->fl, c->fm, G, c->f32);
            float* t = prev;
            prev = cur;
            cur = t;
        }
    }
    prof_mark(c, 2, nsteps - 1);
}

}  // namespace elwh
