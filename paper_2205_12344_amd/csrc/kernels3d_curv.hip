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
// are served by the caches) in straight-line code, so a wavefront has its
// whole footprint in flight at once; one time step per launch.
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

template <typename T, typename U, int MODE, bool FORCE, bool COMP>
__global__ __launch_bounds__(64) void curv3d_kernel(const U* __restrict__ u, const T* uprev, T* unext,
                                                   const double* __restrict__ xbase, T* __restrict__ u0out,
                                                   double* __restrict__ acc, float* __restrict__ acclo,
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
    const int64_t o = (int64_t)k * PS + (int64_t)j * P + i;

    // The gather below is straight-line code: every load is issued without a
    // branch between it and the next, so a wavefront has its whole footprint
    // in flight at once.  j and k are uniform over the wavefront (one (r, s)
    // row per workgroup), so every test on them is a uniform branch; the two
    // tests on i (the q neighbours' being unknowns) are masks.
    const bool flo = A.free_lo && k == 0, fhi = A.free_hi && k == A.ns;
    const bool on_free = flo || fhi;
    const T wp = on_free ? (T)0.5 : (T)1;   // node weight of p, and of its in-plane edges
    const T cq = (T)(0.5 / A.hq), cr = (T)(0.5 / A.hr);
    // D_s at the plane of p: central, one-sided on a free face (the missing
    // plane is read clamped, i.e. as the plane of p itself, and the
    // coefficient doubles)
    const T csp = on_free ? (T)(1.0 / A.hs) : (T)(0.5 / A.hs);
    const int64_t sm = k > 0 ? -PS : 0, sp = k < A.ns ? PS : 0;
    const T iq2 = (T)(1.0 / (A.hq * A.hq)), ir2 = (T)(1.0 / (A.hr * A.hr)), is2 = (T)(1.0 / (A.hs * A.hs));

    struct V3 {
        T x, y, z;
    };
    struct Co {
        T l, m;        // lambda / J, mu / J
        V3 g[3];       // G_q, G_r, G_s
    };
    auto ld = [&](int64_t q) { return V3{(T)u[q], (T)u[q + CS], (T)u[q + 2 * CS]}; };
    auto ldc = [&](int64_t q) {
        Co c;
        c.l = cl[q];
        c.m = cm[q];
#pragma unroll
        for (int a = 0; a < 3; ++a) c.g[a] = V3{G.g[3 * a][q], G.g[3 * a + 1][q], G.g[3 * a + 2][q]};
        return c;
    };
    auto dot = [](const V3& p, const V3& q) { return p.x * q.x + p.y * q.y + p.z * q.z; };
    auto sub = [](const V3& p, const V3& q) { return V3{p.x - q.x, p.y - q.y, p.z - q.z}; };
    // K^ab v = (lambda/J) G_a (G_b . v) + (mu/J) (G_b (G_a . v) + (G_a . G_b) v)
    auto kab = [&](const Co& c, int a, int b, const V3& v) {
        const V3& ga = c.g[a];
        const V3& gb = c.g[b];
        const T gbv = dot(gb, v), gav = dot(ga, v), gab = dot(ga, gb);
        return V3{c.l * ga.x * gbv + c.m * (gb.x * gav + gab * v.x), c.l * ga.y * gbv + c.m * (gb.y * gav + gab * v.y),
                  c.l * ga.z * gbv + c.m * (gb.z * gav + gab * v.z)};
    };
    T Lx = 0, Ly = 0, Lz = 0;
    auto acc3 = [&](T s_, const V3& v) {
        Lx += s_ * v.x;
        Ly += s_ * v.y;
        Lz += s_ * v.z;
    };

    // footprint of u: p, its six face neighbours, its twelve in-plane diagonal neighbours
    const V3 u0 = ld(o);
    const V3 uqm = ld(o - 1), uqp = ld(o + 1), urm = ld(o - P), urp = ld(o + P), usm = ld(o + sm), usp = ld(o + sp);
    const V3 qr_mm = ld(o - 1 - P), qr_mp = ld(o - 1 + P), qr_pm = ld(o + 1 - P), qr_pp = ld(o + 1 + P);
    const V3 qs_mm = ld(o - 1 + sm), qs_mp = ld(o - 1 + sp), qs_pm = ld(o + 1 + sm), qs_pp = ld(o + 1 + sp);
    const V3 rs_mm = ld(o - P + sm), rs_mp = ld(o - P + sp), rs_pm = ld(o + P + sm), rs_pp = ld(o + P + sp);
    const V3 dqm = sub(uqm, u0), dqp = sub(uqp, u0), drm = sub(urm, u0), drp = sub(urp, u0);
    const V3 dsm = sub(usm, u0), dsp = sub(usp, u0);   // 0 across a free face (clamped)

    // edge terms, p's half: sum_a sum_+- w_e/2 K^aa_p (U_n - U_p) / h_a^2
    {
        const Co c = ldc(o);
        const T eq = (T)0.5 * wp * iq2, er = (T)0.5 * wp * ir2, es = (T)0.5 * is2;
        acc3(eq, kab(c, 0, 0, dqm));
        acc3(eq, kab(c, 0, 0, dqp));
        acc3(er, kab(c, 1, 1, drm));
        acc3(er, kab(c, 1, 1, drp));
        acc3(es, kab(c, 2, 2, dsm));
        acc3(es, kab(c, 2, 2, dsp));
        if (on_free) {
            // the one-sided D_s at p itself: (D_s)_pp = -+1/h_s, weight 1/2
            const T s0 = (T)(flo ? 0.5 / A.hs : -0.5 / A.hs);   // -(D_s)_pp w_p
            acc3(s0, kab(c, 2, 0, V3{(uqp.x - uqm.x) * cq, (uqp.y - uqm.y) * cq, (uqp.z - uqm.z) * cq}));
            acc3(s0, kab(c, 2, 1, V3{(urp.x - urm.x) * cr, (urp.y - urm.y) * cr, (urp.z - urm.z) * cr}));
        }
    }
    // q neighbours: the other half of their edge term, and their cross terms
    // -(D_q)_np w_n K^qb_n (D_b U)_n, (D_q)_np = -+1/(2 h_q) for n = p +- e_q
    {
        const T mm = i - 1 >= 1 ? (T)1 : (T)0, mp = i + 1 <= A.nq - 1 ? (T)1 : (T)0;   // unknowns
        const Co cm_ = ldc(o - 1), cp_ = ldc(o + 1);
        const T eq = (T)0.5 * wp * iq2;
        acc3(eq, kab(cm_, 0, 0, dqm));
        acc3(eq, kab(cp_, 0, 0, dqp));
        const T sm_ = -cq * wp * mm, sp_ = cq * wp * mp;   // -(D_q)_np w_n, masked
        acc3(sm_, kab(cm_, 0, 1, V3{(qr_mp.x - qr_mm.x) * cr, (qr_mp.y - qr_mm.y) * cr, (qr_mp.z - qr_mm.z) * cr}));
        acc3(sm_, kab(cm_, 0, 2, V3{(qs_mp.x - qs_mm.x) * csp, (qs_mp.y - qs_mm.y) * csp, (qs_mp.z - qs_mm.z) * csp}));
        acc3(sp_, kab(cp_, 0, 1, V3{(qr_pp.x - qr_pm.x) * cr, (qr_pp.y - qr_pm.y) * cr, (qr_pp.z - qr_pm.z) * cr}));
        acc3(sp_, kab(cp_, 0, 2, V3{(qs_pp.x - qs_pm.x) * csp, (qs_pp.y - qs_pm.y) * csp, (qs_pp.z - qs_pm.z) * csp}));
    }
    // r neighbours (uniform tests)
    {
        const Co cm_ = ldc(o - P), cp_ = ldc(o + P);
        const T er = (T)0.5 * wp * ir2;
        acc3(er, kab(cm_, 1, 1, drm));
        acc3(er, kab(cp_, 1, 1, drp));
        if (j - 1 >= 1) {
            const T s_ = -cr * wp;
            acc3(s_, kab(cm_, 1, 0, V3{(qr_pm.x - qr_mm.x) * cq, (qr_pm.y - qr_mm.y) * cq, (qr_pm.z - qr_mm.z) * cq}));
            acc3(s_, kab(cm_, 1, 2, V3{(rs_mp.x - rs_mm.x) * csp, (rs_mp.y - rs_mm.y) * csp, (rs_mp.z - rs_mm.z) * csp}));
        }
        if (j + 1 <= A.nr - 1) {
            const T s_ = cr * wp;
            acc3(s_, kab(cp_, 1, 0, V3{(qr_pp.x - qr_mp.x) * cq, (qr_pp.y - qr_mp.y) * cq, (qr_pp.z - qr_mp.z) * cq}));
            acc3(s_, kab(cp_, 1, 2, V3{(rs_pp.x - rs_pm.x) * csp, (rs_pp.y - rs_pm.y) * csp, (rs_pp.z - rs_pm.z) * csp}));
        }
    }
    // s neighbours (uniform tests): across a free face there is none (its
    // edge difference is 0 by the clamped read); -(D_s)_np w_n is +-1/(2 h_s)
    // also where n lies on a free face (one-sided coefficient 1/h_s, weight 1/2)
    {
        const Co cm_ = ldc(o + sm), cp_ = ldc(o + sp);
        const T es = (T)0.5 * is2;
        acc3(es, kab(cm_, 2, 2, dsm));
        acc3(es, kab(cp_, 2, 2, dsp));
        const T cs2 = (T)(0.5 / A.hs);
        if (k - 1 >= A.klo) {
            acc3(-cs2, kab(cm_, 2, 0, V3{(qs_pm.x - qs_mm.x) * cq, (qs_pm.y - qs_mm.y) * cq, (qs_pm.z - qs_mm.z) * cq}));
            acc3(-cs2, kab(cm_, 2, 1, V3{(rs_pm.x - rs_mm.x) * cr, (rs_pm.y - rs_mm.y) * cr, (rs_pm.z - rs_mm.z) * cr}));
        }
        if (k + 1 <= A.khi) {
            acc3(cs2, kab(cp_, 2, 0, V3{(qs_pp.x - qs_mp.x) * cq, (qs_pp.y - qs_mp.y) * cq, (qs_pp.z - qs_mp.z) * cq}));
            acc3(cs2, kab(cp_, 2, 1, V3{(rs_pp.x - rs_mp.x) * cr, (rs_pp.y - rs_mp.y) * cr, (rs_pp.z - rs_mp.z) * cr}));
        }
    }
    const T uc[3] = {u0.x, u0.y, u0.z};
    const T L[3] = {Lx, Ly, Lz};

    // L_h / w_p, then the corrected leapfrog with the trapezoid accumulation
    const T iw = (T)1 / wp;
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
            if constexpr (COMP) acclo[oq] = (float)lq;
        }
    }
}

bool tile_valid_curv3(bool fp32, int V, int TY) {
    (void)fp32;
    return V == 1 && TY == 4;
}

template <typename T, typename U, int MODE>
static void launch_c3(bool force, bool comp, const ArgsC3& A, hipStream_t s, const U* u, const T* uprev, T* unext,
                      const double* xbase, T* u0out, double* acc, float* acclo, const T* ca, const T* cl,
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
    float* lo = c->acc_lo;
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
