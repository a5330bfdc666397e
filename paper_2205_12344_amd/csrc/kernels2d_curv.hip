// Fused El-WaveHoltz step on a mapped (curvilinear) 2-D grid, for gfx950.
//
// The domain is the image of the unit square under (q, r) -> (x, y); the
// equations are J times the elastic wave equation in conservation form on
// the square (Sec. 4.1).  With U = (u, v) and the 2x2 blocks
//     K^ab = (1/J) [lam G_a G_b^T + mu (G_a . G_b) I + mu G_b G_a^T],
// G_q = J grad q, G_r = J grad r (stored per node, with lam/J and mu/J), the
// operator at an interior node is
//     L_h U = D+q(Kbar^qq D-q U) + D+r(Kbar^rr D-r U)
//           + D0q(K^qr D0r U) + D0r(K^rq D0q U),     K^rq = (K^qr)^T,
// bars two-point means: the Hessian of a non-negative discrete energy, so
// the scheme conserves it.  One launch advances every interior node by one
// step of the corrected leapfrog (Sec. 4.3)
//     u^{n+1} = 2 u^n - u^{n-1} + a (L_h u^n - J f cos(omega t_n)),
//     a = c dt^2 / (rho J),
// and adds w_{n+1} u^{n+1} into the FP64 filter accumulator in the same pass;
// the half-step launch computes the even-in-time start u^1 = u^0 +
// (a/2)(L_h u^0 - J f) and seeds the accumulator, as on Cartesian grids.
//
// Mapping.  One 64-lane wavefront per block; lane k owns V consecutive q
// nodes; a wavefront marches TY rows in r (up in even row chunks, down in
// odd ones).  Each row is loaded once per
// row visit (u, v, lam/J, mu/J and the four metric values); when it enters
// the register ring its blocks K^qq, K^rr, K^qr and the vector
// Q = (K^qr)^T (U_{i+1} - U_{i-1}) are formed in registers, so the cross
// term D0r(K^rq D0q U) of the centre row is (Q_N - Q_S) / (4 h_q h_r).  The
// other cross term needs P = K^qr (U_N - U_S) at the q neighbours: P is
// formed per lane and moved across lanes by DPP shifts, like K^qq and the
// neighbour displacements.  Dirichlet nodes hold zero displacement and the
// padding zero coefficients, so interior nodes need no special case.
//
// Traction-free r sides (rows r = 0 / r = 1) are closed from the same
// energy with trapezoid weight 1/2 on the side's nodes and q-edges and the
// one-sided r difference in its cross terms; divided by the weight, the row
// of the top side reads
//     D+q(Kbar^qq D-q U) - (K^rr_C + K^rr_S)(U_C - U_S) / h_r^2
//     + [P'_{i+1} - P'_{i-1} - (Q_C + Q_S)] / (2 h_q h_r),
// P' = K^qr (U_C - U_S), and the bottom side mirrors it.
#include "step2d_common.h"

namespace elwh {

namespace {

template <typename T, int V>
struct CRaw {
    T u[V], v[V], l[V], m[V], g0[V], g1[V], g2[V], g3[V];
};

// One row of the ring (S keeps only what the centre row reads of it).
template <typename T, int V>
struct CRow {
    T u[V], v[V];
    T uL, uR, vL, vR;                      // displacements across the lane edges
    T qq0[V], qq1[V], qq2[V];              // K^qq: 00, 01 (= 10), 11
    T rr0[V], rr1[V], rr2[V];              // K^rr
    T qr0[V], qr1[V], qr2[V], qr3[V];      // K^qr: 00, 01, 10, 11
    T Q0[V], Q1[V];                        // (K^qr)^T (U_{i+1} - U_{i-1})
};

template <typename T, int V, bool COMP, bool FORCE, int MODE>
struct CCtr {
    T a[V];
    T up[V], vp[V];
    double hu[V], hv[V];
    float lu[V], lv[V];   // compensation, widened where it is used
    T fu[V], fv[V];
};

template <typename T, int V>
__device__ __forceinline__ T at_left(const T (&x)[V], int k, T edge) {
    return k > 0 ? x[k > 0 ? k - 1 : 0] : edge;
}
template <typename T, int V>
__device__ __forceinline__ T at_right(const T (&x)[V], int k, T edge) {
    return k < V - 1 ? x[k < V - 1 ? k + 1 : 0] : edge;
}

template <typename T, typename U, int V, int TY, int MODE, bool FORCE, bool COMP>
__device__ __forceinline__ void curv2d_body(int bx, int by, const U* __restrict__ u, const T* uprev, T* unext,
                                            const double* __restrict__ xbase, T* __restrict__ u0out,
                                            double* __restrict__ acc, float* __restrict__ acclo,
                                            const T* __restrict__ ca, const T* __restrict__ cl,
                                            const T* __restrict__ cm, const T* __restrict__ g0,
                                            const T* __restrict__ g1, const T* __restrict__ g2,
                                            const T* __restrict__ g3, const T* __restrict__ f, const Args2D& A) {
    constexpr int W = Cols<V>::W;
    const int lane = threadIdx.x;
    const int c0 = W * bx;
    const int col = c0 + V * lane;
    const bool colv = col <= A.nx;
    const int j0 = A.jlo + by * TY;
    if (j0 > A.jhi) return;
    const int j1 = min(j0 + TY - 1, A.jhi);
    const int P = (int)A.P;
    const int64_t CS = A.CS;
    // Mirrored march: odd row chunks march downwards, so that neighbouring
    // chunks read the rows they share at the same time and the second read
    // finds them in L2.  Virtual row v is physical row jb + dir * v.  With
    // the rows below and above exchanged, P changes sign and the compact r
    // term does not, so the mirrored stencil is the same stencil with both
    // cross-term coefficients negated and the two free-row kinds swapped.
    const int dir = (by & 1) ? -1 : 1;
    const int jb = dir > 0 ? 0 : j0 + j1;
    auto phys = [&](int v) { return jb + dir * v; };
    const T cqq2 = (T)A.cxx2, crr2 = (T)A.cyy2, cqr = (T)(dir * A.cxy);
    const T crrf = (T)A.cyyf, cqrf = (T)(dir * A.cfx);   // free rows: 1/h_r^2, +-1/(2 h_q h_r)
    const T two = (T)2;
    const int ilo = max(c0 + 1, 1), ihi = min(c0 + W, A.nx - 1);

    auto load_raw = [&](int jv, CRaw<T, V>& r) {
        const int j = phys(jv);
        if (colv && j >= 0 && j <= A.ny) {
            const int64_t o = (int64_t)j * P + col;
            vload<U, T, V>(u + o, r.u);
            vload<U, T, V>(u + o + CS, r.v);
            vload<T, T, V>(cl + o, r.l);
            vload<T, T, V>(cm + o, r.m);
            vload<T, T, V>(g0 + o, r.g0);
            vload<T, T, V>(g1 + o, r.g1);
            vload<T, T, V>(g2 + o, r.g2);
            vload<T, T, V>(g3 + o, r.g3);
        } else {
            vzero<T, V>(r.u);
            vzero<T, V>(r.v);
            vzero<T, V>(r.l);
            vzero<T, V>(r.m);
            vzero<T, V>(r.g0);
            vzero<T, V>(r.g1);
            vzero<T, V>(r.g2);
            vzero<T, V>(r.g3);
        }
    };
    // blocks and Q of a row entering the ring
    auto finish = [&](const CRaw<T, V>& r, CRow<T, V>& o) {
#pragma unroll
        for (int k = 0; k < V; ++k) {
            const T l = r.l[k], m = r.m[k], lm = l + m;
            const T A0 = r.g0[k], A1 = r.g1[k], B0 = r.g2[k], B1 = r.g3[k];
            const T AA = A0 * A0 + A1 * A1, BB = B0 * B0 + B1 * B1, AB = A0 * B0 + A1 * B1;
            o.u[k] = r.u[k];
            o.v[k] = r.v[k];
            o.qq0[k] = lm * A0 * A0 + m * AA;
            o.qq1[k] = lm * A0 * A1;
            o.qq2[k] = lm * A1 * A1 + m * AA;
            o.rr0[k] = lm * B0 * B0 + m * BB;
            o.rr1[k] = lm * B0 * B1;
            o.rr2[k] = lm * B1 * B1 + m * BB;
            o.qr0[k] = lm * A0 * B0 + m * AB;
            o.qr1[k] = l * A0 * B1 + m * B0 * A1;
            o.qr2[k] = l * A1 * B0 + m * B1 * A0;
            o.qr3[k] = lm * A1 * B1 + m * AB;
        }
        o.uL = lane_from_left(r.u[V - 1]);
        o.uR = lane_from_right(r.u[0]);
        o.vL = lane_from_left(r.v[V - 1]);
        o.vR = lane_from_right(r.v[0]);
#pragma unroll
        for (int k = 0; k < V; ++k) {
            const T du = at_right<T, V>(o.u, k, o.uR) - at_left<T, V>(o.u, k, o.uL);
            const T dv = at_right<T, V>(o.v, k, o.vR) - at_left<T, V>(o.v, k, o.vL);
            o.Q0[k] = o.qr0[k] * du + o.qr2[k] * dv;
            o.Q1[k] = o.qr1[k] * du + o.qr3[k] * dv;
        }
    };
    using Ctr = CCtr<T, V, COMP, FORCE, MODE>;
    auto load_ctr = [&](int jv, Ctr& c) {
        const int j = phys(jv);
        if (colv && j >= A.jlo && j <= A.jhi) {
            const int64_t o = (int64_t)j * P + col;
            vload<T, T, V>(ca + o, c.a);
            if constexpr (MODE == 0) {
                vload<T, T, V>(uprev + o, c.up);
                vload<T, T, V>(uprev + o + CS, c.vp);
                vload<double, double, V>(acc + o, c.hu);
                vload<double, double, V>(acc + o + CS, c.hv);
                if constexpr (COMP) {
                    vload<float, float, V>(acclo + o, c.lu);
                    vload<float, float, V>(acclo + o + CS, c.lv);
                }
            } else {
                if (xbase) {
                    vload<double, double, V>(xbase + o, c.hu);
                    vload<double, double, V>(xbase + o + CS, c.hv);
                } else {
                    vzero<double, V>(c.hu);
                    vzero<double, V>(c.hv);
                }
            }
            if constexpr (FORCE) {
                vload<T, T, V>(f + o, c.fu);
                vload<T, T, V>(f + o + CS, c.fv);
            }
        }
    };

    CRow<T, V> S, C, N;
    {
        CRaw<T, V> r;
        load_raw(j0 - 1, r);
        finish(r, S);
        load_raw(j0, r);
        finish(r, C);
    }
    CRaw<T, V> rawN;
    load_raw(j0 + 1, rawN);
    Ctr ctr;
    load_ctr(j0, ctr);

    for (int j = j0; j <= j1; ++j) {
        CRaw<T, V> rawNN;
        Ctr ctrN;
        if (j + 1 <= j1) {
            load_raw(j + 2, rawNN);
            load_ctr(j + 1, ctrN);
        }
        finish(rawN, N);
        // K^qq of the q neighbours and P = K^qr (U_N - U_S) (one-sided on a
        // free row), across the lane edges
        const int pj = phys(j);
        const int kind0 = (A.free_hi && pj == A.ny) ? 1 : ((A.free_lo && pj == 0) ? 2 : 0);
        const int kind = dir > 0 || kind0 == 0 ? kind0 : 3 - kind0;
        T P0[V], P1[V];
#pragma unroll
        for (int k = 0; k < V; ++k) {
            const T du = (kind == 1 ? C.u[k] : N.u[k]) - (kind == 2 ? C.u[k] : S.u[k]);
            const T dv = (kind == 1 ? C.v[k] : N.v[k]) - (kind == 2 ? C.v[k] : S.v[k]);
            P0[k] = C.qr0[k] * du + C.qr1[k] * dv;
            P1[k] = C.qr2[k] * du + C.qr3[k] * dv;
        }
        const T qq0L = lane_from_left(C.qq0[V - 1]), qq0R = lane_from_right(C.qq0[0]);
        const T qq1L = lane_from_left(C.qq1[V - 1]), qq1R = lane_from_right(C.qq1[0]);
        const T qq2L = lane_from_left(C.qq2[V - 1]), qq2R = lane_from_right(C.qq2[0]);
        const T P0L = lane_from_left(P0[V - 1]), P0R = lane_from_right(P0[0]);
        const T P1L = lane_from_left(P1[V - 1]), P1R = lane_from_right(P1[0]);
        const int64_t o = (int64_t)pj * P + col;

#pragma unroll
        for (int k = 0; k < V; ++k) {
            const int i = col + k;
            if (i < ilo || i > ihi || !colv) continue;
            const T uc = C.u[k], vc = C.v[k];
            const T ul = at_left<T, V>(C.u, k, C.uL), ur = at_right<T, V>(C.u, k, C.uR);
            const T vl = at_left<T, V>(C.v, k, C.vL), vr = at_right<T, V>(C.v, k, C.vR);
            // compact q term
            T kp0 = C.qq0[k] + at_right<T, V>(C.qq0, k, qq0R), km0 = C.qq0[k] + at_left<T, V>(C.qq0, k, qq0L);
            T kp1 = C.qq1[k] + at_right<T, V>(C.qq1, k, qq1R), km1 = C.qq1[k] + at_left<T, V>(C.qq1, k, qq1L);
            T kp2 = C.qq2[k] + at_right<T, V>(C.qq2, k, qq2R), km2 = C.qq2[k] + at_left<T, V>(C.qq2, k, qq2L);
            T dpu = ur - uc, dpv = vr - vc, dmu = uc - ul, dmv = vc - vl;
            T Lu = cqq2 * ((kp0 * dpu + kp1 * dpv) - (km0 * dmu + km1 * dmv));
            T Lv = cqq2 * ((kp1 * dpu + kp2 * dpv) - (km1 * dmu + km2 * dmv));
            // compact r term
            kp0 = C.rr0[k] + N.rr0[k];
            km0 = C.rr0[k] + S.rr0[k];
            kp1 = C.rr1[k] + N.rr1[k];
            km1 = C.rr1[k] + S.rr1[k];
            kp2 = C.rr2[k] + N.rr2[k];
            km2 = C.rr2[k] + S.rr2[k];
            dpu = N.u[k] - uc;
            dpv = N.v[k] - vc;
            dmu = uc - S.u[k];
            dmv = vc - S.v[k];
            const T dP0 = at_right<T, V>(P0, k, P0R) - at_left<T, V>(P0, k, P0L);
            const T dP1 = at_right<T, V>(P1, k, P1R) - at_left<T, V>(P1, k, P1L);
            if (kind == 0) {
                Lu += crr2 * ((kp0 * dpu + kp1 * dpv) - (km0 * dmu + km1 * dmv));
                Lv += crr2 * ((kp1 * dpu + kp2 * dpv) - (km1 * dmu + km2 * dmv));
                // cross terms D0q(K^qr D0r U) + D0r(K^rq D0q U)
                Lu += cqr * (dP0 + (N.Q0[k] - S.Q0[k]));
                Lv += cqr * (dP1 + (N.Q1[k] - S.Q1[k]));
            } else if (kind == 1) {
                Lu -= crrf * (km0 * dmu + km1 * dmv);
                Lv -= crrf * (km1 * dmu + km2 * dmv);
                Lu += cqrf * (dP0 - (C.Q0[k] + S.Q0[k]));
                Lv += cqrf * (dP1 - (C.Q1[k] + S.Q1[k]));
            } else {
                Lu += crrf * (kp0 * dpu + kp1 * dpv);
                Lv += crrf * (kp1 * dpu + kp2 * dpv);
                Lu += cqrf * (dP0 + (C.Q0[k] + N.Q0[k]));
                Lv += cqrf * (dP1 + (C.Q1[k] + N.Q1[k]));
            }
            if constexpr (FORCE) {
                const T fc = (T)A.fc;
                Lu -= fc * ctr.fu[k];
                Lv -= fc * ctr.fv[k];
            }
            const T a = ctr.a[k];
            T nu, nv;
            double hu = ctr.hu[k], hv = ctr.hv[k], lu = 0.0, lv = 0.0;
            if constexpr (MODE == 0) {
                nu = two * uc - ctr.up[k] + a * Lu;
                nv = two * vc - ctr.vp[k] + a * Lv;
                if constexpr (COMP) {
                    lu = ctr.lu[k];
                    lv = ctr.lv[k];
                }
            } else {
                const T ha = (T)0.5 * a;
                nu = uc + ha * Lu;
                nv = vc + ha * Lv;
                acc_add(hu, lu, A.w0 * (double)uc, COMP);
                acc_add(hv, lv, A.w0 * (double)vc, COMP);
                if (u0out) {
                    u0out[o + k] = uc;
                    u0out[o + k + CS] = vc;
                }
            }
            unext[o + k] = nu;
            unext[o + k + CS] = nv;
            acc_add(hu, lu, A.w * (double)nu, COMP);
            acc_add(hv, lv, A.w * (double)nv, COMP);
            if (COMP && A.final_) {
                acc[o + k] = hu + lu;
                acc[o + k + CS] = hv + lv;
            } else {
                acc[o + k] = hu;
                acc[o + k + CS] = hv;
                if constexpr (COMP) {
                    acclo[o + k] = (float)lu;
                    acclo[o + k + CS] = (float)lv;
                }
            }
        }
        S = C;
        C = N;
        if (j + 1 <= j1) {
            rawN = rawNN;
            ctr = ctrN;
        }
    }
}

struct Metric4 {
    const void *g0, *g1, *g2, *g3;
};

template <typename T, typename U, int V, int TY, int MODE, bool FORCE, bool COMP>
__global__ __launch_bounds__(64) void curv2d_kernel(const U* __restrict__ u, const T* uprev, T* unext,
                                                   const double* __restrict__ xbase, T* __restrict__ u0out,
                                                   double* __restrict__ acc, float* __restrict__ acclo,
                                                   const T* __restrict__ ca, const T* __restrict__ cl,
                                                   const T* __restrict__ cm, Metric4 g, const T* __restrict__ f,
                                                   Args2D A) {
    const int nbx = (A.nx - 1 + Cols<V>::W - 1) / Cols<V>::W;
    const int nby = (A.jhi - A.jlo + 1 + TY - 1) / TY;
    int t;
    if (!xcd_tile((int)blockIdx.x, nbx * nby, t)) return;
    curv2d_body<T, U, V, TY, MODE, FORCE, COMP>(
        t % nbx, t / nbx, u, uprev, unext, xbase, u0out, acc, acclo, ca, cl, cm,
        reinterpret_cast<const T*>(g.g0), reinterpret_cast<const T*>(g.g1), reinterpret_cast<const T*>(g.g2),
        reinterpret_cast<const T*>(g.g3), f, A);
}

template <typename T, typename U, int V, int TY, int MODE>
void curv_launch_t(bool force, bool comp, dim3 grid, hipStream_t s, const U* u, const T* uprev, T* unext,
                   const double* xbase, T* u0out, double* acc, float* acclo, const T* ca, const T* cl, const T* cm,
                   const Metric4& g, const T* f, const Args2D& A) {
#define ELWH_LC(F, CMP)                                                                                  \
    hipLaunchKernelGGL((curv2d_kernel<T, U, V, TY, MODE, F, CMP>), grid, dim3(64), 0, s, u, uprev, unext, \
                       xbase, u0out, acc, acclo, ca, cl, cm, g, f, A)
    if (force) {
        if (comp && sizeof(T) == 4) ELWH_LC(true, sizeof(T) == 4); else ELWH_LC(true, false);
    } else {
        if (comp && sizeof(T) == 4) ELWH_LC(false, sizeof(T) == 4); else ELWH_LC(false, false);
    }
#undef ELWH_LC
}

template <typename T, typename U, int MODE>
void curv_launch(int V, int TY, bool force, bool comp, int nx, int nrows, hipStream_t s, const U* u,
                 const T* uprev, T* unext, const double* xbase, T* u0out, double* acc, float* acclo, const T* ca,
                 const T* cl, const T* cm, const Metric4& g, const T* f, const Args2D& A) {
    auto grid_for = [&](int W, int ty) {
        return dim3((unsigned)xcd_grid(((nx - 1 + W - 1) / W) * ((nrows + ty - 1) / ty)), 1, 1);
    };
#define ELWH_CC(VV, TT)                                                                                     \
    if (V == VV && TY == TT) {                                                                              \
        curv_launch_t<T, U, VV, TT, MODE>(force, comp, grid_for(Cols<VV>::W, TT), s, u, uprev, unext, xbase, \
                                          u0out, acc, acclo, ca, cl, cm, g, f, A);                          \
        return;                                                                                             \
    }
    ELWH_CC(1, 8) ELWH_CC(1, 16) ELWH_CC(2, 8) ELWH_CC(2, 16)
#undef ELWH_CC
    curv_launch_t<T, U, 1, 8, MODE>(force, comp, grid_for(Cols<1>::W, 8), s, u, uprev, unext, xbase, u0out, acc,
                                    acclo, ca, cl, cm, g, f, A);
}

}  // namespace

Args2D make_args2d(const elwh_ctx* c);

bool tile_valid_curv(bool /*fp32*/, int V, int TY) { return (V == 1 || V == 2) && (TY == 8 || TY == 16); }

// One filter application on a mapped grid: the half step, then K N_T - 1
// single steps, u^{n+1} over u^{n-1} (FP64: u^0 is read from x itself, so
// the first full step writes a third state buffer).
void run_filter_curv2d(elwh_ctx* c, const double* x, bool with_force, bool amode, bool fp32, double* out) {
    hipStream_t s = c->stream;
    Args2D A = make_args2d(c);
    const int nrows = A.jhi - A.jlo + 1;
    const Tile t = fp32 ? c->tile32 : c->tile64;
    const int nsteps = c->plan.nt * c->opts.periods;
    const double sgn = amode ? -1.0 : 1.0;
    const bool comp = fp32 && c->opts.compensated;
    double* acc = out;
    float* lo = c->acc_lo;
    A.w0 = sgn * c->w[0];
    A.w = sgn * c->w[1];
    A.fc = c->cosn[0];
    prof_mark(c, 0);
    if (!fp32) {
        double *b1 = c->s64[1], *b2 = c->s64[2];
        const Metric4 g{c->cg[0], c->cg[1], c->cg[2], c->cg[3]};
        curv_launch<double, double, 1>(t.V, t.TY, with_force, false, A.nx, nrows, s, x, nullptr, b1,
                                       amode ? x : nullptr, nullptr, acc, lo, c->ca, c->cl, c->cm, g, c->f64, A);
        prof_mark(c, 1);
        // u^0 is the caller's x (read only): the first step writes b2, every
        // later one overwrites u^{n-1} in place
        const double* prev = x;
        double* cur = b1;
        for (int n = 1; n < nsteps; ++n) {
            double* nxt = prev == x ? b2 : const_cast<double*>(prev);
            A.w = sgn * c->w[n + 1];
            A.fc = c->cosn[n];
            A.final_ = (n == nsteps - 1);
            curv_launch<double, double, 0>(t.V, t.TY, with_force, false, A.nx, nrows, s, cur, prev, nxt, nullptr,
                                           nullptr, acc, lo, c->ca, c->cl, c->cm, g, c->f64, A);
            prev = cur;
            cur = nxt;
        }
    } else {
        float *b0 = c->s32[0], *b1 = c->s32[1];
        const Metric4 g{c->fg[0], c->fg[1], c->fg[2], c->fg[3]};
        curv_launch<float, double, 1>(t.V, t.TY, with_force, comp, A.nx, nrows, s, x, nullptr, b1,
                                      amode ? x : nullptr, b0, acc, lo, c->fa, c->fl, c->fm, g, c->f32, A);
        prof_mark(c, 1);
        float* prev = b0;
        float* cur = b1;
        for (int n = 1; n < nsteps; ++n) {
            A.w = sgn * c->w[n + 1];
            A.fc = c->cosn[n];
            A.final_ = (n == nsteps - 1);
            // u^{n+1} overwrites u^{n-1} in place
            curv_launch<float, float, 0>(t.V, t.TY, with_force, comp, A.nx, nrows, s, cur, prev, prev, nullptr,
                                         nullptr, acc, lo, c->fa, c->fl, c->fm, g, c->f32, A);
            float* tmp = prev;
            prev = cur;
            cur = tmp;
        }
    }
    prof_mark(c, 2, nsteps - 1);
}

}  // namespace elwh
