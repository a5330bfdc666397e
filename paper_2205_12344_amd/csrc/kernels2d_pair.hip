// 2-D fused El-WaveHoltz step pair for gfx950: two time steps per launch.
//
// One launch advances every unknown node from (u^n, u^{n-1}) to
// (u^{n+2}, u^{n+1}) with the corrected leapfrog (Sec. 4.3, eq.
// elastic-time-explicit-corrected) and adds w_{n+1} u^{n+1} + w_{n+2} u^{n+2}
// into the filter accumulator (trapezoid rule of eq. el_WHI_OP), so state,
// coefficients and accumulator cross HBM once per two steps instead of once
// per step: per unknown node and FP64 step pair, 120 B (read u^n, u^{n-1},
// a, lambda, mu, acc; write u^{n+1}, u^{n+2}, acc) against 2 x 104 B for two
// single-step launches.
//
// Mapping.  As the single-step kernel (one 64-lane wavefront per block, V
// nodes per lane, rows marched upwards with the stencil rows in registers and
// DPP for the x neighbours), with a two-stage pipeline along the march:
//   stage 1 at row r computes u^{n+1}(r) from u^n rows r-1..r+1,
//   stage 2 at row r-1 computes u^{n+2}(r-1) from the u^{n+1} rows r-2..r
//   that stage 1 left in registers.
// u^{n+1} is needed one node beyond the block on every side, so each
// wavefront loads two halo columns per side (W = 64 V - 2H computed columns,
// H = 2, or 4 for V = 4 to keep vector loads aligned) and stage 1 runs over
// the rows j0-1 .. j1+1 (computed twice at block edges, written once).
// u^{n+1} and u^{n+2} go to two buffers other than the inputs: a node's
// u^{n-1} is read by the blocks on both sides of it, so it cannot be
// overwritten in place within the launch.
#include "step2d_common.h"

namespace elwh {

template <int V>
struct PairCols {
    static constexpr int H = V == 4 ? 4 : 2;            // halo columns per side
    static constexpr int W = 64 * V - 2 * H;            // computed columns per wavefront
};

// Centre-row loads of stage 1 (row r): a, u^{n-1}, forcing.
template <typename T, int V, bool FORCE>
struct Ctr1 {
    T a[V];
    T up[V], vp[V];
    T fu[V], fv[V];
};

// Accumulator of stage 2 (row r-1).
template <int V, bool COMP>
struct AccRow {
    double hu[V], hv[V];
    double lu[V], lv[V];
};

// u^{n+1} row with x neighbours of the end nodes.
template <typename T, int V>
struct Half {
    T u[V], v[V];
    T uL, uR, vL, vR;
};

template <typename T, int V>
__device__ __forceinline__ Nb<T> node_mix(const Half<T, V>& h, const T (&l)[V], const T (&m)[V], int k) {
    Nb<T> n;
    n.u = h.u[k];
    n.v = h.v[k];
    n.uL = k > 0 ? h.u[k > 0 ? k - 1 : 0] : h.uL;
    n.uR = k < V - 1 ? h.u[k < V - 1 ? k + 1 : 0] : h.uR;
    n.vL = k > 0 ? h.v[k > 0 ? k - 1 : 0] : h.vL;
    n.vR = k < V - 1 ? h.v[k < V - 1 ? k + 1 : 0] : h.vR;
    n.l = l[k];
    n.m = m[k];
    return n;
}

template <typename T, int V, int TY, bool FORCE, bool COMP>
__device__ __forceinline__ void pair2d_body(int bx, int by, const T* __restrict__ u, const T* __restrict__ uprev,
                                            T* __restrict__ u1out, T* __restrict__ u2out,
                                            double* __restrict__ acc, double* __restrict__ acclo,
                                            const T* __restrict__ ca, const T* __restrict__ cl,
                                            const T* __restrict__ cm, const T* __restrict__ f, const Args2D& A) {
    constexpr int W = PairCols<V>::W, H = PairCols<V>::H;
    const int lane = threadIdx.x;
    const int own0 = W * bx;                      // first owned column of this wavefront
    const int c0 = own0 - H;                      // first loaded column
    const int col = c0 + V * lane;                // first column of this lane
    const bool colv = col >= 0 && col <= A.nx;    // vector lies in the padded row
    const int j0 = A.jlo + by * TY;
    if (j0 > A.jhi) return;
    const int j1 = min(j0 + TY - 1, A.jhi);
    const int P = (int)A.P;
    const int64_t CS = A.CS;
    const T cxx2 = (T)A.cxx2, cyy2 = (T)A.cyy2, cxy = (T)A.cxy, cyyf = (T)A.cyyf, cfx = (T)A.cfx;
    const T two = (T)2;
    // stage 1 covers the owned columns and one more on each side; stage 2 the owned ones
    const int i1lo = max(own0 - 1, 1), i1hi = min(own0 + W, A.nx - 1);
    const int i2lo = max(own0, 1), i2hi = min(own0 + W - 1, A.nx - 1);

    auto load_raw = [&](int j, RawRow<T, V>& r) {
        if (colv && j >= 0 && j <= A.ny) {
            const int64_t o = (int64_t)j * P + col;
            vload<T, T, V>(u + o, r.u);
            vload<T, T, V>(u + o + CS, r.v);
            vload<T, T, V>(cl + o, r.l);
            vload<T, T, V>(cm + o, r.m);
        } else {
            vzero<T, V>(r.u);
            vzero<T, V>(r.v);
            vzero<T, V>(r.l);
            vzero<T, V>(r.m);
        }
    };
    auto finish = [&](const RawRow<T, V>& r, Row<T, V>& o) {
#pragma unroll
        for (int k = 0; k < V; ++k) {
            o.u[k] = r.u[k];
            o.v[k] = r.v[k];
            o.l[k] = r.l[k];
            o.m[k] = r.m[k];
        }
        o.uL = lane_from_left(r.u[V - 1]);
        o.uR = lane_from_right(r.u[0]);
        o.vL = lane_from_left(r.v[V - 1]);
        o.vR = lane_from_right(r.v[0]);
    };
    using C1 = Ctr1<T, V, FORCE>;
    auto load_c1 = [&](int j, C1& c) {
        if (colv && j >= A.jlo && j <= A.jhi) {
            const int64_t o = (int64_t)j * P + col;
            vload<T, T, V>(ca + o, c.a);
            vload<T, T, V>(uprev + o, c.up);
            vload<T, T, V>(uprev + o + CS, c.vp);
            if constexpr (FORCE) {
                vload<T, T, V>(f + o, c.fu);
                vload<T, T, V>(f + o + CS, c.fv);
            }
        } else {
            vzero<T, V>(c.a);
            vzero<T, V>(c.up);
            vzero<T, V>(c.vp);
            if constexpr (FORCE) {
                vzero<T, V>(c.fu);
                vzero<T, V>(c.fv);
            }
        }
    };
    using AR = AccRow<V, COMP>;
    auto load_acc = [&](int j, AR& a) {
        if (colv && j >= j0 && j <= j1) {
            const int64_t o = (int64_t)j * P + col;
            vload<double, double, V>(acc + o, a.hu);
            vload<double, double, V>(acc + o + CS, a.hv);
            if constexpr (COMP) {
                vload<double, double, V>(acclo + o, a.lu);
                vload<double, double, V>(acclo + o + CS, a.lv);
            }
        }
    };
    auto kind_of = [&](int j) { return (A.free_hi && j == A.ny) ? 1 : ((A.free_lo && j == 0) ? 2 : 0); };

    // u^n ring: O (coefficients only) = r-2, S = r-1, C = r, N = r+1
    Row<T, V> S, C, N;
    T Ol[V], Om[V];
    vzero<T, V>(Ol);
    vzero<T, V>(Om);
    {
        RawRow<T, V> r;
        load_raw(j0 - 2, r);
        finish(r, S);
        load_raw(j0 - 1, r);
        finish(r, C);
    }
    RawRow<T, V> rawN;
    load_raw(j0, rawN);
    C1 c1;
    load_c1(j0 - 1, c1);
    // stage-2 operands carried from the previous row: a and forcing of row r-1
    T aq[V], fuq[V], fvq[V];
    vzero<T, V>(aq);
    vzero<T, V>(fuq);
    vzero<T, V>(fvq);
    AR accq;
    // u^{n+1} ring: P0 = r-2, P1 = r-1, P2 = r
    Half<T, V> P0, P1, P2;
    vzero<T, V>(P1.u);
    vzero<T, V>(P1.v);
    P1.uL = P1.uR = P1.vL = P1.vR = (T)0;

    for (int r = j0 - 1; r <= j1 + 1; ++r) {
        RawRow<T, V> rawNN;
        C1 c1N;
        AR accN;
        if (r + 1 <= j1 + 1) {
            load_raw(r + 2, rawNN);
            load_c1(r + 1, c1N);
            load_acc(r, accN);
        }
        finish(rawN, N);

        // ---- stage 1: u^{n+1}(r) ----------------------------------------
        const bool row1 = r >= A.jlo && r <= A.jhi;
        const int kind1 = kind_of(r);
        const T lamL0 = lane_from_left(C.l[V - 1]), lamR0 = lane_from_right(C.l[0]);
        const T muL0 = lane_from_left(C.m[V - 1]), muR0 = lane_from_right(C.m[0]);
        const int64_t o1 = (int64_t)r * P + col;
        const bool own1 = r >= j0 && r <= j1;
#pragma unroll
        for (int k = 0; k < V; ++k) {
            const int i = col + k;
            T nu = (T)0, nv = (T)0;
            if (row1 && colv && i >= i1lo && i <= i1hi) {
                const Nb<T> s = node_of<T, V>(S, k), cc = node_of<T, V>(C, k), nn = node_of<T, V>(N, k);
                const T lamL = k > 0 ? C.l[k > 0 ? k - 1 : 0] : lamL0;
                const T lamR = k < V - 1 ? C.l[k < V - 1 ? k + 1 : 0] : lamR0;
                const T muL = k > 0 ? C.m[k > 0 ? k - 1 : 0] : muL0;
                const T muR = k < V - 1 ? C.m[k < V - 1 ? k + 1 : 0] : muR0;
                T Lu, Lv;
                stencil2d<T>(kind1, s, cc, nn, lamL, lamR, muL, muR, cxx2, cyy2, cxy, cyyf, cfx, Lu, Lv);
                if constexpr (FORCE) {
                    const T fc = (T)A.fc;
                    Lu -= fc * c1.fu[k];
                    Lv -= fc * c1.fv[k];
                }
                nu = two * cc.u - c1.up[k] + c1.a[k] * Lu;
                nv = two * cc.v - c1.vp[k] + c1.a[k] * Lv;
                if (own1 && i >= i2lo && i <= i2hi) {
                    u1out[o1 + k] = nu;
                    u1out[o1 + k + CS] = nv;
                }
            }
            P2.u[k] = nu;
            P2.v[k] = nv;
        }
        P2.uL = lane_from_left(P2.u[V - 1]);
        P2.uR = lane_from_right(P2.u[0]);
        P2.vL = lane_from_left(P2.v[V - 1]);
        P2.vR = lane_from_right(P2.v[0]);

        // ---- stage 2: u^{n+2}(r-1) and the accumulator ------------------
        const int q = r - 1;
        if (q >= j0) {
            const int kind2 = kind_of(q);
            // centre-row coefficients of row q are those of S
            const T lamL0q = lane_from_left(S.l[V - 1]), lamR0q = lane_from_right(S.l[0]);
            const T muL0q = lane_from_left(S.m[V - 1]), muR0q = lane_from_right(S.m[0]);
            const int64_t o2 = (int64_t)q * P + col;
#pragma unroll
            for (int k = 0; k < V; ++k) {
                const int i = col + k;
                if (!colv || i < i2lo || i > i2hi) continue;
                const Nb<T> s = node_mix<T, V>(P0, Ol, Om, k), cc = node_mix<T, V>(P1, S.l, S.m, k),
                            nn = node_mix<T, V>(P2, C.l, C.m, k);
                const T lamL = k > 0 ? S.l[k > 0 ? k - 1 : 0] : lamL0q;
                const T lamR = k < V - 1 ? S.l[k < V - 1 ? k + 1 : 0] : lamR0q;
                const T muL = k > 0 ? S.m[k > 0 ? k - 1 : 0] : muL0q;
                const T muR = k < V - 1 ? S.m[k < V - 1 ? k + 1 : 0] : muR0q;
                T Lu, Lv;
                stencil2d<T>(kind2, s, cc, nn, lamL, lamR, muL, muR, cxx2, cyy2, cxy, cyyf, cfx, Lu, Lv);
                if constexpr (FORCE) {
                    const T fc = (T)A.fc2;
                    Lu -= fc * fuq[k];
                    Lv -= fc * fvq[k];
                }
                // u^n(q) is the centre value of S
                const T nu = two * cc.u - S.u[k] + aq[k] * Lu;
                const T nv = two * cc.v - S.v[k] + aq[k] * Lv;
                u2out[o2 + k] = nu;
                u2out[o2 + k + CS] = nv;
                double hu = accq.hu[k], hv = accq.hv[k], lu = 0.0, lv = 0.0;
                if constexpr (COMP) {
                    lu = accq.lu[k];
                    lv = accq.lv[k];
                }
                acc_add(hu, lu, A.w * (double)cc.u, COMP);
                acc_add(hv, lv, A.w * (double)cc.v, COMP);
                acc_add(hu, lu, A.w2 * (double)nu, COMP);
                acc_add(hv, lv, A.w2 * (double)nv, COMP);
                if (COMP && A.final_) {
                    acc[o2 + k] = hu + lu;
                    acc[o2 + k + CS] = hv + lv;
                } else {
                    acc[o2 + k] = hu;
                    acc[o2 + k + CS] = hv;
                    if constexpr (COMP) {
                        acclo[o2 + k] = lu;
                        acclo[o2 + k + CS] = lv;
                    }
                }
            }
        }

        // ---- roll -------------------------------------------------------
#pragma unroll
        for (int k = 0; k < V; ++k) {
            Ol[k] = S.l[k];
            Om[k] = S.m[k];
            aq[k] = c1.a[k];
            if constexpr (FORCE) {
                fuq[k] = c1.fu[k];
                fvq[k] = c1.fv[k];
            }
        }
        S = C;
        C = N;
        P0 = P1;
        P1 = P2;
        if (r + 1 <= j1 + 1) {
            rawN = rawNN;
            c1 = c1N;
            accq = accN;
        }
    }
}

template <typename T, int V, int TY, bool FORCE, bool COMP>
__global__ __launch_bounds__(64) void pair2d_kernel(const T* __restrict__ u, const T* __restrict__ uprev,
                                                   T* __restrict__ u1out, T* __restrict__ u2out,
                                                   double* __restrict__ acc, double* __restrict__ acclo,
                                                   const T* __restrict__ ca, const T* __restrict__ cl,
                                                   const T* __restrict__ cm, const T* __restrict__ f, Args2D A) {
    constexpr int W = PairCols<V>::W;
    const int nbx = (A.nx - 1 + W) / W;
    const int nby = (A.jhi - A.jlo + 1 + TY - 1) / TY;
    int t;
    if (!xcd_tile((int)blockIdx.x, nbx * nby, t)) return;
    pair2d_body<T, V, TY, FORCE, COMP>(t % nbx, t / nbx, u, uprev, u1out, u2out, acc, acclo, ca, cl,
                                       cm, f, A);
}

template <typename T, int V, int TY>
static void pair_launch_t(bool force, bool comp, hipStream_t s, int nrows, const T* u, const T* uprev, T* u1out,
                          T* u2out, double* acc, double* acclo, const T* ca, const T* cl, const T* cm, const T* f,
                          const Args2D& A) {
    constexpr int W = PairCols<V>::W;
    const dim3 grid((unsigned)xcd_grid(((A.nx - 1 + W) / W) * ((nrows + TY - 1) / TY)), 1, 1);
#define ELWH_LP(F, CMP)                                                                                        \
    hipLaunchKernelGGL((pair2d_kernel<T, V, TY, F, CMP>), grid, dim3(64), 0, s, u, uprev, u1out, u2out, acc, \
                       acclo, ca, cl, cm, f, A)
    if (force) {
        if (comp) ELWH_LP(true, true); else ELWH_LP(true, false);
    } else {
        if (comp) ELWH_LP(false, true); else ELWH_LP(false, false);
    }
#undef ELWH_LP
}

bool pair_tile_valid_2d(bool fp32, int V, int TY) {
    const bool v_ok = V == 1 || V == 2 || (fp32 && V == 4);
    return v_ok && (TY == 4 || TY == 8 || TY == 16);
}

template <typename T>
void launch_pair2d(int V, int TY, bool force, bool comp, hipStream_t s, int nrows, const T* u, const T* uprev,
                   T* u1out, T* u2out, double* acc, double* acclo, const T* ca, const T* cl, const T* cm,
                   const T* f, const Args2D& A) {
#define ELWH_PC(VV, TT)                                                                                          \
    if (V == VV && TY == TT) {                                                                                   \
        pair_launch_t<T, VV, TT>(force, comp, s, nrows, u, uprev, u1out, u2out, acc, acclo, ca, cl, cm, f, A); \
        return;                                                                                                  \
    }
    ELWH_PC(1, 4) ELWH_PC(1, 8) ELWH_PC(1, 16)
    ELWH_PC(2, 4) ELWH_PC(2, 8) ELWH_PC(2, 16)
    if constexpr (sizeof(T) == 4) {
        ELWH_PC(4, 4) ELWH_PC(4, 8) ELWH_PC(4, 16)
    }
#undef ELWH_PC
    pair_launch_t<T, 1, 8>(force, comp, s, nrows, u, uprev, u1out, u2out, acc, acclo, ca, cl, cm, f, A);
}

template void launch_pair2d<double>(int, int, bool, bool, hipStream_t, int, const double*, const double*, double*,
                                    double*, double*, double*, const double*, const double*, const double*,
                                    const double*, const Args2D&);
template void launch_pair2d<float>(int, int, bool, bool, hipStream_t, int, const float*, const float*, float*,
                                   float*, double*, double*, const float*, const float*, const float*, const float*,
                                   const Args2D&);

}  // namespace elwh
