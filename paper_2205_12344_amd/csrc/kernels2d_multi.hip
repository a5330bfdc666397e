// 2-D fused El-WaveHoltz multi-step kernel for gfx950: K = 2, 3 or 4 time
// steps per launch (temporal blocking in registers).
//
// One launch advances every unknown node from (u^n, u^{n-1}) to
// (u^{n+K}, u^{n+K-1}) with the corrected leapfrog (Sec. 4.3, eq.
// elastic-time-explicit-corrected) and adds sum_{s=1..K} w_{n+s} u^{n+s}
// into the filter accumulator (trapezoid rule of eq. el_WHI_OP).  State,
// coefficients and accumulator cross HBM once per K steps: per unknown node
// and FP64 launch 120 B (read u^n, u^{n-1}, a, lambda, mu, acc; write
// u^{n+K-1}, u^{n+K}, acc), i.e. 120/K B per lattice update against 104 B
// for single-step launches.  The levels u^{n+1} .. u^{n+K-2} never leave
// registers.
//
// Mapping.  As the single-step kernel (one 64-lane wavefront per block, V
// nodes per lane, rows marched with the stencil rows in registers and DPP for
// the x neighbours; odd row chunks march downwards, see below), with a
// K-stage pipeline along the march: at row
// iteration r, stage s computes u^{n+s} at row r-s+1 from the three rows of
// u^{n+s-1} that stage s-1 has left in registers (stage 1 from u^n).  Level
// s is needed K-s nodes beyond the block on every side, so each wavefront
// loads H >= K halo columns per side (W = 64 V - 2H computed columns; H a
// multiple of V keeps vector loads aligned) and stage s runs over the rows
// j0-(K-s) .. j1+(K-s) (recomputed by neighbouring blocks, written once).
// Each row's accumulator is read when stage 1 reaches it and written after
// stage K has added its term, so the accumulation order per node is that of
// K single steps.  The two output levels go to buffers other than the inputs:
// a node's u^{n-1} and u^n are read by the blocks on both sides of it.
#include <type_traits>

#include "step2d_common.h"

namespace elwh {

template <int V, int K>
struct MultiCols {
    static constexpr int H = ((K + V - 1) / V) * V;     // halo columns per side
    static constexpr int W = 64 * V - 2 * H;            // computed columns per wavefront
};

// Centre-row loads of stage 1 (row r): a, u^{n-1}, forcing.
template <typename T, int V>
struct Ctr1 {
    T a[V];
    T up[V], vp[V];
    T fu[V], fv[V];
};

// One row of a computed level, with the x neighbours of the end nodes.
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

template <typename T, int V>
__device__ __forceinline__ Half<T, V> half_of(const Row<T, V>& r) {
    Half<T, V> h;
#pragma unroll
    for (int k = 0; k < V; ++k) {
        h.u[k] = r.u[k];
        h.v[k] = r.v[k];
    }
    h.uL = r.uL;
    h.uR = r.uR;
    h.vL = r.vL;
    h.vR = r.vR;
    return h;
}

template <typename T, int V, int TY, int K, bool FORCE, bool COMP>
__device__ __forceinline__ void multi2d_body(int bx, int by, const T* __restrict__ u, const T* __restrict__ uprev,
                                             T* __restrict__ outA, T* __restrict__ outB,
                                             double* __restrict__ acc, float* __restrict__ acclo,
                                             const T* __restrict__ ca, const T* __restrict__ cl,
                                             const T* __restrict__ cm, const T* __restrict__ f, const Args2D& A) {
    constexpr int W = MultiCols<V, K>::W, H = MultiCols<V, K>::H;
    const int lane = threadIdx.x;
    const int own0 = W * bx;                      // first owned column of this wavefront
    const int col = own0 - H + V * lane;          // first column of this lane
    const bool colv = col >= 0 && col <= A.nx;    // vector lies in the padded row
    const int j0 = A.jlo + by * TY;
    if (j0 > A.jhi) return;
    const int j1 = min(j0 + TY - 1, A.jhi);
    const int P = (int)A.P;
    const int64_t CS = A.CS;
    // Mirrored march (K = 2).  Odd row chunks march downwards, so that two
    // neighbouring chunks read the halo rows they share at the same time
    // (both at the start or both at the end of their marches) and the second
    // read finds them in L2.  The march below runs over virtual rows v in
    // [j0 - K + 1, j1 + K - 1]; row v is physical row jb + dir * v.  Mirrored
    // about the chunk, the stencil of a node keeps its form with the roles of
    // the rows below and above exchanged, which is the same stencil with the
    // mixed-derivative coefficients negated and a traction-free top row taken
    // as a free bottom row (and the reverse).  (For K = 3, 4, which are bound
    // by instruction issue, the mirrored march measured 4 % slower.)
    const int dir = (K == 2 && (by & 1)) ? -1 : 1;
    const int jb = dir > 0 ? 0 : j0 + j1;
    auto phys = [&](int v) { return jb + dir * v; };
    const T cxx2 = (T)A.cxx2, cyy2 = (T)A.cyy2, cxy = (T)(dir * A.cxy), cyyf = (T)A.cyyf, cfx = (T)(dir * A.cfx);
    const T two = (T)2;
    const int olo = max(own0, 1), ohi = min(own0 + W - 1, A.nx - 1);   // owned columns

    auto load_raw = [&](int jv, RawRow<T, V>& r) {
        const int j = phys(jv);
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
    auto load_c1 = [&](int jv, Ctr1<T, V>& c) {
        const int j = phys(jv);
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
    // (the FP32 compensation words are widened when the row enters the
    // pipeline, not at the load, which would wait for it there)
    auto load_acc = [&](int jv, double (&hu)[V], double (&hv)[V], float (&lu)[V], float (&lv)[V]) {
        if (colv && jv >= j0 && jv <= j1) {
            const int64_t o = (int64_t)phys(jv) * P + col;
            vload<double, double, V>(acc + o, hu);
            vload<double, double, V>(acc + o + CS, hv);
            if constexpr (COMP) {
                vload<float, float, V>(acclo + o, lu);
                vload<float, float, V>(acclo + o + CS, lv);
            }
        }
    };
    // stencil kind of virtual row v: 1 a traction-free row whose neighbour
    // is the row before it in the march, 2 one whose neighbour is the row after
    auto kind_of = [&](int v) {
        const int j = phys(v);
        const int k = (A.free_hi && j == A.ny) ? 1 : ((A.free_lo && j == 0) ? 2 : 0);
        return dir > 0 || k == 0 ? k : 3 - k;
    };

    const int r0 = j0 - K + 1, r1 = j1 + K - 1;
    // u^n rows r-1 (S), r (C), r+1 (N), with lambda, mu; older coefficient
    // rows r-2-e in Ol[e], Om[e]
    Row<T, V> S, C, N;
    T Ol[K - 1][V], Om[K - 1][V];
#pragma unroll
    for (int e = 0; e < K - 1; ++e) {
        vzero<T, V>(Ol[e]);
        vzero<T, V>(Om[e]);
    }
    {
        RawRow<T, V> r;
        load_raw(r0 - 1, r);
        finish(r, S);
        load_raw(r0, r);
        finish(r, C);
    }
    RawRow<T, V> rawN;
    load_raw(r0 + 1, rawN);
    Ctr1<T, V> c1;
    load_c1(r0, c1);
    // a and forcing of rows r-d, d = 0..K-1 (the row of stage d+1)
    T ar[K][V], fur[K][V], fvr[K][V];
    // accumulator of rows r-d
    double ahu[K][V], ahv[K][V], alu[K][V], alv[K][V];
#pragma unroll
    for (int d = 0; d < K; ++d) {
        vzero<T, V>(ar[d]);
        vzero<T, V>(fur[d]);
        vzero<T, V>(fvr[d]);
        vzero<double, V>(ahu[d]);
        vzero<double, V>(ahv[d]);
        vzero<double, V>(alu[d]);
        vzero<double, V>(alv[d]);
    }
    {
        float l0u[V], l0v[V];
        vzero<float, V>(l0u);
        vzero<float, V>(l0v);
        load_acc(r0, ahu[0], ahv[0], l0u, l0v);
#pragma unroll
        for (int k = 0; k < V; ++k) {
            alu[0][k] = l0u[k];
            alv[0][k] = l0v[k];
        }
    }
    // computed levels 1..K-1: rows (q-2, q-1, q) of the last stage-s row q
    Half<T, V> L[K - 1][3];
#pragma unroll
    for (int s = 0; s < K - 1; ++s)
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            vzero<T, V>(L[s][e].u);
            vzero<T, V>(L[s][e].v);
            L[s][e].uL = L[s][e].uR = L[s][e].vL = L[s][e].vR = (T)0;
        }

    for (int r = r0; r <= r1; ++r) {
        RawRow<T, V> rawNN;
        Ctr1<T, V> c1N;
        double nhu[V], nhv[V];
        float nlu[V], nlv[V];
        vzero<double, V>(nhu);
        vzero<double, V>(nhv);
        vzero<float, V>(nlu);
        vzero<float, V>(nlv);
        if (r < r1) {
            load_raw(r + 2, rawNN);
            load_c1(r + 1, c1N);
            load_acc(r + 1, nhu, nhv, nlu, nlv);
        }
        finish(rawN, N);
#pragma unroll
        for (int k = 0; k < V; ++k) {
            ar[0][k] = c1.a[k];
            if constexpr (FORCE) {
                fur[0][k] = c1.fu[k];
                fvr[0][k] = c1.fv[k];
            }
        }

        auto stage = [&](auto sc) {
            constexpr int s = decltype(sc)::value;
            const int q = r - s + 1;                          // (virtual) row of stage s
            const int pq = phys(q);
            // level s is needed on rows j0-(K-s) .. j1+(K-s); zero on boundary rows
            const bool rowv = q >= j0 - (K - s) && pq >= A.jlo && pq <= A.jhi;
            const bool own = q >= j0 && q <= j1;
            const int ilo = max(own0 - (K - s), 1), ihi = min(own0 + W - 1 + (K - s), A.nx - 1);
            // coefficient rows q-1, q, q+1; row r-d is N (d = -1), C (0), S (1), Ol[d-2] (d >= 2)
            T lSc[V], mSc[V], lCc[V], mCc[V], lNc[V], mNc[V];
#pragma unroll
            for (int k = 0; k < V; ++k) {
                if constexpr (s == 1) {
                    lSc[k] = S.l[k]; mSc[k] = S.m[k];
                    lCc[k] = C.l[k]; mCc[k] = C.m[k];
                    lNc[k] = N.l[k]; mNc[k] = N.m[k];
                } else if constexpr (s == 2) {
                    lSc[k] = Ol[0][k]; mSc[k] = Om[0][k];
                    lCc[k] = S.l[k]; mCc[k] = S.m[k];
                    lNc[k] = C.l[k]; mNc[k] = C.m[k];
                } else if constexpr (s == 3) {
                    lSc[k] = Ol[1][k]; mSc[k] = Om[1][k];
                    lCc[k] = Ol[0][k]; mCc[k] = Om[0][k];
                    lNc[k] = S.l[k]; mNc[k] = S.m[k];
                } else {
                    lSc[k] = Ol[s - 2][k]; mSc[k] = Om[s - 2][k];
                    lCc[k] = Ol[s - 3][k]; mCc[k] = Om[s - 3][k];
                    lNc[k] = Ol[s - 4][k]; mNc[k] = Om[s - 4][k];
                }
            }
            const T lamL0 = lane_from_left(lCc[V - 1]), lamR0 = lane_from_right(lCc[0]);
            const T muL0 = lane_from_left(mCc[V - 1]), muR0 = lane_from_right(mCc[0]);
            // the level below: rows q-1, q, q+1 of u^{n+s-1}
            Half<T, V> lo, ce, hi;
            if constexpr (s == 1) {
                lo = half_of<T, V>(S);
                ce = half_of<T, V>(C);
                hi = half_of<T, V>(N);
            } else {
                lo = L[s - 2][0];
                ce = L[s - 2][1];
                hi = L[s - 2][2];
            }
            const int kind = kind_of(q);
            const double wgt = A.wk[s - 1];
            const T fcs = (T)A.fck[s - 1];
            const int64_t o = (int64_t)pq * P + col;
            Half<T, V> nw;
#pragma unroll
            for (int k = 0; k < V; ++k) {
                const int i = col + k;
                T nu = (T)0, nv = (T)0;
                if (rowv && colv && i >= ilo && i <= ihi) {
                    const Nb<T> sn = node_mix<T, V>(lo, lSc, mSc, k), cc = node_mix<T, V>(ce, lCc, mCc, k),
                                nn = node_mix<T, V>(hi, lNc, mNc, k);
                    const T lamL = k > 0 ? lCc[k > 0 ? k - 1 : 0] : lamL0;
                    const T lamR = k < V - 1 ? lCc[k < V - 1 ? k + 1 : 0] : lamR0;
                    const T muL = k > 0 ? mCc[k > 0 ? k - 1 : 0] : muL0;
                    const T muR = k < V - 1 ? mCc[k < V - 1 ? k + 1 : 0] : muR0;
                    T Lu, Lv;
                    stencil2d<T>(kind, sn, cc, nn, lamL, lamR, muL, muR, cxx2, cyy2, cxy, cyyf, cfx, Lu, Lv);
                    if constexpr (FORCE) {
                        Lu -= fcs * fur[s - 1][k];
                        Lv -= fcs * fvr[s - 1][k];
                    }
                    // u^{n+s-2} at row q: u^{n-1} for stage 1, u^n (S) for stage 2,
                    // the oldest row of level s-2 beyond
                    T pu, pv;
                    if constexpr (s == 1) {
                        pu = c1.up[k];
                        pv = c1.vp[k];
                    } else if constexpr (s == 2) {
                        pu = S.u[k];
                        pv = S.v[k];
                    } else {
                        pu = L[s - 3][0].u[k];
                        pv = L[s - 3][0].v[k];
                    }
                    const T a = ar[s - 1][k];
                    nu = two * cc.u - pu + a * Lu;
                    nv = two * cc.v - pv + a * Lv;
                    if (own && i >= olo && i <= ohi) {
                        acc_add(ahu[s - 1][k], alu[s - 1][k], wgt * (double)nu, COMP);
                        acc_add(ahv[s - 1][k], alv[s - 1][k], wgt * (double)nv, COMP);
                        if constexpr (s == K - 1) {
                            outA[o + k] = nu;
                            outA[o + k + CS] = nv;
                        } else if constexpr (s == K) {
                            outB[o + k] = nu;
                            outB[o + k + CS] = nv;
                            if (COMP && A.final_) {
                                acc[o + k] = ahu[s - 1][k] + alu[s - 1][k];
                                acc[o + k + CS] = ahv[s - 1][k] + alv[s - 1][k];
                            } else {
                                acc[o + k] = ahu[s - 1][k];
                                acc[o + k + CS] = ahv[s - 1][k];
                                if constexpr (COMP) {
                                    acclo[o + k] = (float)alu[s - 1][k];
                                    acclo[o + k + CS] = (float)alv[s - 1][k];
                                }
                            }
                        }
                    }
                }
                nw.u[k] = nu;
                nw.v[k] = nv;
            }
            if constexpr (s < K) {
                nw.uL = lane_from_left(nw.u[V - 1]);
                nw.uR = lane_from_right(nw.u[0]);
                nw.vL = lane_from_left(nw.v[V - 1]);
                nw.vR = lane_from_right(nw.v[0]);
                L[s - 1][0] = L[s - 1][1];
                L[s - 1][1] = L[s - 1][2];
                L[s - 1][2] = nw;
            }
        };
        stage(std::integral_constant<int, 1>{});
        stage(std::integral_constant<int, 2>{});
        if constexpr (K >= 3) stage(std::integral_constant<int, (K >= 3 ? 3 : 1)>{});
        if constexpr (K >= 4) stage(std::integral_constant<int, (K >= 4 ? 4 : 1)>{});

        // ---- roll -------------------------------------------------------
#pragma unroll
        for (int e = K - 2; e > 0; --e)
#pragma unroll
            for (int k = 0; k < V; ++k) {
                Ol[e][k] = Ol[e - 1][k];
                Om[e][k] = Om[e - 1][k];
            }
#pragma unroll
        for (int k = 0; k < V; ++k) {
            Ol[0][k] = S.l[k];
            Om[0][k] = S.m[k];
        }
#pragma unroll
        for (int d = K - 1; d > 0; --d)
#pragma unroll
            for (int k = 0; k < V; ++k) {
                ar[d][k] = ar[d - 1][k];
                fur[d][k] = fur[d - 1][k];
                fvr[d][k] = fvr[d - 1][k];
                ahu[d][k] = ahu[d - 1][k];
                ahv[d][k] = ahv[d - 1][k];
                alu[d][k] = alu[d - 1][k];
                alv[d][k] = alv[d - 1][k];
            }
#pragma unroll
        for (int k = 0; k < V; ++k) {
            ahu[0][k] = nhu[k];
            ahv[0][k] = nhv[k];
            alu[0][k] = nlu[k];
            alv[0][k] = nlv[k];
        }
        S = C;
        C = N;
        if (r < r1) {
            rawN = rawNN;
            c1 = c1N;
        }
    }
}

template <typename T, int V, int TY, int K, bool FORCE, bool COMP>
__global__ __launch_bounds__(64) void multi2d_kernel(const T* __restrict__ u, const T* __restrict__ uprev,
                                                    T* __restrict__ outA, T* __restrict__ outB,
                                                    double* __restrict__ acc, float* __restrict__ acclo,
                                                    const T* __restrict__ ca, const T* __restrict__ cl,
                                                    const T* __restrict__ cm, const T* __restrict__ f, Args2D A) {
    constexpr int W = MultiCols<V, K>::W;
    const int nbx = (A.nx - 1 + W) / W;
    const int nby = (A.jhi - A.jlo + 1 + TY - 1) / TY;
    int t;
    if (!xcd_tile((int)blockIdx.x, nbx * nby, t)) return;
    multi2d_body<T, V, TY, K, FORCE, COMP>(t % nbx, t / nbx, u, uprev, outA, outB, acc, acclo, ca, cl, cm, f, A);
}

template <typename T, int V, int TY, int K>
static void multi_launch_t(bool force, bool comp, hipStream_t s, int nrows, const T* u, const T* uprev, T* outA,
                           T* outB, double* acc, float* acclo, const T* ca, const T* cl, const T* cm, const T* f,
                           const Args2D& A) {
    constexpr int W = MultiCols<V, K>::W;
    const dim3 grid((unsigned)xcd_grid(((A.nx - 1 + W) / W) * ((nrows + TY - 1) / TY)), 1, 1);
#define ELWH_LM(F, CMP)                                                                                         \
    hipLaunchKernelGGL((multi2d_kernel<T, V, TY, K, F, CMP>), grid, dim3(64), 0, s, u, uprev, outA, outB, acc, \
                       acclo, ca, cl, cm, f, A)
    if constexpr (sizeof(T) == 8) {
        // the compensated accumulator is an FP32-path option
        if (force) ELWH_LM(true, false); else ELWH_LM(false, false);
    } else {
        if (force) {
            if (comp) ELWH_LM(true, true); else ELWH_LM(true, false);
        } else {
            if (comp) ELWH_LM(false, true); else ELWH_LM(false, false);
        }
    }
#undef ELWH_LM
}

template <typename T, int K>
static void multi_launch_k(int V, int TY, bool force, bool comp, hipStream_t s, int nrows, const T* u,
                           const T* uprev, T* outA, T* outB, double* acc, float* acclo, const T* ca, const T* cl,
                           const T* cm, const T* f, const Args2D& A) {
#define ELWH_MC(VV, TT)                                                                                            \
    if (V == VV && TY == TT) {                                                                                     \
        multi_launch_t<T, VV, TT, K>(force, comp, s, nrows, u, uprev, outA, outB, acc, acclo, ca, cl, cm, f, A); \
        return;                                                                                                    \
    }
    ELWH_MC(1, 4) ELWH_MC(1, 8) ELWH_MC(1, 10) ELWH_MC(1, 12) ELWH_MC(1, 16)
    ELWH_MC(2, 4) ELWH_MC(2, 8) ELWH_MC(2, 16)
    if constexpr (sizeof(T) == 4) {
        ELWH_MC(4, 4) ELWH_MC(4, 8) ELWH_MC(4, 16)
    }
#undef ELWH_MC
    multi_launch_t<T, 1, 8, K>(force, comp, s, nrows, u, uprev, outA, outB, acc, acclo, ca, cl, cm, f, A);
}

template <typename T>
void launch_multi2d(int K, int V, int TY, bool force, bool comp, hipStream_t s, int nrows, const T* u,
                    const T* uprev, T* outA, T* outB, double* acc, float* acclo, const T* ca, const T* cl,
                    const T* cm, const T* f, const Args2D& A) {
    if (K == 4)
        multi_launch_k<T, 4>(V, TY, force, comp, s, nrows, u, uprev, outA, outB, acc, acclo, ca, cl, cm, f, A);
    else if (K == 3)
        multi_launch_k<T, 3>(V, TY, force, comp, s, nrows, u, uprev, outA, outB, acc, acclo, ca, cl, cm, f, A);
    else
        multi_launch_k<T, 2>(V, TY, force, comp, s, nrows, u, uprev, outA, outB, acc, acclo, ca, cl, cm, f, A);
}

template void launch_multi2d<double>(int, int, int, bool, bool, hipStream_t, int, const double*, const double*,
                                     double*, double*, double*, float*, const double*, const double*,
                                     const double*, const double*, const Args2D&);
template void launch_multi2d<float>(int, int, int, bool, bool, hipStream_t, int, const float*, const float*,
                                    float*, float*, double*, float*, const float*, const float*, const float*,
                                    const float*, const Args2D&);

}  // namespace elwh

// ===========================================================================
// Ragged batch: the K-step tick (K = 2 or 4) of every active problem with at
// least K steps left in its application (the other problems take the
// single-step tick of kernels2d.hip in the same tick).  Tiles of the K-step
// tiling of all problems are concatenated and dealt in XCD bands.
// ===========================================================================
namespace elwh {

template <typename T, int V, int TY, int K, bool FORCE, bool COMP>
__global__ __launch_bounds__(64) void batch_multi2d_kernel(const BProb2D* __restrict__ pr,
                                                           const BState* __restrict__ st, int np, int ntiles,
                                                           double sgn) {
    int b;
    if (!xcd_tile((int)blockIdx.x, ntiles, b)) return;
    const int p = batch_problem_of(pr, np, b, true);
    const BProb2D& q = pr[p];
    if (!st[p].active) return;
    const int neff = st[p].end ? 0 : st[p].n;
    if (!batch_multi_step(neff, q.nsteps, K)) return;
    const int local = b - q.off2;
    if (local >= q.nblk2) return;
    Args2D A = q.A;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        A.wk[k] = sgn * q.w[neff + 1 + k];
        A.fck[k] = q.cosn[neff + k];
    }
    A.final_ = neff + K == q.nsteps;
    const int ic = st[p].ic, ip = st[p].ip;
    int x1, x2;
    batch_free_two(ic, ip, x1, x2);
    const T* prev = ip >= 0 ? reinterpret_cast<const T*>(q.s[ip]) : reinterpret_cast<const T*>(q.src);
    multi2d_body<T, V, TY, K, FORCE, COMP>(local % q.nbx2, local / q.nbx2, reinterpret_cast<const T*>(q.s[ic]), prev,
                                           reinterpret_cast<T*>(q.s[x1]), reinterpret_cast<T*>(q.s[x2]), q.out, q.lo,
                                           reinterpret_cast<const T*>(q.ca), reinterpret_cast<const T*>(q.cl),
                                           reinterpret_cast<const T*>(q.cm), reinterpret_cast<const T*>(q.f), A);
}

template <typename T, int V, int TY, int K>
static void batch_multi_t(bool force, bool comp, int nblocks2, hipStream_t s, const BProb2D* pr, const BState* st,
                          int np, double sgn) {
#define ELWH_BM(F, C)                                                                                           \
    hipLaunchKernelGGL((batch_multi2d_kernel<T, V, TY, K, F, C>), dim3((unsigned)xcd_grid(nblocks2)), dim3(64), 0, \
                       s, pr, st, np, nblocks2, sgn)
    if constexpr (sizeof(T) == 8) {
        if (force) ELWH_BM(true, false); else ELWH_BM(false, false);
    } else {
        if (force) {
            if (comp) ELWH_BM(true, true); else ELWH_BM(true, false);
        } else {
            if (comp) ELWH_BM(false, true); else ELWH_BM(false, false);
        }
    }
#undef ELWH_BM
}

int batch_cols_k(int V, int kb) {
    if (kb == 4) return V == 1 ? MultiCols<1, 4>::W : (V == 2 ? MultiCols<2, 4>::W : MultiCols<4, 4>::W);
    return V == 1 ? MultiCols<1, 2>::W : (V == 2 ? MultiCols<2, 2>::W : MultiCols<4, 2>::W);
}

void launch_batch_multi(bool fp32, int V, int TY, int kb, bool force, bool comp, int nblocks2, hipStream_t s,
                        const BProb2D* pr, const BState* st, int np, double sgn, int amode) {
    (void)amode;   // the sign of the weights carries the A_h form
    if (nblocks2 <= 0) return;
#define ELWH_BMT(T, VV, TT, KK)                                                       \
    if (V == VV && TY == TT && kb == KK) {                                            \
        batch_multi_t<T, VV, TT, KK>(force, comp, nblocks2, s, pr, st, np, sgn);      \
        return;                                                                       \
    }
    if (fp32) {
        ELWH_BMT(float, 1, 4, 2) ELWH_BMT(float, 1, 8, 2) ELWH_BMT(float, 2, 4, 2) ELWH_BMT(float, 2, 8, 2)
        ELWH_BMT(float, 2, 16, 2) ELWH_BMT(float, 4, 8, 2)
        ELWH_BMT(float, 1, 4, 4) ELWH_BMT(float, 1, 8, 4) ELWH_BMT(float, 1, 10, 4) ELWH_BMT(float, 2, 8, 4)
    } else {
        ELWH_BMT(double, 1, 4, 2) ELWH_BMT(double, 1, 8, 2) ELWH_BMT(double, 2, 4, 2) ELWH_BMT(double, 2, 8, 2)
        ELWH_BMT(double, 2, 16, 2)
        ELWH_BMT(double, 1, 4, 4) ELWH_BMT(double, 1, 8, 4) ELWH_BMT(double, 1, 10, 4)
    }
#undef ELWH_BMT
}

}  // namespace elwh
