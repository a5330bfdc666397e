// 2-D fused El-WaveHoltz step for gfx950.
//
// One launch advances every unknown node by one time step of the corrected
// leapfrog (Sec. 4.3, eq. elastic-time-explicit-corrected)
//     u^{n+1} = 2 u^n - u^{n-1} + a (Ltilde u^n - f cos(omega t_n)),   a = c dt^2 / rho,
// and adds w_{n+1} u^{n+1} into the FP64 filter accumulator (trapezoid rule
// of eq. el_WHI_OP) in the same pass.  The half-step launch computes the
// even-in-time start u^1 = u^0 + (a/2)(Ltilde u^0 - f) and seeds the
// accumulator with w_0 u^0 + w_1 u^1 (or x - w_0 u^0 - w_1 u^1 for A_h x).
//
// Ltilde is the conservative second-order stress divergence
//     u-row: D+x(Abar D-x u) + D+y(mubar D-y u) + D0x(lam D0y v) + D0y(mu D0x v)
//     v-row: D+x(mubar D-x v) + D+y(Abar D-y v) + D0x(mu D0y u) + D0y(lam D0x u)
// (A = lam + 2 mu, bars = two-point means), with the rows of a traction-free
// y face closed from the discrete energy (one-sided normal differences, the
// trapezoid weight 1/2 divided out).
//
// Mapping.  One 64-lane wavefront per block; each lane owns V consecutive x
// nodes (one vector load per array and row), so a wavefront covers 64 V
// columns of which the outer halo columns are loaded but not computed
// (W = 62, 126, 252 computed columns for V = 1, 2, 4).  The wavefront marches
// TY rows in y (up in even row chunks, down in odd ones, so that two
// neighbouring chunks read their shared rows together): rows j-1, j, j+1
// live in registers and roll, the loads of
// row j+2 and of the centre-row arrays of row j+1 are issued one iteration
// ahead, and x neighbours across lanes come from DPP wavefront shifts.
// Every array element is read from memory once per row visit.
#include "step2d_common.h"

namespace elwh {

template <typename T, int V, bool COMP, bool FORCE, int MODE>
struct Centre {
    T a[V];
    T up[V], vp[V];             // u^{n-1} (MODE 0)
    double hu[V], hv[V];        // accumulator (MODE 0) or base x (MODE 1)
    float lu[V], lv[V];         // compensation (MODE 0, COMP), widened where it is used
    T fu[V], fv[V];             // forcing
};

// One wavefront's share of one step: the x-strip bx and row chunk by.
// MODE 0: time step; MODE 1: initial half step.  U: element type of the
// u^n input (double for the half step from an FP64 vector, T otherwise).
template <typename T, typename U, int V, int TY, int MODE, bool FORCE, bool COMP>
__device__ __forceinline__ void step2d_body(int bx, int by, const U* __restrict__ u, const T* uprev, T* unext,
                                            const double* __restrict__ xbase, T* __restrict__ u0out,
                                            double* __restrict__ acc, float* __restrict__ acclo,
                                            const T* __restrict__ ca, const T* __restrict__ cl,
                                            const T* __restrict__ cm, const T* __restrict__ f, const Args2D& A) {
    constexpr int W = Cols<V>::W;
    const int lane = threadIdx.x;
    const int c0 = W * bx;
    const int col = c0 + V * lane;                // first column of this lane
    const bool colv = col <= A.nx;                // vector lies in the padded row
    const int j0 = A.jlo + by * TY;
    if (j0 > A.jhi) return;
    const int j1 = min(j0 + TY - 1, A.jhi);
    const int P = (int)A.P;
    const int64_t CS = A.CS;
    // Mirrored march: odd row chunks march downwards, so that neighbouring
    // chunks read the rows they share at the same time and the second read
    // finds them in L2.  Virtual row v is physical row jb + dir * v; mirrored,
    // the stencil exchanges the rows below and above, i.e. negates the
    // mixed-derivative coefficients and swaps the two free-row kinds.
    const int dir = (by & 1) ? -1 : 1;
    const int jb = dir > 0 ? 0 : j0 + j1;
    auto phys = [&](int v) { return jb + dir * v; };
    const T cxx2 = (T)A.cxx2, cyy2 = (T)A.cyy2, cxy = (T)(dir * A.cxy), cyyf = (T)A.cyyf, cfx = (T)(dir * A.cfx);
    const T two = (T)2;
    const int ilo = max(c0 + 1, 1), ihi = min(c0 + W, A.nx - 1);   // computed column range

    auto load_raw = [&](int jv, RawRow<T, V>& r) {
        const int j = phys(jv);
        if (colv && j >= 0 && j <= A.ny) {
            const int64_t o = (int64_t)j * P + col;
            vload<U, T, V>(u + o, r.u);
            vload<U, T, V>(u + o + CS, r.v);
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
    using Ctr = Centre<T, V, COMP, FORCE, MODE>;
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

    Row<T, V> S, C, N;
    {
        RawRow<T, V> r;
        load_raw(j0 - 1, r);
        finish(r, S);
        load_raw(j0, r);
        finish(r, C);
    }
    RawRow<T, V> rawN;
    load_raw(j0 + 1, rawN);
    Ctr ctr;
    load_ctr(j0, ctr);

    for (int j = j0; j <= j1; ++j) {
        // issue the loads of the next iteration before computing this one
        RawRow<T, V> rawNN;
        Ctr ctrN;
        if (j + 1 <= j1) {
            load_raw(j + 2, rawNN);
            load_ctr(j + 1, ctrN);
        }
        finish(rawN, N);
        const T lamL0 = lane_from_left(C.l[V - 1]), lamR0 = lane_from_right(C.l[0]);
        const T muL0 = lane_from_left(C.m[V - 1]), muR0 = lane_from_right(C.m[0]);
        const int pj = phys(j);
        const int kind0 = (A.free_hi && pj == A.ny) ? 1 : ((A.free_lo && pj == 0) ? 2 : 0);
        const int kind = dir > 0 || kind0 == 0 ? kind0 : 3 - kind0;
        const int64_t o = (int64_t)pj * P + col;

#pragma unroll
        for (int k = 0; k < V; ++k) {
            const int i = col + k;
            if (i < ilo || i > ihi || !colv) continue;
            const Nb<T> s = node_of<T, V>(S, k), cc = node_of<T, V>(C, k), nn = node_of<T, V>(N, k);
            const T lamL = k > 0 ? C.l[k > 0 ? k - 1 : 0] : lamL0;
            const T lamR = k < V - 1 ? C.l[k < V - 1 ? k + 1 : 0] : lamR0;
            const T muL = k > 0 ? C.m[k > 0 ? k - 1 : 0] : muL0;
            const T muR = k < V - 1 ? C.m[k < V - 1 ? k + 1 : 0] : muR0;
            T Lu, Lv;
            stencil2d<T>(kind, s, cc, nn, lamL, lamR, muL, muR, cxx2, cyy2, cxy, cyyf, cfx, Lu, Lv);
            if constexpr (FORCE) {
                const T fc = (T)A.fc;
                Lu -= fc * ctr.fu[k];
                Lv -= fc * ctr.fv[k];
            }
            const T a = ctr.a[k];
            T nu, nv;
            double hu = ctr.hu[k], hv = ctr.hv[k], lu = 0.0, lv = 0.0;
            if constexpr (MODE == 0) {
                nu = two * cc.u - ctr.up[k] + a * Lu;
                nv = two * cc.v - ctr.vp[k] + a * Lv;
                if constexpr (COMP) {
                    lu = ctr.lu[k];
                    lv = ctr.lv[k];
                }
            } else {
                const T ha = (T)0.5 * a;
                nu = cc.u + ha * Lu;
                nv = cc.v + ha * Lv;
                acc_add(hu, lu, A.w0 * (double)cc.u, COMP);
                acc_add(hv, lv, A.w0 * (double)cc.v, COMP);
                if (u0out) {
                    u0out[o + k] = cc.u;
                    u0out[o + k + CS] = cc.v;
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

template <typename T, typename U, int V, int TY, int MODE, bool FORCE, bool COMP>
__global__ __launch_bounds__(64) void step2d_kernel(const U* __restrict__ u, const T* uprev, T* unext,
                                                   const double* __restrict__ xbase, T* __restrict__ u0out,
                                                   double* __restrict__ acc, float* __restrict__ acclo,
                                                   const T* __restrict__ ca, const T* __restrict__ cl,
                                                   const T* __restrict__ cm, const T* __restrict__ f, Args2D A) {
    const int nbx = (A.nx - 1 + Cols<V>::W - 1) / Cols<V>::W;
    const int nby = (A.jhi - A.jlo + 1 + TY - 1) / TY;
    int t;
    if (!xcd_tile((int)blockIdx.x, nbx * nby, t)) return;
    step2d_body<T, U, V, TY, MODE, FORCE, COMP>(t % nbx, t / nbx, u, uprev, unext, xbase, u0out,
                                                acc, acclo, ca, cl, cm, f, A);
}

// ---------------------------------------------------------------------------

template <typename T, typename U, int V, int TY, int MODE>
static void launch_t(bool force, bool comp, dim3 grid, hipStream_t s, const U* u, const T* uprev, T* unext,
                     const double* xbase, T* u0out, double* acc, float* acclo, const T* ca, const T* cl,
                     const T* cm, const T* f, const Args2D& A) {
#define ELWH_L2(F, CMP)                                                                                  \
    hipLaunchKernelGGL((step2d_kernel<T, U, V, TY, MODE, F, CMP>), grid, dim3(64), 0, s, u, uprev, unext, \
                       xbase, u0out, acc, acclo, ca, cl, cm, f, A)
    if (force) {
        if (comp) ELWH_L2(true, true); else ELWH_L2(true, false);
    } else {
        if (comp) ELWH_L2(false, true); else ELWH_L2(false, false);
    }
#undef ELWH_L2
}

// Dispatch over the tunable (V, TY) pairs.
template <typename T, typename U, int MODE>
static void launch_v(int V, int TY, bool force, bool comp, int nx, int nrows, hipStream_t s, const U* u,
                     const T* uprev, T* unext, const double* xbase, T* u0out, double* acc, float* acclo,
                     const T* ca, const T* cl, const T* cm, const T* f, const Args2D& A) {
    auto grid_for = [&](int W, int ty) {
        return dim3((unsigned)xcd_grid(((nx - 1 + W - 1) / W) * ((nrows + ty - 1) / ty)), 1, 1);
    };
#define ELWH_CASE(VV, TT)                                                                                \
    if (V == VV && TY == TT) {                                                                           \
        launch_t<T, U, VV, TT, MODE>(force, comp, grid_for(Cols<VV>::W, TT), s, u, uprev, unext, xbase, u0out, \
                                     acc, acclo, ca, cl, cm, f, A);                                      \
        return;                                                                                          \
    }
    ELWH_CASE(1, 4) ELWH_CASE(1, 8) ELWH_CASE(1, 10) ELWH_CASE(1, 12) ELWH_CASE(1, 16)
    ELWH_CASE(2, 4) ELWH_CASE(2, 8) ELWH_CASE(2, 16)
    if constexpr (sizeof(T) == 4) {
        ELWH_CASE(4, 4) ELWH_CASE(4, 8) ELWH_CASE(4, 16)
    }
#undef ELWH_CASE
    // unreachable for validated tiles; fall back to the smallest tile
    launch_t<T, U, 1, 8, MODE>(force, comp, grid_for(Cols<1>::W, 8), s, u, uprev, unext, xbase, u0out, acc, acclo,
                               ca, cl, cm, f, A);
}

Args2D make_args2d(const elwh_ctx* c) {
    Args2D A;
    A.nx = c->L.nx;
    A.ny = c->L.ny;
    A.P = c->L.P;
    A.CS = c->L.CS;
    A.jlo = c->mr.lo;
    A.jhi = c->mr.hi;
    A.free_lo = c->mr.free_lo;
    A.free_hi = c->mr.free_hi;
    A.cxx2 = c->st.cxx2;
    A.cyy2 = c->st.cyy2;
    A.cxy = c->st.cxy;
    A.cyyf = c->st.cyyf;
    A.cfx = c->st.cfxy;
    A.w = A.w0 = A.fc = 0;
    for (int q = 0; q < 4; ++q) A.wk[q] = A.fck[q] = 0;
    A.final_ = 0;
    return A;
}

bool tile_valid_2d(bool fp32, int V, int TY) {
    const bool v_ok = V == 1 || V == 2 || (fp32 && V == 4);
    return v_ok && (TY == 4 || TY == 8 || TY == 16 || (V == 1 && (TY == 10 || TY == 12)));
}

// ===========================================================================
// Ragged batch: many 2-D problems of different size, medium, omega and N_T in
// one launch per time step.  Each problem keeps its own step counter and CG
// scalars in device memory (BState); block b of a launch belongs to the
// problem whose block range contains b.  A problem that finishes an
// application in a tick runs its CG update in the same tick and starts its
// next application in the next one, independently of the others.
// ===========================================================================

// Single-step tick: the half step that starts an application, and every
// step of problems that do not take a kb-step launch this tick (kb = 0, or
// fewer than kb steps left).  u^{n+1} overwrites u^{n-1} when that is a
// state buffer.
template <typename T, int V, int TY, bool FORCE, bool COMP>
__global__ __launch_bounds__(64) void batch_step2d_kernel(const BProb2D* __restrict__ pr, const BState* __restrict__ st,
                                                          int np, int ntiles, double sgn, int amode, int kb) {
    // XCD bands over the concatenated tiles of all problems
    int b;
    if (!xcd_tile((int)blockIdx.x, ntiles, b)) return;
    const int p = batch_problem_of(pr, np, b, false);
    const BProb2D& q = pr[p];
    if (!st[p].active) return;
    const int neff = st[p].end ? 0 : st[p].n;
    if (batch_multi_step(neff, q.nsteps, kb)) return;
    const int local = b - q.off;
    if (local >= q.nblk) return;
    const int bx = local % q.nbx, by = local / q.nbx;
    Args2D A = q.A;
    const T* ca = reinterpret_cast<const T*>(q.ca);
    const T* cl = reinterpret_cast<const T*>(q.cl);
    const T* cm = reinterpret_cast<const T*>(q.cm);
    const T* f = reinterpret_cast<const T*>(q.f);
    if (neff == 0) {
        // u^1 into s[1]; FP32 also keeps u^0 in s[0]
        A.w0 = sgn * q.w[0];
        A.w = sgn * q.w[1];
        A.fc = q.cosn[0];
        A.final_ = 0;
        step2d_body<T, double, V, TY, 1, FORCE, COMP>(bx, by, q.src, nullptr, reinterpret_cast<T*>(q.s[1]),
                                                      amode ? q.src : nullptr,
                                                      sizeof(T) == 4 ? reinterpret_cast<T*>(q.s[0]) : nullptr, q.out,
                                                      q.lo, ca, cl, cm, f, A);
    } else {
        A.w = sgn * q.w[neff + 1];
        A.fc = q.cosn[neff];
        A.final_ = neff == q.nsteps - 1;
        const int ic = st[p].ic, ip = st[p].ip;
        T* cur = reinterpret_cast<T*>(q.s[ic]);
        T* nxt = reinterpret_cast<T*>(q.s[batch_single_target(ic, ip)]);
        const T* prev = ip >= 0 ? reinterpret_cast<const T*>(q.s[ip]) : reinterpret_cast<const T*>(q.src);
        step2d_body<T, T, V, TY, 0, FORCE, COMP>(bx, by, cur, prev, nxt, nullptr, nullptr, q.out, q.lo, ca, cl, cm, f,
                                                 A);
    }
}

template <typename T, int V, int TY>
static void batch_step_t(bool force, bool comp, int nblocks, hipStream_t s, const BProb2D* pr, const BState* st,
                         int np, double sgn, int amode, int kb) {
#define ELWH_B2(F, C) \
    hipLaunchKernelGGL((batch_step2d_kernel<T, V, TY, F, C>), dim3((unsigned)xcd_grid(nblocks)), dim3(64), 0, s, pr, st, \
                       np, nblocks, sgn, amode, kb)
    if (force) {
        if (comp) ELWH_B2(true, true); else ELWH_B2(true, false);
    } else {
        if (comp) ELWH_B2(false, true); else ELWH_B2(false, false);
    }
#undef ELWH_B2
}

bool batch_tile_valid(bool fp32, int V, int TY, int kb) {
    if (kb == 4) return (V == 1 && (TY == 4 || TY == 8 || TY == 10)) || (fp32 && V == 2 && TY == 8);
    if (V == 1 && (TY == 4 || TY == 8)) return true;
    if (V == 2 && (TY == 4 || TY == 8 || TY == 16)) return true;
    return fp32 && V == 4 && TY == 8;
}

int batch_cols(int V) { return V == 1 ? Cols<1>::W : (V == 2 ? Cols<2>::W : Cols<4>::W); }

void launch_batch_step(bool fp32, int V, int TY, bool force, bool comp, int nblocks, hipStream_t s,
                       const BProb2D* pr, const BState* st, int np, double sgn, int amode, int kb) {
#define ELWH_BT(T, VV, TT)                                                                          \
    if (V == VV && TY == TT) {                                                                      \
        batch_step_t<T, VV, TT>(force, comp, nblocks, s, pr, st, np, sgn, amode, kb);               \
        return;                                                                                     \
    }
    if (fp32) {
        ELWH_BT(float, 1, 4) ELWH_BT(float, 1, 8) ELWH_BT(float, 1, 10) ELWH_BT(float, 2, 4) ELWH_BT(float, 2, 8)
        ELWH_BT(float, 2, 16) ELWH_BT(float, 4, 8)
    } else {
        ELWH_BT(double, 1, 4) ELWH_BT(double, 1, 8) ELWH_BT(double, 1, 10) ELWH_BT(double, 2, 4)
        ELWH_BT(double, 2, 8) ELWH_BT(double, 2, 16)
    }
#undef ELWH_BT
}

Args2D make_args2d(const elwh_ctx* c);

// One filter application (2-D), see elwh_internal.h.
// The two state buffers of bufs[0..3] that are neither a nor b.
template <typename T>
static void free_pair(T* const* bufs, const void* a, const void* b, T** x, T** y) {
    T* got[2] = {nullptr, nullptr};
    int k = 0;
    for (int i = 0; i < 4 && k < 2; ++i)
        if (bufs[i] != a && bufs[i] != b) got[k++] = bufs[i];
    *x = got[0];
    *y = got[1];
}

// Steps 1 .. nsteps-1 after the half step: launches of K = fuse steps (a
// shorter multi-step launch, or a single step, for the remainder); or single
// steps in place (fuse = 1).  prev/cur hold u^0/u^1 on entry; prev may be the
// caller's vector (never written).
template <typename T>
static void run_steps_2d(elwh_ctx* c, Args2D A, int nrows, Tile t, bool with_force, bool comp, double sgn,
                         const T* prev, T* cur, T* const* bufs, double* acc, float* lo, const T* ca, const T* cl,
                         const T* cm, const T* f, int nsteps) {
    hipStream_t s = c->stream;
    int n = 1;
    if (c->opts.fuse >= 2) {
        while (nsteps - n >= 2) {
            const int k = std::min(c->opts.fuse, nsteps - n);
            T *x1, *x2;
            free_pair(bufs, prev, cur, &x1, &x2);
            for (int q = 1; q <= k; ++q) {
                A.wk[q - 1] = sgn * c->w[n + q];
                A.fck[q - 1] = c->cosn[n + q - 1];
            }
            A.final_ = (n + k == nsteps);
            launch_multi2d<T>(k, t.V, t.TY, with_force, comp, s, nrows, cur, prev, x1, x2, acc, lo, ca, cl, cm, f, A);
            prev = x1;
            cur = x2;
            n += k;
        }
    }
    for (; n < nsteps; ++n) {
        // u^{n+1} overwrites u^{n-1} when that is one of the state buffers
        T* nxt = nullptr;
        for (int i = 0; i < 4; ++i)
            if (bufs[i] == prev) nxt = bufs[i];
        if (!nxt) {
            T* dummy;
            free_pair(bufs, prev, cur, &nxt, &dummy);
        }
        A.w = sgn * c->w[n + 1];
        A.fc = c->cosn[n];
        A.final_ = (n == nsteps - 1);
        launch_v<T, T, 0>(t.V, t.TY, with_force, comp, A.nx, nrows, s, cur, prev, nxt, nullptr, nullptr, acc, lo,
                          ca, cl, cm, f, A);
        prev = cur;
        cur = nxt;
    }
}

void run_filter_2d(elwh_ctx* c, const double* x, bool with_force, bool amode, bool fp32, double* out) {
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
        // half step: u^1 into s64[1]; u^0 is read from x itself afterwards
        double* b1 = c->s64[1];
        launch_v<double, double, 1>(t.V, t.TY, with_force, false, A.nx, nrows, s, x, nullptr, b1,
                                    amode ? x : nullptr, nullptr, acc, lo, c->ca, c->cl, c->cm, c->f64, A);
        prof_mark(c, 1);
        run_steps_2d<double>(c, A, nrows, t, with_force, false, sgn, x, b1, c->s64, acc, lo, c->ca, c->cl, c->cm,
                             c->f64, nsteps);
    } else {
        // half step: FP32 u^0 into s32[0], u^1 into s32[1]
        float *b0 = c->s32[0], *b1 = c->s32[1];
        launch_v<float, double, 1>(t.V, t.TY, with_force, comp, A.nx, nrows, s, x, nullptr, b1,
                                   amode ? x : nullptr, b0, acc, lo, c->fa, c->fl, c->fm, c->f32, A);
        prof_mark(c, 1);
        run_steps_2d<float>(c, A, nrows, t, with_force, comp, sgn, b0, b1, c->s32, acc, lo, c->fa, c->fl, c->fm,
                            c->f32, nsteps);
    }
    prof_mark(c, 2, nsteps - 1);
}

}  // namespace elwh
