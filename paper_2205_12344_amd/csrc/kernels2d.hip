// 2-D fused El-WaveHoltz step for gfx950.
//
// One launch advances every unknown node by one time step of the corrected
// leapfrog (Sec. 4.3, eq. elastic-time-explicit-corrected)
//     u^{n+1} = 2 u^n - u^{n-1} + a (Ltilde u^n - f cos(omega t_n)),   a = c dt^2 / rho,
// and adds w_{n+1} u^{n+1} into the FP64 filter accumulator (trapezoid rule
// of eq. el_WHI_OP), in the same pass.  The initial launch computes the
// even-in-time start u^1 = u^0 + (a/2)(Ltilde u^0 - f) and seeds the
// accumulator with w_0 u^0 + w_1 u^1 (or x - w_0 u^0 - w_1 u^1 for A_h x).
//
// Ltilde is the conservative second-order stress divergence
//     u-row: D+x(Abar D-x u) + D+y(mubar D-y u) + D0x(lam D0y v) + D0y(mu D0x v)
//     v-row: D+x(mubar D-x v) + D+y(Abar D-y v) + D0x(mu D0y u) + D0y(lam D0x u)
// (A = lam + 2 mu, bars = two-point means), with the traction-free rows of a
// free y face closed from the discrete energy (one-sided normal
// differences, trapezoid weight 1/2 divided out).
//
// Mapping: one 64-lane wavefront per block owns 64 consecutive x nodes of
// which lanes 1..62 are computed (lanes 0 and 63 are the x halo), and
// marches up TY rows in y.  Rows j-1, j, j+1 live in registers and roll;
// x neighbours come from the adjacent lanes by cross-lane moves, so every
// array element is loaded by one lane of one wavefront per row visit.
#include "elwh_internal.h"
#include "lanes.h"

namespace elwh {

struct Args2D {
    int nx, ny;
    int64_t P, CS;
    int jlo, jhi, free_lo, free_hi;
    double cxx2, cyy2, cxy, cyyf, cfx;
    double w, w0, fc;
    int final_;
};

template <typename T>
struct Row {
    T u, v, uL, uR, vL, vR, lam, mu;
};

template <typename T>
__device__ __forceinline__ void neighbours(Row<T>& r) {
    r.uL = lane_from_left(r.u);
    r.uR = lane_from_right(r.u);
    r.vL = lane_from_left(r.v);
    r.vR = lane_from_right(r.v);
}

__device__ __forceinline__ void acc_add(double& hi, double& lo, double x, bool comp) {
    if (comp) {
        // Knuth's TwoSum: hi + x = t + e exactly; e goes to the compensation
        const double t = hi + x;
        const double z = t - hi;
        const double e = (hi - (t - z)) + (x - z);
        hi = t;
        lo += e;
    } else {
        hi += x;
    }
}

// MODE 0: time step; MODE 1: initial half step.
// U: element type of the u^n input (double for the half step from an FP64
// vector; T otherwise).
template <typename T, typename U, int TY, int MODE, bool FORCE, bool COMP>
__global__ __launch_bounds__(64) void step2d_kernel(const U* __restrict__ u, const T* uprev, T* unext,
                                                   const double* __restrict__ xbase, T* __restrict__ u0out,
                                                   double* __restrict__ acc, double* __restrict__ acclo,
                                                   const T* __restrict__ ca, const T* __restrict__ cl,
                                                   const T* __restrict__ cm, const T* __restrict__ f,
                                                   Args2D A) {
    const int lane = threadIdx.x;
    const int i = 62 * blockIdx.x + lane;
    const bool colv = i <= A.nx;
    const bool store = lane >= 1 && lane <= 62 && i >= 1 && i <= A.nx - 1;
    const int j0 = A.jlo + (int)blockIdx.y * TY;
    if (j0 > A.jhi) return;
    const int j1 = min(j0 + TY - 1, A.jhi);
    const int64_t P = A.P, CS = A.CS;

    const T cxx2 = (T)A.cxx2, cyy2 = (T)A.cyy2, cxy = (T)A.cxy, cyyf = (T)A.cyyf, cfx = (T)A.cfx;
    const T two = (T)2;

    auto load_row = [&](int j, Row<T>& r) {
        if (colv && j >= 0 && j <= A.ny) {
            const int64_t o = (int64_t)j * P + i;
            r.u = (T)u[o];
            r.v = (T)u[o + CS];
            r.lam = cl[o];
            r.mu = cm[o];
        } else {
            r.u = r.v = r.lam = r.mu = (T)0;
        }
        neighbours(r);
    };

    Row<T> S, C, N;
    load_row(j0 - 1, S);
    load_row(j0, C);

    for (int j = j0; j <= j1; ++j) {
        load_row(j + 1, N);
        const T lamL = lane_from_left(C.lam), lamR = lane_from_right(C.lam);
        const T muL = lane_from_left(C.mu), muR = lane_from_right(C.mu);
        const int64_t o = (int64_t)j * P + i;

        T Lu, Lv;
        const T AL = lamL + two * muL, AC = C.lam + two * C.mu, AR = lamR + two * muR;
        // in-row compact x terms (all row kinds)
        const T xu = cxx2 * ((AR + AC) * (C.uR - C.u) - (AC + AL) * (C.u - C.uL));
        const T xv = cxx2 * ((muR + C.mu) * (C.vR - C.v) - (C.mu + muL) * (C.v - C.vL));
        if (A.free_hi && j == A.ny) {
            // traction-free top row: S is the row below
            const T AS = S.lam + two * S.mu;
            Lu = xu - cyyf * (C.mu + S.mu) * (C.u - S.u) -
                 cfx * (C.mu * (C.vR - C.vL) + S.mu * (S.vR - S.vL)) +
                 cfx * (lamR * (C.vR - S.vR) - lamL * (C.vL - S.vL));
            Lv = xv - cyyf * (AC + AS) * (C.v - S.v) -
                 cfx * (C.lam * (C.uR - C.uL) + S.lam * (S.uR - S.uL)) +
                 cfx * (muR * (C.uR - S.uR) - muL * (C.uL - S.uL));
        } else if (A.free_lo && j == 0) {
            // traction-free bottom row: N is the row above
            const T AN = N.lam + two * N.mu;
            Lu = xu + cyyf * (C.mu + N.mu) * (N.u - C.u) +
                 cfx * (C.mu * (C.vR - C.vL) + N.mu * (N.vR - N.vL)) +
                 cfx * (lamR * (N.vR - C.vR) - lamL * (N.vL - C.vL));
            Lv = xv + cyyf * (AC + AN) * (N.v - C.v) +
                 cfx * (C.lam * (C.uR - C.uL) + N.lam * (N.uR - N.uL)) +
                 cfx * (muR * (N.uR - C.uR) - muL * (N.uL - C.uL));
        } else {
            const T AN = N.lam + two * N.mu, AS = S.lam + two * S.mu;
            Lu = xu + cyy2 * ((N.mu + C.mu) * (N.u - C.u) - (C.mu + S.mu) * (C.u - S.u)) +
                 cxy * (lamR * (N.vR - S.vR) - lamL * (N.vL - S.vL) + N.mu * (N.vR - N.vL) -
                        S.mu * (S.vR - S.vL));
            Lv = xv + cyy2 * ((AN + AC) * (N.v - C.v) - (AC + AS) * (C.v - S.v)) +
                 cxy * (muR * (N.uR - S.uR) - muL * (N.uL - S.uL) + N.lam * (N.uR - N.uL) -
                        S.lam * (S.uR - S.uL));
        }

        if (store) {
            const T a = ca[o];
            if constexpr (FORCE) {
                const T fc = (T)A.fc;
                Lu -= fc * f[o];
                Lv -= fc * f[o + CS];
            }
            T nu, nv;
            double hu, hv, lu = 0.0, lv = 0.0;
            if constexpr (MODE == 0) {
                nu = two * C.u - uprev[o] + a * Lu;
                nv = two * C.v - uprev[o + CS] + a * Lv;
                hu = acc[o];
                hv = acc[o + CS];
                if constexpr (COMP) {
                    lu = acclo[o];
                    lv = acclo[o + CS];
                }
            } else {
                const T ha = (T)0.5 * a;
                nu = C.u + ha * Lu;
                nv = C.v + ha * Lv;
                hu = xbase ? xbase[o] : 0.0;
                hv = xbase ? xbase[o + CS] : 0.0;
                acc_add(hu, lu, A.w0 * (double)C.u, COMP);
                acc_add(hv, lv, A.w0 * (double)C.v, COMP);
                if (u0out) {
                    u0out[o] = C.u;
                    u0out[o + CS] = C.v;
                }
            }
            unext[o] = nu;
            unext[o + CS] = nv;
            acc_add(hu, lu, A.w * (double)nu, COMP);
            acc_add(hv, lv, A.w * (double)nv, COMP);
            if (COMP && A.final_) {
                acc[o] = hu + lu;
                acc[o + CS] = hv + lv;
            } else {
                acc[o] = hu;
                acc[o + CS] = hv;
                if constexpr (COMP) {
                    acclo[o] = lu;
                    acclo[o + CS] = lv;
                }
            }
        }
        S = C;
        C = N;
    }
}

// ---------------------------------------------------------------------------

template <typename T, typename U, int TY, int MODE>
static void launch_t(bool force, bool comp, dim3 grid, hipStream_t s, const U* u, const T* uprev, T* unext,
                     const double* xbase, T* u0out, double* acc, double* acclo, const T* ca, const T* cl,
                     const T* cm, const T* f, const Args2D& A) {
#define ELWH_L2(F, CMP)                                                                           \
    hipLaunchKernelGGL((step2d_kernel<T, U, TY, MODE, F, CMP>), grid, dim3(64), 0, s, u, uprev, unext, \
                       xbase, u0out, acc, acclo, ca, cl, cm, f, A)
    if (force) {
        if (comp) ELWH_L2(true, true); else ELWH_L2(true, false);
    } else {
        if (comp) ELWH_L2(false, true); else ELWH_L2(false, false);
    }
#undef ELWH_L2
}

struct Sweep2D {
    dim3 grid;
    Args2D A;
};

static Sweep2D setup2d(const elwh_ctx* c, int ty) {
    Sweep2D s;
    Args2D& A = s.A;
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
    A.final_ = 0;
    const int nrows = A.jhi - A.jlo + 1;
    s.grid = dim3((unsigned)((A.nx - 1 + 61) / 62), (unsigned)((nrows + ty - 1) / ty), 1);
    return s;
}

constexpr int TY2 = 16;

// One filter application (2-D), see elwh_internal.h.
void run_filter_2d(elwh_ctx* c, const double* x, bool with_force, bool amode, bool fp32, double* out) {
    hipStream_t s = c->stream;
    Sweep2D sw = setup2d(c, TY2);
    Args2D& A = sw.A;
    const int nsteps = c->plan.nt * c->opts.periods;
    const double sgn = amode ? -1.0 : 1.0;
    const bool comp = fp32 && c->opts.compensated;
    double* acc = out;
    double* lo = c->acc_lo;
    A.w0 = sgn * c->w[0];
    A.w = sgn * c->w[1];
    A.fc = c->cosn[0];
    if (!fp32) {
        double *b0 = c->s64[0], *b1 = c->s64[1];
        prof_begin(c);
        launch_t<double, double, TY2, 1>(with_force, false, sw.grid, s, x, nullptr, b1, amode ? x : nullptr,
                                         nullptr, acc, lo, c->ca, c->cl, c->cm, c->f64, A);
        prof_end(c, 1);
        // step 1 reads u^0 from x itself and writes u^2 into b0; from step 2
        // on u^{n+1} overwrites u^{n-1} in place
        const double* prev = x;
        double* cur = b1;
        for (int n = 1; n < nsteps; ++n) {
            double* nxt = (n == 1) ? b0 : const_cast<double*>(prev);
            A.w = sgn * c->w[n + 1];
            A.fc = c->cosn[n];
            prof_begin(c);
            launch_t<double, double, TY2, 0>(with_force, false, sw.grid, s, cur, prev, nxt, nullptr, nullptr,
                                             acc, lo, c->ca, c->cl, c->cm, c->f64, A);
            prof_end(c, 0);
            prev = cur;
            cur = nxt;
        }
    } else {
        float *b0 = c->s32[0], *b1 = c->s32[1];
        prof_begin(c);
        launch_t<float, double, TY2, 1>(with_force, comp, sw.grid, s, x, nullptr, b1, amode ? x : nullptr, b0,
                                        acc, lo, c->fa, c->fl, c->fm, c->f32, A);
        prof_end(c, 1);
        float* prev = b0;
        float* cur = b1;
        for (int n = 1; n < nsteps; ++n) {
            A.w = sgn * c->w[n + 1];
            A.fc = c->cosn[n];
            A.final_ = (n == nsteps - 1);
            prof_begin(c);
            launch_t<float, float, TY2, 0>(with_force, comp, sw.grid, s, cur, prev, prev, nullptr, nullptr, acc,
                                           lo, c->fa, c->fl, c->fm, c->f32, A);
            prof_end(c, 0);
            float* t = prev;
            prev = cur;
            cur = t;
        }
    }
}

}  // namespace elwh
