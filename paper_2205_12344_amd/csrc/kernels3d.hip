// 3-D fused El-WaveHoltz step for gfx950.
//
// Same update as the 2-D kernel (corrected leapfrog of Sec. 4.3, trapezoid
// accumulation of eq. el_WHI_OP fused into the step), with the 3-D
// conservative stress divergence: for the u-row
//   D+x(Abar D-x u) + D+y(mubar D-y u) + D+z(mubar D-z u)
//   + D0x(lam D0y v) + D0y(mu D0x v) + D0x(lam D0z w) + D0z(mu D0x w)
// and cyclically for v and w (a 19-point footprint).  Traction-free z faces
// are closed from the discrete energy (one-sided normal differences, the
// trapezoid weight 1/2 divided out).
//
// Mapping: a workgroup of RB 64-lane wavefronts owns 64 x nodes (62
// computed) of RB consecutive y rows, one row per wavefront, and marches TZ
// planes in z.  Three planes x three rows of the displacement live in
// registers and roll in z; x neighbours come from the adjacent lanes;
// y-neighbour rows are separate coalesced row loads.  The rows j - 1 and
// j + 1 a wavefront loads are the own rows of the wavefronts beside it in the
// same workgroup, which load them at about the same time on the same CU, so
// they are served by that CU's cache and the L2 instead of being fetched
// again after the L2 has dropped them (RB = 1 leaves that reuse to chance
// across workgroups).
#include "elwh_internal.h"
#include "lanes.h"
#include "step3d_common.h"
#include "xcd.h"

namespace elwh {

template <typename T>
struct Plane {
    T u[3], v[3], w[3];  // rows j-1, j, j+1
    T lam, mu;           // row j
};

template <typename T, bool COMP, bool FORCE, int MODE>
struct Centre3 {
    T a, lam_m, lam_p, mu_m, mu_p;   // a; lambda, mu at rows j-1, j+1 of the plane
    T up[3];
    double h[3];
    float l[3];          // compensation, widened where it is used
    T f[3];
};

template <typename T, typename U, int TZ, int RB, int MODE, bool FORCE, bool COMP>
__global__ __launch_bounds__(64 * RB) void step3d_kernel(const U* __restrict__ u, const T* uprev, T* unext,
                                                   const double* __restrict__ xbase, T* __restrict__ u0out,
                                                   double* __restrict__ acc, float* __restrict__ acclo,
                                                   const T* __restrict__ ca, const T* __restrict__ cl,
                                                   const T* __restrict__ cm, const T* __restrict__ f,
                                                   Args3D A) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // tiles (x-strip, group of RB y-rows, z-chunk) in XCD bands, x fastest
    const int nbx = (A.nx - 1 + 61) / 62, nyg = (A.ny - 1 + RB - 1) / RB;
    const int nzc = (A.khi - A.klo + 1 + TZ - 1) / TZ;
    int t;
    if (!xcd_tile((int)blockIdx.x, nbx * nyg * nzc, t)) return;
    const int i = 62 * (t % nbx) + lane;
    const int j = 1 + ((t / nbx) % nyg) * RB + wave;
    if (j > A.ny - 1) return;   // the last row group is ragged (wavefront-uniform exit)
    const bool colv = i <= A.nx;
    const bool store = lane >= 1 && lane <= 62 && i >= 1 && i <= A.nx - 1;
    const int k0 = A.klo + (t / (nbx * nyg)) * TZ;
    if (k0 > A.khi) return;
    const int k1 = min(k0 + TZ - 1, A.khi);
    const int64_t P = A.P, PS = A.PS, CS = A.CS;
    const T two = (T)2;

    auto load_plane = [&](int k, Plane<T>& q) {
        if (colv && k >= 0 && k <= A.nz) {
            const int64_t o = (int64_t)k * PS + (int64_t)j * P + i;
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                const int64_t orow = o + (int64_t)(r - 1) * P;
                q.u[r] = (T)u[orow];
                q.v[r] = (T)u[orow + CS];
                q.w[r] = (T)u[orow + 2 * CS];
            }
            q.lam = cl[o];
            q.mu = cm[o];
        } else {
#pragma unroll
            for (int r = 0; r < 3; ++r) q.u[r] = q.v[r] = q.w[r] = (T)0;
            q.lam = q.mu = (T)0;
        }
    };
    using Ctr = Centre3<T, COMP, FORCE, MODE>;
    auto load_ctr = [&](int k, Ctr& c) {
        if (colv && k <= A.khi) {
            const int64_t o = (int64_t)k * PS + (int64_t)j * P + i;
            c.a = ca[o];
            c.lam_m = cl[o - P];
            c.lam_p = cl[o + P];
            c.mu_m = cm[o - P];
            c.mu_p = cm[o + P];
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                if constexpr (MODE == 0) {
                    c.up[q] = uprev[o + q * CS];
                    c.h[q] = acc[o + q * CS];
                    if constexpr (COMP) c.l[q] = acclo[o + q * CS];
                } else {
                    c.h[q] = xbase ? xbase[o + q * CS] : 0.0;
                }
                if constexpr (FORCE) c.f[q] = f[o + q * CS];
            }
        } else {
            c.a = c.lam_m = c.lam_p = c.mu_m = c.mu_p = (T)0;
        }
    };

    Plane<T> D, C, Up;
    load_plane(k0 - 1, D);
    load_plane(k0, C);
    load_plane(k0 + 1, Up);
    Ctr ctr;
    load_ctr(k0, ctr);

    for (int k = k0; k <= k1; ++k) {
        // issue the loads of the next plane before computing this one
        Plane<T> Up2;
        Ctr ctrN;
        if (k + 1 <= k1) {
            load_plane(k + 2, Up2);
            load_ctr(k + 1, ctrN);
        }
        const int64_t o = (int64_t)k * PS + (int64_t)j * P + i;
        // the footprint: x neighbours by lane moves (all lanes take part)
        Nb3<T> nb;
        nb.uc = C.u[1]; nb.vc = C.v[1]; nb.wc = C.w[1];
        nb.uL = lane_from_left(C.u[1]); nb.uR = lane_from_right(C.u[1]);
        nb.vL = lane_from_left(C.v[1]); nb.vR = lane_from_right(C.v[1]);
        nb.wL = lane_from_left(C.w[1]); nb.wR = lane_from_right(C.w[1]);
        nb.u0 = C.u[0]; nb.u2 = C.u[2]; nb.v0 = C.v[0]; nb.v2 = C.v[2]; nb.w0 = C.w[0]; nb.w2 = C.w[2];
        nb.u_mL = lane_from_left(C.u[0]); nb.u_mR = lane_from_right(C.u[0]);
        nb.u_pL = lane_from_left(C.u[2]); nb.u_pR = lane_from_right(C.u[2]);
        nb.v_mL = lane_from_left(C.v[0]); nb.v_mR = lane_from_right(C.v[0]);
        nb.v_pL = lane_from_left(C.v[2]); nb.v_pR = lane_from_right(C.v[2]);
        nb.Du = D.u[1]; nb.Dv = D.v[1]; nb.Dw = D.w[1];
        nb.Dv0 = D.v[0]; nb.Dv2 = D.v[2]; nb.Dw0 = D.w[0]; nb.Dw2 = D.w[2];
        nb.u_DL = lane_from_left(D.u[1]); nb.u_DR = lane_from_right(D.u[1]);
        nb.w_DL = lane_from_left(D.w[1]); nb.w_DR = lane_from_right(D.w[1]);
        nb.Uu = Up.u[1]; nb.Uv = Up.v[1]; nb.Uw = Up.w[1];
        nb.Uv0 = Up.v[0]; nb.Uv2 = Up.v[2]; nb.Uw0 = Up.w[0]; nb.Uw2 = Up.w[2];
        nb.u_UL = lane_from_left(Up.u[1]); nb.u_UR = lane_from_right(Up.u[1]);
        nb.w_UL = lane_from_left(Up.w[1]); nb.w_UR = lane_from_right(Up.w[1]);
        nb.lc = C.lam; nb.mc = C.mu;
        nb.lamL = lane_from_left(C.lam); nb.lamR = lane_from_right(C.lam);
        nb.muL = lane_from_left(C.mu); nb.muR = lane_from_right(C.mu);
        nb.lam_m = ctr.lam_m; nb.lam_p = ctr.lam_p; nb.mu_m = ctr.mu_m; nb.mu_p = ctr.mu_p;
        nb.lD = D.lam; nb.mD = D.mu; nb.lU = Up.lam; nb.mU = Up.mu;
        T Lu, Lv, Lw;
        stencil3d(nb, k, A, Lu, Lv, Lw);
        const T uc = nb.uc, vc = nb.vc, wc = nb.wc;

        if (store) {
            const T a = ctr.a;
            if constexpr (FORCE) {
                const T fc = (T)A.fc;
                Lu -= fc * ctr.f[0];
                Lv -= fc * ctr.f[1];
                Lw -= fc * ctr.f[2];
            }
            const T Ls[3] = {Lu, Lv, Lw};
            const T cs[3] = {uc, vc, wc};
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const int64_t oq = o + q * CS;
                T nq;
                double hq = ctr.h[q], lq = 0.0;
                if constexpr (MODE == 0) {
                    nq = two * cs[q] - ctr.up[q] + a * Ls[q];
                    if constexpr (COMP) lq = ctr.l[q];
                } else {
                    nq = cs[q] + (T)0.5 * a * Ls[q];
                    acc_add3(hq, lq, A.w0 * (double)cs[q], COMP);
                    if (u0out) u0out[oq] = cs[q];
                }
                unext[oq] = nq;
                acc_add3(hq, lq, A.w * (double)nq, COMP);
                if (COMP && A.final_) {
                    acc[oq] = hq + lq;
                } else {
                    acc[oq] = hq;
                    if constexpr (COMP) acclo[oq] = (float)lq;
                }
            }
        }
        D = C;
        C = Up;
        if (k + 1 <= k1) {
            Up = Up2;
            ctr = ctrN;
        }
    }
}

template <typename T, typename U, int TZ, int RB, int MODE>
static void launch3_t(bool force, bool comp, dim3 grid, hipStream_t s, const U* u, const T* uprev, T* unext,
                      const double* xbase, T* u0out, double* acc, float* acclo, const T* ca, const T* cl,
                      const T* cm, const T* f, const Args3D& A) {
#define ELWH_L3(F, CMP)                                                                                          \
    hipLaunchKernelGGL((step3d_kernel<T, U, TZ, RB, MODE, F, CMP>), grid, dim3(64 * RB), 0, s, u, uprev, unext, \
                       xbase, u0out, acc, acclo, ca, cl, cm, f, A)
    if (force) {
        if (comp) ELWH_L3(true, true); else ELWH_L3(true, false);
    } else {
        if (comp) ELWH_L3(false, true); else ELWH_L3(false, false);
    }
#undef ELWH_L3
}

// 3-D tiling: V = y rows per workgroup (one wavefront each), TZ = planes
// marched per wavefront.
bool tile_valid_3d(bool fp32, int V, int TZ) {
    (void)fp32;
    return (V == 1 || V == 2 || V == 4 || V == 8) && (TZ == 4 || TZ == 8 || TZ == 16 || TZ == 32);
}

template <typename T, typename U, int MODE>
static void launch3_z(int RB, int TZ, bool force, bool comp, const Args3D& A, hipStream_t s, const U* u,
                      const T* uprev, T* unext, const double* xbase, T* u0out, double* acc, float* acclo,
                      const T* ca, const T* cl, const T* cm, const T* f) {
    const int nplanes = A.khi - A.klo + 1;
    auto grid = [&](int rb, int tz) {
        const int nyg = (A.ny - 1 + rb - 1) / rb;
        return dim3((unsigned)xcd_grid(((A.nx - 1 + 61) / 62) * nyg * ((nplanes + tz - 1) / tz)), 1, 1);
    };
    // the half step (MODE 1) runs once per application: one wavefront per block
    if constexpr (MODE == 1) RB = 1;
#define ELWH_Z(RR, TT)                                                                                           \
    if (RB == RR && TZ == TT) {                                                                                  \
        launch3_t<T, U, TT, RR, MODE>(force, comp, grid(RR, TT), s, u, uprev, unext, xbase, u0out, acc, acclo, ca, \
                                      cl, cm, f, A);                                                             \
        return;                                                                                                  \
    }
    ELWH_Z(1, 4) ELWH_Z(1, 8) ELWH_Z(1, 16) ELWH_Z(1, 32)
    if constexpr (MODE == 0) {
        ELWH_Z(2, 4) ELWH_Z(2, 8) ELWH_Z(2, 16) ELWH_Z(2, 32)
        ELWH_Z(4, 4) ELWH_Z(4, 8) ELWH_Z(4, 16) ELWH_Z(4, 32)
        ELWH_Z(8, 4) ELWH_Z(8, 8) ELWH_Z(8, 16) ELWH_Z(8, 32)
    }
#undef ELWH_Z
    launch3_t<T, U, 16, 1, MODE>(force, comp, grid(1, 16), s, u, uprev, unext, xbase, u0out, acc, acclo, ca, cl, cm,
                                 f, A);
}

// The two state buffers of bufs[0..3] that are neither a nor b.
template <typename T>
static void free_pair3(T* const* bufs, const void* a, const void* b, T** x, T** y) {
    T* got[2] = {nullptr, nullptr};
    int k = 0;
    for (int i = 0; i < 4 && k < 2; ++i)
        if (bufs[i] != a && bufs[i] != b) got[k++] = bufs[i];
    *x = got[0];
    *y = got[1];
}

// Steps 1 .. nsteps-1 after the half step: two-step launches while two or
// more steps remain (fuse >= 2), then single steps.  prev/cur hold u^0/u^1 on
// entry; prev may be the caller's vector (never written).  With fuse = 1 the
// single steps alternate between two buffers as before.
template <typename T>
static void run_steps_3d(elwh_ctx* c, Args3D A, int RB1, int TZ, bool k2, int RB2, bool with_force, bool comp,
                         double sgn, const T* prev, T* cur, T* const* bufs, double* acc, float* lo, const T* ca,
                         const T* cl, const T* cm, const T* f, int nsteps) {
    hipStream_t s = c->stream;
    int n = 1;
    if (k2) {
        while (nsteps - n >= 2) {
            T *x1, *x2;
            free_pair3(bufs, prev, cur, &x1, &x2);
            A.w = sgn * c->w[n + 1];
            A.fc = c->cosn[n];
            A.w1 = sgn * c->w[n + 2];
            A.fc1 = c->cosn[n + 1];
            A.final_ = (n + 2 == nsteps);
            launch_step3d_k2<T>(RB2, TZ, with_force, comp, s, cur, prev, x1, x2, acc, lo, ca, cl, cm, f, A);
            prev = x1;
            cur = x2;
            n += 2;
        }
    }
    for (; n < nsteps; ++n) {
        // u^{n+1} overwrites u^{n-1} when that is one of the state buffers
        T* nxt = nullptr;
        for (int i = 0; i < 4; ++i)
            if (bufs[i] && bufs[i] == prev) nxt = bufs[i];
        if (!nxt) {
            T* dummy;
            free_pair3(bufs, prev, cur, &nxt, &dummy);
        }
        A.w = sgn * c->w[n + 1];
        A.fc = c->cosn[n];
        A.final_ = (n == nsteps - 1);
        launch3_z<T, T, 0>(RB1, TZ, with_force, comp, A, s, cur, prev, nxt, nullptr, nullptr, acc, lo, ca, cl, cm, f);
        prev = cur;
        cur = nxt;
    }
}

void run_filter_3d(elwh_ctx* c, const double* x, bool with_force, bool amode, bool fp32, double* out) {
    hipStream_t s = c->stream;
    Args3D A;
    A.nx = c->L.nx;
    A.ny = c->L.ny;
    A.nz = c->L.nz;
    A.P = c->L.P;
    A.PS = c->L.PS;
    A.CS = c->L.CS;
    A.klo = c->mr.lo;
    A.khi = c->mr.hi;
    A.free_lo = c->mr.free_lo;
    A.free_hi = c->mr.free_hi;
    A.cxx2 = c->st.cxx2;
    A.cyy2 = c->st.cyy2;
    A.czz2 = c->st.czz2;
    A.cxy = c->st.cxy;
    A.cxz = c->st.cxz;
    A.cyz = c->st.cyz;
    A.czzf = c->st.czzf;
    A.cfxz = c->st.cfxz;
    A.cfyz = c->st.cfyz;
    A.w1 = A.fc1 = 0.0;
    A.final_ = 0;
    const Tile tk = fp32 ? c->tile32 : c->tile64;
    // with fuse >= 2 the tile holds the two-step tiling (RB 2, 4, 6), or RB 1
    // for single steps throughout; the half step and a single remaining step
    // take a single-step tiling of the same TZ
    const bool k2 = c->opts.fuse >= 2 && tk.V >= 2;
    const int TZ = tk.TY;
    const int RB1 = k2 ? (tile_valid_3d(fp32, tk.V, TZ) ? tk.V : 2) : tk.V;
    const int nsteps = c->plan.nt * c->opts.periods;
    const double sgn = amode ? -1.0 : 1.0;
    const bool comp = fp32 && c->opts.compensated;
    double* acc = out;
    float* lo = c->acc_lo;
    A.w0 = sgn * c->w[0];
    A.w = sgn * c->w[1];
    A.fc = c->cosn[0];
    if (!fp32) {
        double* b1 = c->s64[1];
        prof_mark(c, 0);
        launch3_z<double, double, 1>(RB1, TZ, with_force, false, A, s, x, nullptr, b1, amode ? x : nullptr, nullptr,
                                     acc, lo, c->ca, c->cl, c->cm, c->f64);
        prof_mark(c, 1);
        run_steps_3d<double>(c, A, RB1, TZ, k2, tk.V, with_force, false, sgn, x, b1, c->s64, acc, lo, c->ca, c->cl,
                             c->cm, c->f64, nsteps);
    } else {
        float *b0 = c->s32[0], *b1 = c->s32[1];
        prof_mark(c, 0);
        launch3_z<float, double, 1>(RB1, TZ, with_force, comp, A, s, x, nullptr, b1, amode ? x : nullptr, b0, acc,
                                    lo, c->fa, c->fl, c->fm, c->f32);
        prof_mark(c, 1);
        run_steps_3d<float>(c, A, RB1, TZ, k2, tk.V, with_force, comp, sgn, b0, b1, c->s32, acc, lo, c->fa, c->fl,
                            c->fm, c->f32, nsteps);
    }
    prof_mark(c, 2, nsteps - 1);
}

}  // namespace elwh
