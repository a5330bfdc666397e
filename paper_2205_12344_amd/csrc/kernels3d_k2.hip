// Two time steps per launch on the 3-D Cartesian grid: temporal blocking of
// the fused El-WaveHoltz step (corrected leapfrog of Sec. 4.3 with the
// trapezoid accumulation of eq. el_WHI_OP), the 3-D analogue of the 2-D
// K-step kernel.
//
// A workgroup of RB + 2 wavefronts owns a strip of 64 x nodes of RB + 2
// consecutive y rows (one row per wavefront) and marches a chunk of TZ
// planes in z.  Stage 1 advances every row of the workgroup from u^n to
// u^{n+1} one plane ahead (the rows j0 - 1 and j0 + RB are halo rows: they
// are computed only because stage 2 needs them) and parks the new plane in
// a ring of three LDS planes; stage 2 advances the RB inner rows from
// u^{n+1} to u^{n+2} on the plane behind, reading the 19-point footprint of
// u^{n+1} from that ring (x neighbours at lanes -+ 1, y neighbours in the
// rows of the wavefronts beside it, z neighbours in the other two planes).
// Stage 1 is exact on lanes 1..62, stage 2 on lanes 2..61: a strip computes
// 60 columns.  Per node the launch reads u^n, u^{n-1}, the coefficients and
// the accumulator once and writes u^{n+1}, u^{n+2} and the accumulator once,
// instead of twice each: 168 (FP64) or 132 (FP32 state, compensated FP64
// accumulator with an FP32 compensation word) bytes for two lattice
// updates, against 144 per update.  The
// accumulation order per node (w_{n+1} u^{n+1}, then w_{n+2} u^{n+2}) is that
// of two single steps.
#include "elwh_internal.h"
#include "lanes.h"
#include "step3d_common.h"
#include "xcd.h"

namespace elwh {

namespace {

template <typename T>
struct PlaneK2 {
    T u[3], v[3], w[3];  // rows j-1, j, j+1 of u^n
    T lam, mu;           // row j
};

template <typename T>
struct CtrK2 {
    T a, lam_m, lam_p, mu_m, mu_p;   // a; lambda, mu at rows j -+ 1
    T up[3];                          // u^{n-1}
    T f[3];                           // forcing
};

}  // namespace

template <typename T, int TZ, int RB, bool FORCE, bool COMP>
__global__ __launch_bounds__(64 * (RB + 2)) void step3d_k2_kernel(const T* __restrict__ u, const T* __restrict__ uprev,
                                                                 T* __restrict__ outA, T* __restrict__ outB,
                                                                 double* __restrict__ acc, float* __restrict__ acclo,
                                                                 const T* __restrict__ ca, const T* __restrict__ cl,
                                                                 const T* __restrict__ cm, const T* __restrict__ f,
                                                                 Args3D A) {
    __shared__ T ring[3][RB + 2][3][64];   // u^{n+1}: plane slot, row, component, lane
    const int lane = threadIdx.x & 63, wave = (int)(threadIdx.x >> 6);
    const int nbx = (A.nx - 1 + 59) / 60, nyg = (A.ny - 1 + RB - 1) / RB;
    const int nzc = (A.khi - A.klo + 1 + TZ - 1) / TZ;
    int t;
    // every wavefront of a workgroup reaches every barrier: the exits below
    // are workgroup-uniform
    if (!xcd_tile((int)blockIdx.x, nbx * nyg * nzc, t)) return;
    const int k0 = A.klo + (t / (nbx * nyg)) * TZ;
    if (k0 > A.khi) return;
    const int k1 = min(k0 + TZ - 1, A.khi);
    const int i = 60 * (t % nbx) - 1 + lane;          // lane 2 -> first column of the strip
    const int j = ((t / nbx) % nyg) * RB + wave;      // wave 1 -> first row of the group
    const int64_t P = A.P, PS = A.PS, CS = A.CS;
    const bool inner = wave >= 1 && wave <= RB;
    const bool xin1 = lane >= 1 && lane <= 62 && i >= 1 && i <= A.nx - 1;   // stage 1 exact here
    const bool xin2 = lane >= 2 && lane <= 61 && i >= 1 && i <= A.nx - 1;   // stage 2 output
    const bool yin = j >= 1 && j <= A.ny - 1;
    const T two = (T)2;

    // Loads outside the grid are masked and read 0.  (Unconditional loads at
    // clamped indices were measured: they save the zero fills but let the
    // compiler hoist loads across the march, and the extra registers cost
    // more than the fills.)
    const bool colv = i >= 0 && i <= A.nx;
    auto load_plane = [&](int k, PlaneK2<T>& q) {
        const bool kv = colv && k >= 0 && k <= A.nz;
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            const int jr = j + r - 1;
            const bool ok = kv && jr >= 0 && jr <= A.ny;
            T a = (T)0, b = (T)0, c = (T)0;
            if (ok) {
                const int64_t orow = (int64_t)k * PS + (int64_t)jr * P + i;
                a = u[orow];
                b = u[orow + CS];
                c = u[orow + 2 * CS];
            }
            q.u[r] = a;
            q.v[r] = b;
            q.w[r] = c;
        }
        T l = (T)0, m = (T)0;
        if (kv && j >= 0 && j <= A.ny) {
            const int64_t o = (int64_t)k * PS + (int64_t)j * P + i;
            l = cl[o];
            m = cm[o];
        }
        q.lam = l;
        q.mu = m;
    };
    auto unk = [&](int k) { return xin1 && yin && k >= A.klo && k <= A.khi; };
    auto load_ctr = [&](int k, CtrK2<T>& c) {
        T a = (T)0, lm = (T)0, lp = (T)0, mm = (T)0, mp = (T)0;
        T u0 = (T)0, u1 = (T)0, u2 = (T)0, f0 = (T)0, f1 = (T)0, f2 = (T)0;
        if (unk(k)) {
            const int64_t o = (int64_t)k * PS + (int64_t)j * P + i;
            a = ca[o];
            lm = cl[o - P];
            lp = cl[o + P];
            mm = cm[o - P];
            mp = cm[o + P];
            u0 = uprev[o];
            u1 = uprev[o + CS];
            u2 = uprev[o + 2 * CS];
            if constexpr (FORCE) {
                f0 = f[o];
                f1 = f[o + CS];
                f2 = f[o + 2 * CS];
            }
        }
        c.a = a;
        c.lam_m = lm;
        c.lam_p = lp;
        c.mu_m = mm;
        c.mu_p = mp;
        c.up[0] = u0;
        c.up[1] = u1;
        c.up[2] = u2;
        c.f[0] = f0;
        c.f[1] = f1;
        c.f[2] = f2;
    };

    // the accumulator at the stage-2 node of plane k, read one iteration early
    // (FP32 state only: the FP64 instances have no registers to spare)
    constexpr bool PF = sizeof(T) == 4;
    // (masked: the accumulator is written in this launch, and only a lane's
    // own stage-2 node is its to read)
    // (the compensation words stay FP32 until they are used: converting at
    // the load would wait for it there)
    auto load_acc = [&](int k, double* h, float* l) {
        double a0 = 0.0, a1 = 0.0, a2 = 0.0;
        float b0 = 0.0f, b1 = 0.0f, b2 = 0.0f;
        if (inner && xin2 && yin && k >= k0 && k <= k1 && k >= A.klo && k <= A.khi) {
            const int64_t o = (int64_t)k * PS + (int64_t)j * P + i;
            a0 = acc[o];
            a1 = acc[o + CS];
            a2 = acc[o + 2 * CS];
            if constexpr (COMP) {
                b0 = acclo[o];
                b1 = acclo[o + CS];
                b2 = acclo[o + 2 * CS];
            }
        }
        h[0] = a0;
        h[1] = a1;
        h[2] = a2;
        l[0] = b0;
        l[1] = b1;
        l[2] = b2;
    };
    // The z-march keeps four planes of u^n (D, C, Up = kk - 1, kk, kk + 1 and
    // Up2 = kk + 2, in flight), three centre records (prv, ctr, ctrN = kk - 1,
    // kk, kk + 1) and two accumulator records.  (Unrolling the march to rename
    // them instead of copying was measured: it needs more registers than it
    // saves moves.)
    using Acc3 = double[3];
    using Lo3 = float[3];
    T Dp_lam = (T)0, Dp_mu = (T)0;   // lambda, mu of plane kk - 2 (row j)
    const int kA = k0 - 1, kB = k1 + 1;

    auto sub = [&](const int kk, PlaneK2<T>& D, PlaneK2<T>& C, PlaneK2<T>& Up, PlaneK2<T>& Up2, CtrK2<T>& prv,
                   CtrK2<T>& ctr, CtrK2<T>& ctrN, Acc3& accH, Lo3& accL, Acc3& accHN, Lo3& accLN) {
        if (kk + 1 <= kB) {
            load_plane(kk + 2, Up2);
            load_ctr(kk + 1, ctrN);
        }
        if constexpr (PF) load_acc(kk, accHN, accLN);
        // ---- stage 1: u^{n+1} on plane kk (every row of the workgroup) ----
        T n1[3] = {(T)0, (T)0, (T)0};
        {
            Nb3<T> nb;
            nb.uc = C.u[1]; nb.vc = C.v[1]; nb.wc = C.w[1];
            nb.uL = lane_from_left_z(C.u[1]); nb.uR = lane_from_right_z(C.u[1]);
            nb.vL = lane_from_left_z(C.v[1]); nb.vR = lane_from_right_z(C.v[1]);
            nb.wL = lane_from_left_z(C.w[1]); nb.wR = lane_from_right_z(C.w[1]);
            nb.u0 = C.u[0]; nb.u2 = C.u[2]; nb.v0 = C.v[0]; nb.v2 = C.v[2]; nb.w0 = C.w[0]; nb.w2 = C.w[2];
            nb.u_mL = lane_from_left_z(C.u[0]); nb.u_mR = lane_from_right_z(C.u[0]);
            nb.u_pL = lane_from_left_z(C.u[2]); nb.u_pR = lane_from_right_z(C.u[2]);
            nb.v_mL = lane_from_left_z(C.v[0]); nb.v_mR = lane_from_right_z(C.v[0]);
            nb.v_pL = lane_from_left_z(C.v[2]); nb.v_pR = lane_from_right_z(C.v[2]);
            nb.Du = D.u[1]; nb.Dv = D.v[1]; nb.Dw = D.w[1];
            nb.Dv0 = D.v[0]; nb.Dv2 = D.v[2]; nb.Dw0 = D.w[0]; nb.Dw2 = D.w[2];
            nb.u_DL = lane_from_left_z(D.u[1]); nb.u_DR = lane_from_right_z(D.u[1]);
            nb.w_DL = lane_from_left_z(D.w[1]); nb.w_DR = lane_from_right_z(D.w[1]);
            nb.Uu = Up.u[1]; nb.Uv = Up.v[1]; nb.Uw = Up.w[1];
            nb.Uv0 = Up.v[0]; nb.Uv2 = Up.v[2]; nb.Uw0 = Up.w[0]; nb.Uw2 = Up.w[2];
            nb.u_UL = lane_from_left_z(Up.u[1]); nb.u_UR = lane_from_right_z(Up.u[1]);
            nb.w_UL = lane_from_left_z(Up.w[1]); nb.w_UR = lane_from_right_z(Up.w[1]);
            nb.lc = C.lam; nb.mc = C.mu;
            nb.lamL = lane_from_left_z(C.lam); nb.lamR = lane_from_right_z(C.lam);
            nb.muL = lane_from_left_z(C.mu); nb.muR = lane_from_right_z(C.mu);
            nb.lam_m = ctr.lam_m; nb.lam_p = ctr.lam_p; nb.mu_m = ctr.mu_m; nb.mu_p = ctr.mu_p;
            nb.lD = D.lam; nb.mD = D.mu; nb.lU = Up.lam; nb.mU = Up.mu;
            T L[3];
            stencil3d(nb, kk, A, L[0], L[1], L[2]);
            if (unk(kk)) {
                const T cs[3] = {C.u[1], C.v[1], C.w[1]};
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    T Lq = L[q];
                    if constexpr (FORCE) Lq -= (T)A.fc * ctr.f[q];
                    n1[q] = two * cs[q] - ctr.up[q] + ctr.a * Lq;
                }
                if (inner && xin2 && kk >= k0 && kk <= k1) {
                    const int64_t o = (int64_t)kk * PS + (int64_t)j * P;
#pragma unroll
                    for (int q = 0; q < 3; ++q) outA[o + q * CS + i] = n1[q];
                }
            }
        }
        const int s1 = ((kk % 3) + 3) % 3;
#pragma unroll
        for (int q = 0; q < 3; ++q) ring[s1][wave][q][lane] = n1[q];
        // lambda, mu of plane kk - 1 (row j, x neighbours) for stage 2: every
        // lane takes part in the lane moves
        const T pl = D.lam, pm = D.mu;
        const T plL = lane_from_left_z(pl), plR = lane_from_right_z(pl);
        const T pmL = lane_from_left_z(pm), pmR = lane_from_right_z(pm);
        __syncthreads();
        // ---- stage 2: u^{n+2} on plane k = kk - 1 (inner rows) ----
        const int k = kk - 1;
        if (inner && k >= k0) {
            if (xin2 && yin && k >= A.klo && k <= A.khi) {
                const int sD = (((k - 1) % 3) + 3) % 3, sC = (((k % 3) + 3) % 3), sU = s1;
                const int lL = lane - 1, lR = lane + 1;   // lanes 2..61 here: in range
                auto R = [&](int sl, int row, int q, int ln) { return ring[sl][row][q][ln]; };
                Nb3<T> nb;
                nb.uc = R(sC, wave, 0, lane); nb.vc = R(sC, wave, 1, lane); nb.wc = R(sC, wave, 2, lane);
                nb.uL = R(sC, wave, 0, lL); nb.uR = R(sC, wave, 0, lR);
                nb.vL = R(sC, wave, 1, lL); nb.vR = R(sC, wave, 1, lR);
                nb.wL = R(sC, wave, 2, lL); nb.wR = R(sC, wave, 2, lR);
                nb.u0 = R(sC, wave - 1, 0, lane); nb.u2 = R(sC, wave + 1, 0, lane);
                nb.v0 = R(sC, wave - 1, 1, lane); nb.v2 = R(sC, wave + 1, 1, lane);
                nb.w0 = R(sC, wave - 1, 2, lane); nb.w2 = R(sC, wave + 1, 2, lane);
                nb.u_mL = R(sC, wave - 1, 0, lL); nb.u_mR = R(sC, wave - 1, 0, lR);
                nb.u_pL = R(sC, wave + 1, 0, lL); nb.u_pR = R(sC, wave + 1, 0, lR);
                nb.v_mL = R(sC, wave - 1, 1, lL); nb.v_mR = R(sC, wave - 1, 1, lR);
                nb.v_pL = R(sC, wave + 1, 1, lL); nb.v_pR = R(sC, wave + 1, 1, lR);
                nb.Du = R(sD, wave, 0, lane); nb.Dv = R(sD, wave, 1, lane); nb.Dw = R(sD, wave, 2, lane);
                nb.Dv0 = R(sD, wave - 1, 1, lane); nb.Dv2 = R(sD, wave + 1, 1, lane);
                nb.Dw0 = R(sD, wave - 1, 2, lane); nb.Dw2 = R(sD, wave + 1, 2, lane);
                nb.u_DL = R(sD, wave, 0, lL); nb.u_DR = R(sD, wave, 0, lR);
                nb.w_DL = R(sD, wave, 2, lL); nb.w_DR = R(sD, wave, 2, lR);
                nb.Uu = R(sU, wave, 0, lane); nb.Uv = R(sU, wave, 1, lane); nb.Uw = R(sU, wave, 2, lane);
                nb.Uv0 = R(sU, wave - 1, 1, lane); nb.Uv2 = R(sU, wave + 1, 1, lane);
                nb.Uw0 = R(sU, wave - 1, 2, lane); nb.Uw2 = R(sU, wave + 1, 2, lane);
                nb.u_UL = R(sU, wave, 0, lL); nb.u_UR = R(sU, wave, 0, lR);
                nb.w_UL = R(sU, wave, 2, lL); nb.w_UR = R(sU, wave, 2, lR);
                nb.lc = pl; nb.mc = pm;
                nb.lamL = plL; nb.lamR = plR; nb.muL = pmL; nb.muR = pmR;
                nb.lam_m = prv.lam_m; nb.lam_p = prv.lam_p; nb.mu_m = prv.mu_m; nb.mu_p = prv.mu_p;
                nb.lD = Dp_lam; nb.mD = Dp_mu; nb.lU = C.lam; nb.mU = C.mu;
                T L[3];
                stencil3d(nb, k, A, L[0], L[1], L[2]);
                const int64_t o = (int64_t)k * PS + (int64_t)j * P;
                const T n1c[3] = {nb.uc, nb.vc, nb.wc};
                const T n0c[3] = {D.u[1], D.v[1], D.w[1]};
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    T Lq = L[q];
                    if constexpr (FORCE) Lq -= (T)A.fc1 * prv.f[q];
                    const T n2 = two * n1c[q] - n0c[q] + prv.a * Lq;
                    outB[o + q * CS + i] = n2;
                    double hq, lq = 0.0;
                    if constexpr (PF) {
                        hq = accH[q];
                        lq = accL[q];
                    } else {
                        hq = acc[o + q * CS + i];
                        if constexpr (COMP) lq = acclo[o + q * CS + i];
                    }
                    acc_add3(hq, lq, A.w * (double)n1c[q], COMP);
                    acc_add3(hq, lq, A.w1 * (double)n2, COMP);
                    if (COMP && A.final_) {
                        acc[o + q * CS + i] = hq + lq;
                    } else {
                        acc[o + q * CS + i] = hq;
                        if constexpr (COMP) acclo[o + q * CS + i] = (float)lq;
                    }
                }
            }
        }
        __syncthreads();   // the next stage 1 overwrites the ring slot stage 2 read as plane k - 1
        Dp_lam = D.lam;
        Dp_mu = D.mu;
    };

    PlaneK2<T> P0, P1, P2, P3;
    CtrK2<T> Q0, Q1, Q2;
    Acc3 H0 = {0.0, 0.0, 0.0}, H1;
    Lo3 L0 = {0.0f, 0.0f, 0.0f}, L1;
    load_plane(kA - 1, P0);
    load_plane(kA, P1);
    load_plane(kA + 1, P2);
    load_ctr(kA - 1, Q0);
    load_ctr(kA, Q1);
    // (the trip count is uniform over the workgroup: every wavefront reaches
    // every barrier inside a sub-step)
    for (int kk = kA; kk <= kB; ++kk) {
        sub(kk, P0, P1, P2, P3, Q0, Q1, Q2, H0, L0, H1, L1);
        P0 = P1;
        P1 = P2;
        P2 = P3;
        Q0 = Q1;
        Q1 = Q2;
        if constexpr (PF) {
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                H0[q] = H1[q];
                L0[q] = L1[q];
            }
        }
    }
}

// Tilings of a context that takes two steps per launch: RB = 2, 4, 6 rows
// with TZ = 8, 16, 32, 64 planes, or RB = 1, which has no two-step form and runs
// every step as a single-step launch of TZ planes (on some grids, FP64 among
// them, that is the faster choice).
bool tile_valid_3d_k2(bool fp32, int RB, int TZ) {
    if (RB == 1) return tile_valid_3d(fp32, 1, TZ);
    return (RB == 2 || RB == 4 || RB == 6) && (TZ == 8 || TZ == 16 || TZ == 32 || TZ == 64);
}

template <typename T>
void launch_step3d_k2(int RB, int TZ, bool force, bool comp, hipStream_t s, const T* u, const T* uprev, T* outA,
                      T* outB, double* acc, float* acclo, const T* ca, const T* cl, const T* cm, const T* f,
                      const Args3D& A) {
    const int nbx = (A.nx - 1 + 59) / 60;
    auto grid = [&](int rb, int tz) {
        const int nyg = (A.ny - 1 + rb - 1) / rb;
        const int nzc = (A.khi - A.klo + 1 + tz - 1) / tz;
        return dim3((unsigned)xcd_grid(nbx * nyg * nzc));
    };
#define ELWH_K2(RR, TT)                                                                                         \
    if (RB == RR && TZ == TT) {                                                                                 \
        if (force) {                                                                                            \
            if (comp)                                                                                           \
                hipLaunchKernelGGL((step3d_k2_kernel<T, TT, RR, true, true>), grid(RR, TT), dim3(64 * (RR + 2)), \
                                   0, s, u, uprev, outA, outB, acc, acclo, ca, cl, cm, f, A);                  \
            else                                                                                                \
                hipLaunchKernelGGL((step3d_k2_kernel<T, TT, RR, true, false>), grid(RR, TT),                    \
                                   dim3(64 * (RR + 2)), 0, s, u, uprev, outA, outB, acc, acclo, ca, cl, cm, f, A); \
        } else {                                                                                                \
            if (comp)                                                                                           \
                hipLaunchKernelGGL((step3d_k2_kernel<T, TT, RR, false, true>), grid(RR, TT),                    \
                                   dim3(64 * (RR + 2)), 0, s, u, uprev, outA, outB, acc, acclo, ca, cl, cm, f, A); \
            else                                                                                                \
                hipLaunchKernelGGL((step3d_k2_kernel<T, TT, RR, false, false>), grid(RR, TT),                   \
                                   dim3(64 * (RR + 2)), 0, s, u, uprev, outA, outB, acc, acclo, ca, cl, cm, f, A); \
        }                                                                                                       \
        return;                                                                                                 \
    }
    ELWH_K2(2, 8) ELWH_K2(2, 16) ELWH_K2(2, 32) ELWH_K2(2, 64)
    ELWH_K2(4, 8) ELWH_K2(4, 16) ELWH_K2(4, 32) ELWH_K2(4, 64)
    ELWH_K2(6, 8) ELWH_K2(6, 16) ELWH_K2(6, 32) ELWH_K2(6, 64)
#undef ELWH_K2
}

template void launch_step3d_k2<double>(int, int, bool, bool, hipStream_t, const double*, const double*, double*,
                                       double*, double*, float*, const double*, const double*, const double*,
                                       const double*, const Args3D&);
template void launch_step3d_k2<float>(int, int, bool, bool, hipStream_t, const float*, const float*, float*, float*,
                                      double*, float*, const float*, const float*, const float*, const float*,
                                      const Args3D&);

}  // namespace elwh
