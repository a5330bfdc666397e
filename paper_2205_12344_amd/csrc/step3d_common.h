// The 3-D conservative stress divergence at one node (shared by the
// single-step and the two-step 3-D kernels).
//
// For the u-row
//   D+x(Abar D-x u) + D+y(mubar D-y u) + D+z(mubar D-z u)
//   + D0x(lam D0y v) + D0y(mu D0x v) + D0x(lam D0z w) + D0z(mu D0x w)
// and cyclically for v and w (a 19-point footprint), A = lam + 2 mu.
// Traction-free z faces are closed from the discrete energy (one-sided
// normal differences, the trapezoid weight 1/2 divided out).  The caller
// gathers the footprint into an Nb3 (from registers and lane moves, or from
// LDS) and gets Lu, Lv, Lw.
#pragma once
#include <hip/hip_runtime.h>

namespace elwh {

struct Args3D {
    int nx, ny, nz;
    int64_t P, PS, CS;
    int klo, khi, free_lo, free_hi;
    double cxx2, cyy2, czz2, cxy, cxz, cyz, czzf, cfxz, cfyz;
    double w, w0, fc;
    double w1, fc1;   // two-step launch: weight of u^{n+2}, forcing factor of step n+1
    int final_;
};

// The footprint of the stencil at node (i, j, k): C = plane k, D = k - 1,
// U = k + 1; rows 0, 1, 2 = j - 1, j, j + 1; L, R = i - 1, i + 1.
template <typename T>
struct Nb3 {
    // displacement, plane k
    T uc, vc, wc, uL, uR, vL, vR, wL, wR;
    T u0, u2, v0, v2, w0, w2;                 // rows j -+ 1, centre
    T u_mL, u_mR, u_pL, u_pR, v_mL, v_mR, v_pL, v_pR;
    // plane k - 1 and k + 1
    T Du, Dv, Dw, Dv0, Dv2, Dw0, Dw2, u_DL, u_DR, w_DL, w_DR;
    T Uu, Uv, Uw, Uv0, Uv2, Uw0, Uw2, u_UL, u_UR, w_UL, w_UR;
    // lambda, mu: plane k row j (centre, x neighbours), rows j -+ 1, planes k -+ 1
    T lc, mc, lamL, lamR, muL, muR, lam_m, lam_p, mu_m, mu_p, lD, mD, lU, mU;
};

template <typename T>
__device__ __forceinline__ void stencil3d(const Nb3<T>& n, int k, const Args3D& A, T& Lu_, T& Lv_, T& Lw_) {
    const T two = (T)2;
    const T cxx2 = (T)A.cxx2, cyy2 = (T)A.cyy2, czz2 = (T)A.czz2;
    const T cxy = (T)A.cxy, cxz = (T)A.cxz, cyz = (T)A.cyz;
    const T czzf = (T)A.czzf, cfxz = (T)A.cfxz, cfyz = (T)A.cfyz;
    const T uc = n.uc, vc = n.vc, wc = n.wc, lc = n.lc, mc = n.mc;
    const T lamL = n.lamL, lamR = n.lamR, muL = n.muL, muR = n.muR;
    const T lam_m = n.lam_m, lam_p = n.lam_p, mu_m = n.mu_m, mu_p = n.mu_p;
    const T AL = lamL + two * muL, AC = lc + two * mc, AR = lamR + two * muR;
    const T Am = lam_m + two * mu_m, Ap = lam_p + two * mu_p;

    // in-plane compact and xy mixed terms (all plane kinds)
    T Lu = cxx2 * ((AR + AC) * (n.uR - uc) - (AC + AL) * (uc - n.uL)) +
           cyy2 * ((mu_p + mc) * (n.u2 - uc) - (mc + mu_m) * (uc - n.u0)) +
           cxy * (lamR * (n.v_pR - n.v_mR) - lamL * (n.v_pL - n.v_mL) + mu_p * (n.v_pR - n.v_pL) -
                  mu_m * (n.v_mR - n.v_mL));
    T Lv = cxx2 * ((muR + mc) * (n.vR - vc) - (mc + muL) * (vc - n.vL)) +
           cyy2 * ((Ap + AC) * (n.v2 - vc) - (AC + Am) * (vc - n.v0)) +
           cxy * (muR * (n.u_pR - n.u_mR) - muL * (n.u_pL - n.u_mL) + lam_p * (n.u_pR - n.u_pL) -
                  lam_m * (n.u_mR - n.u_mL));
    T Lw = cxx2 * ((muR + mc) * (n.wR - wc) - (mc + muL) * (wc - n.wL)) +
           cyy2 * ((mu_p + mc) * (n.w2 - wc) - (mc + mu_m) * (wc - n.w0));

    if (A.free_hi && k == A.nz) {
        const T lD = n.lD, mD = n.mD, AD = lD + two * mD;
        Lu += -czzf * (mc + mD) * (uc - n.Du) - cfxz * (mc * (n.wR - n.wL) + mD * (n.w_DR - n.w_DL)) +
              cfxz * (lamR * (n.wR - n.w_DR) - lamL * (n.wL - n.w_DL));
        Lv += -czzf * (mc + mD) * (vc - n.Dv) - cfyz * (mc * (n.w2 - n.w0) + mD * (n.Dw2 - n.Dw0)) +
              cfyz * (lam_p * (n.w2 - n.Dw2) - lam_m * (n.w0 - n.Dw0));
        Lw += -czzf * (AC + AD) * (wc - n.Dw) - cfxz * (lc * (n.uR - n.uL) + lD * (n.u_DR - n.u_DL)) +
              cfxz * (muR * (n.uR - n.u_DR) - muL * (n.uL - n.u_DL)) -
              cfyz * (lc * (n.v2 - n.v0) + lD * (n.Dv2 - n.Dv0)) +
              cfyz * (mu_p * (n.v2 - n.Dv2) - mu_m * (n.v0 - n.Dv0));
    } else if (A.free_lo && k == 0) {
        const T lU = n.lU, mU = n.mU, AU = lU + two * mU;
        Lu += czzf * (mc + mU) * (n.Uu - uc) + cfxz * (mc * (n.wR - n.wL) + mU * (n.w_UR - n.w_UL)) +
              cfxz * (lamR * (n.w_UR - n.wR) - lamL * (n.w_UL - n.wL));
        Lv += czzf * (mc + mU) * (n.Uv - vc) + cfyz * (mc * (n.w2 - n.w0) + mU * (n.Uw2 - n.Uw0)) +
              cfyz * (lam_p * (n.Uw2 - n.w2) - lam_m * (n.Uw0 - n.w0));
        Lw += czzf * (AC + AU) * (n.Uw - wc) + cfxz * (lc * (n.uR - n.uL) + lU * (n.u_UR - n.u_UL)) +
              cfxz * (muR * (n.u_UR - n.uR) - muL * (n.u_UL - n.uL)) +
              cfyz * (lc * (n.v2 - n.v0) + lU * (n.Uv2 - n.Uv0)) +
              cfyz * (mu_p * (n.Uv2 - n.v2) - mu_m * (n.Uv0 - n.v0));
    } else {
        const T lD = n.lD, mD = n.mD, lU = n.lU, mU = n.mU;
        const T AD = lD + two * mD, AU = lU + two * mU;
        Lu += czz2 * ((mU + mc) * (n.Uu - uc) - (mc + mD) * (uc - n.Du)) +
              cxz * (lamR * (n.w_UR - n.w_DR) - lamL * (n.w_UL - n.w_DL) + mU * (n.w_UR - n.w_UL) -
                     mD * (n.w_DR - n.w_DL));
        Lv += czz2 * ((mU + mc) * (n.Uv - vc) - (mc + mD) * (vc - n.Dv)) +
              cyz * (lam_p * (n.Uw2 - n.Dw2) - lam_m * (n.Uw0 - n.Dw0) + mU * (n.Uw2 - n.Uw0) -
                     mD * (n.Dw2 - n.Dw0));
        Lw += czz2 * ((AU + AC) * (n.Uw - wc) - (AC + AD) * (wc - n.Dw)) +
              cxz * (muR * (n.u_UR - n.u_DR) - muL * (n.u_UL - n.u_DL) + lU * (n.u_UR - n.u_UL) -
                     lD * (n.u_DR - n.u_DL)) +
              cyz * (mu_p * (n.Uv2 - n.Dv2) - mu_m * (n.Uv0 - n.Dv0) + lU * (n.Uv2 - n.Uv0) -
                     lD * (n.Dv2 - n.Dv0));
    }
    Lu_ = Lu;
    Lv_ = Lv;
    Lw_ = Lw;
}

__device__ __forceinline__ void acc_add3(double& hi, double& lo, double x, bool comp) {
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

}  // namespace elwh
