// 2-D two-field El-WaveHoltz step for impedance (absorbing) faces, FP64.
//
// The filter of the remark in Sec. 3 acts on the initial displacement and
// velocity together, Pi [u0; u1] = (2/T) int (cos(omega t) - 1/4) [u; u_t] dt.
// One launch advances every unknown node from level n to n+1 of the
// corrected leapfrog (Sec. 4.3) with a centred damping term on the rows of
// the impedance faces,
//     (1 + g) u^{n+1} = 2 u^n - (1 - g) u^{n-1} + a (Ltilde u^n - f cos(omega t_n)),
// g = c dt Bt / 2 per node and component (zero away from those rows), and
// adds w_{n+1} u^{n+1} to the displacement accumulator and
// w_n (u^{n+1} - u^{n-1}) / (2 dt) -- the centred velocity of level n -- to
// the velocity accumulator.  The start launch takes u^1 = u^0 + dt (1 - g) u1
// + (a/2) (Ltilde u^0 - f) from the two fields and seeds the accumulators
// with w_0 u^0 + w_1 u^1 and w_0 u1 (or the A_h bases x - ...).  One extra
// step beyond the window supplies the velocity of the last level.
//
// The impedance face is a traction-type face of the discrete energy
// (Sec. 4.1): on the y faces the stencil rows are the traction-free closure
// of the one-field kernels; on an impedance x face the face column's rows
// (corners included) are the energy gradient evaluated directly, by extra
// blocks of the same launch (one row per lane) so that the strip march keeps
// its registers, while the rows one column inside keep the interior stencil
// (the x face's half weight and its one-sided difference cancel there).  The
// damping values are per node of the face rows and columns; at a corner the
// two faces' terms add.
// Mapping and loads are those of the one-field single-step kernel: one
// 64-lane wavefront per x-strip of 64 V columns, TY rows marched upward with
// the three stencil rows in registers and the next row's loads issued one
// iteration ahead.
#include "step2d_common.h"

namespace elwh {

namespace {

// Ltilde at a node of an impedance (traction-type) x face, column i with
// inward neighbour column i + d (d = +1 on the -x face, -1 on the +x face),
// from the discrete energy: compact terms with the edge-to-node weight
// ratio (2 across the x face, and 2 along y on a free y face), and the cross
// terms lambda X(u) Y(v) + mu Y(u) X(v) of the nodes whose differences
// involve this one -- the node itself, its inward neighbour and its
// neighbours along the face -- each with its trapezoid weight, X one-sided
// on the face column and central inside, Y one-sided on free y faces.
// S, C, N: rows j-1, j, j+1 at column i; Si, Ci, Ni: the same at column
// i + d (lI, mI the inward node's lambda, mu).
__device__ __forceinline__ void xface_rows(double d, int j, int ny, bool free_lo, bool free_hi, double cxx2,
                                           double cyy2, double hx, double hy, double uS, double uC, double uN,
                                           double vS, double vC, double vN, double uSi, double uCi, double uNi,
                                           double vSi, double vCi, double vNi, double lS, double lC, double lN,
                                           double mS, double mC, double mN, double lI, double mI, double& Lu,
                                           double& Lv) {
    const bool onlo = free_lo && j == 0, onhi = free_hi && j == ny, onface = onlo || onhi;
    const bool hasS = j > 0, hasN = j < ny;
    const double fy = onface ? 2.0 : 1.0;
    const double AC = lC + 2.0 * mC, AI = lI + 2.0 * mI, AS = lS + 2.0 * mS, AN = lN + 2.0 * mN;
    double cu = 2.0 * cxx2 * (AI + AC) * (uCi - uC);
    double cv = 2.0 * cxx2 * (mI + mC) * (vCi - vC);
    if (hasN) {
        cu += fy * cyy2 * (mN + mC) * (uN - uC);
        cv += fy * cyy2 * (AN + AC) * (vN - vC);
    }
    if (hasS) {
        cu -= fy * cyy2 * (mC + mS) * (uC - uS);
        cv -= fy * cyy2 * (AC + AS) * (vC - vS);
    }
    auto ydiff = [&](double fs, double fc, double fn, int jj) {
        if (free_lo && jj == 0) return (fn - fc) / hy;
        if (free_hi && jj == ny) return (fc - fs) / hy;
        return (fn - fs) / (2.0 * hy);
    };
    const double wp = onface ? 0.25 : 0.5, wI = onface ? 0.5 : 1.0;
    const double cXp = -d / hx, cXi = -d / (2.0 * hx);
    const double cYp = onlo ? -1.0 / hy : (onhi ? 1.0 / hy : 0.0);
    double xu = wp * (lC * cXp * ydiff(vS, vC, vN, j) + mC * cYp * d * (vCi - vC) / hx);
    double xv = wp * (lC * d * (uCi - uC) / hx * cYp + mC * ydiff(uS, uC, uN, j) * cXp);
    xu += wI * lI * cXi * ydiff(vSi, vCi, vNi, j);
    xv += wI * mI * ydiff(uSi, uCi, uNi, j) * cXi;
    if (hasN && !(j + 1 == ny && !free_hi)) {
        const bool on = free_hi && j + 1 == ny;
        const double wN = on ? 0.25 : 0.5, cY = on ? -1.0 / hy : -0.5 / hy;
        xu += wN * mN * cY * d * (vNi - vN) / hx;
        xv += wN * lN * d * (uNi - uN) / hx * cY;
    }
    if (hasS && !(j - 1 == 0 && !free_lo)) {
        const bool on = free_lo && j - 1 == 0;
        const double wS = on ? 0.25 : 0.5, cY = on ? 1.0 / hy : 0.5 / hy;
        xu += wS * mS * cY * d * (vSi - vS) / hx;
        xv += wS * lS * d * (uSi - uS) / hx * cY;
    }
    Lu = cu - xu / wp;
    Lv = cv - xv / wp;
}

template <int V, int MODE, bool FORCE>
struct DCentre {
    double a[V];
    double up[V], vp[V];        // u^{n-1} (MODE 0) or the second field u1 (MODE 1)
    double h0u[V], h0v[V];      // displacement accumulator (MODE 0) or its base (MODE 1)
    double h1u[V], h1v[V];      // velocity accumulator (MODE 0) or its base (MODE 1)
    double fu[V], fv[V];
};

template <int V, int TY, int MODE, bool FORCE>
__device__ __forceinline__ void damped2d_body(int bx, int by, const double* __restrict__ u, const double* uprev,
                                              double* unext, const double* __restrict__ base0,
                                              const double* __restrict__ base1, double* __restrict__ acc0,
                                              double* __restrict__ acc1, const double* __restrict__ dmp,
                                              const double* __restrict__ dmpx, const double* __restrict__ ca,
                                              const double* __restrict__ cl, const double* __restrict__ cm,
                                              const double* __restrict__ f, const Damp2D& D) {
    using T = double;
    const Args2D& A = D.A;
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
    const T cxx2 = A.cxx2, cyy2 = A.cyy2, cxy = A.cxy, cyyf = A.cyyf, cfx = A.cfx;
    const int ilo = max(c0 + 1, 1), ihi = min(c0 + W, A.nx - 1);   // columns 1..nx-1

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
    using Ctr = DCentre<V, MODE, FORCE>;
    auto load_ctr = [&](int j, Ctr& c) {
        if (colv && j <= A.jhi) {
            const int64_t o = (int64_t)j * P + col;
            vload<T, T, V>(ca + o, c.a);
            vload<T, T, V>(uprev + o, c.up);
            vload<T, T, V>(uprev + o + CS, c.vp);
            const double* b0 = MODE == 0 ? acc0 : base0;
            const double* b1 = MODE == 0 ? acc1 : base1;
            if (b0) {
                vload<T, T, V>(b0 + o, c.h0u);
                vload<T, T, V>(b0 + o + CS, c.h0v);
            } else {
                vzero<T, V>(c.h0u);
                vzero<T, V>(c.h0v);
            }
            if (b1) {
                vload<T, T, V>(b1 + o, c.h1u);
                vload<T, T, V>(b1 + o + CS, c.h1v);
            } else {
                vzero<T, V>(c.h1u);
                vzero<T, V>(c.h1v);
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
        RawRow<T, V> rawNN;
        Ctr ctrN;
        if (j + 1 <= j1) {
            load_raw(j + 2, rawNN);
            load_ctr(j + 1, ctrN);
        }
        finish(rawN, N);
        const T lamL0 = lane_from_left(C.l[V - 1]), lamR0 = lane_from_right(C.l[0]);
        const T muL0 = lane_from_left(C.m[V - 1]), muR0 = lane_from_right(C.m[0]);
        const int kind = (A.free_hi && j == A.ny) ? 1 : ((A.free_lo && j == 0) ? 2 : 0);
        // damping rows: dmp[0], dmp[1] (u, v) of the low face, dmp[2], dmp[3] of the high face
        const bool damped = (kind == 1 && D.imp_hi) || (kind == 2 && D.imp_lo);
        const double* gu_row = dmp + (int64_t)(kind == 1 ? 2 : 0) * P;
        const double* gv_row = gu_row + P;
        const int64_t o = (int64_t)j * P + col;

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
                Lu -= A.fc * ctr.fu[k];
                Lv -= A.fc * ctr.fv[k];
            }
            const T a = ctr.a[k];
            const double gu = damped ? gu_row[i] : 0.0, gv = damped ? gv_row[i] : 0.0;
            T nu, nv, h0u, h0v, h1u, h1v;
            if constexpr (MODE == 0) {
                nu = 2.0 * cc.u - ctr.up[k] + a * Lu;
                nv = 2.0 * cc.v - ctr.vp[k] + a * Lv;
                if (damped) {
                    nu = (nu + gu * ctr.up[k]) / (1.0 + gu);
                    nv = (nv + gv * ctr.vp[k]) / (1.0 + gv);
                }
                h0u = ctr.h0u[k] + A.w * nu;
                h0v = ctr.h0v[k] + A.w * nv;
                h1u = ctr.h1u[k] + D.wv * (nu - ctr.up[k]);
                h1v = ctr.h1v[k] + D.wv * (nv - ctr.vp[k]);
            } else {
                // ctr.up / ctr.vp hold the second field u1 here
                nu = cc.u + D.dtw * (1.0 - gu) * ctr.up[k] + 0.5 * a * Lu;
                nv = cc.v + D.dtw * (1.0 - gv) * ctr.vp[k] + 0.5 * a * Lv;
                h0u = ctr.h0u[k] + A.w0 * cc.u + A.w * nu;
                h0v = ctr.h0v[k] + A.w0 * cc.v + A.w * nv;
                h1u = ctr.h1u[k] + D.w0v * ctr.up[k];
                h1v = ctr.h1v[k] + D.w0v * ctr.vp[k];
            }
            unext[o + k] = nu;
            unext[o + k + CS] = nv;
            acc0[o + k] = h0u;
            acc0[o + k + CS] = h0v;
            acc1[o + k] = h1u;
            acc1[o + k + CS] = h1v;
        }
        S = C;
        C = N;
        if (j + 1 <= j1) {
            rawN = rawNN;
            ctr = ctrN;
        }
    }
}

// The face column of an impedance x face, one row per lane: block fb of the
// face blocks takes 64 rows of the -x face column (fb < nchunk when that
// face is an impedance face) or of the +x face column.  Same update and
// accumulation as the strip march; strided loads (two columns only).
template <int MODE, bool FORCE>
__device__ __forceinline__ void damped2d_face(int fb, const double* __restrict__ u, const double* uprev,
                                              double* unext, const double* __restrict__ base0,
                                              const double* __restrict__ base1, double* __restrict__ acc0,
                                              double* __restrict__ acc1, const double* __restrict__ dmp,
                                              const double* __restrict__ dmpx, const double* __restrict__ ca,
                                              const double* __restrict__ cl, const double* __restrict__ cm,
                                              const double* __restrict__ f, const Damp2D& D) {
    const Args2D& A = D.A;
    const int nchunk = (A.jhi - A.jlo + 1 + 63) / 64;
    const bool lo = D.ximp_lo && fb < nchunk;
    const int j = A.jlo + (fb % nchunk) * 64 + (int)threadIdx.x;
    if (j > A.jhi) return;
    const int i = lo ? 0 : A.nx, in = lo ? 1 : A.nx - 1;
    const int64_t P = A.P, CS = A.CS, o = (int64_t)j * P + i;
    auto at = [&](const double* b, int ii, int jj) { return (jj >= 0 && jj <= A.ny) ? b[jj * P + ii] : 0.0; };
    const double* v = u + CS;
    double Lu, Lv;
    xface_rows(lo ? 1.0 : -1.0, j, A.ny, A.free_lo, A.free_hi, A.cxx2, A.cyy2, D.hx, D.hy, at(u, i, j - 1),
               at(u, i, j), at(u, i, j + 1), at(v, i, j - 1), at(v, i, j), at(v, i, j + 1), at(u, in, j - 1),
               at(u, in, j), at(u, in, j + 1), at(v, in, j - 1), at(v, in, j), at(v, in, j + 1), at(cl, i, j - 1),
               at(cl, i, j), at(cl, i, j + 1), at(cm, i, j - 1), at(cm, i, j), at(cm, i, j + 1), at(cl, in, j),
               at(cm, in, j), Lu, Lv);
    if constexpr (FORCE) {
        Lu -= A.fc * f[o];
        Lv -= A.fc * f[o + CS];
    }
    // damping of this face column, plus that of an impedance y face at the corners
    const double* gx = dmpx + (int64_t)(lo ? 0 : 2) * (A.ny + 1);
    double gu = gx[j], gv = gx[A.ny + 1 + j];
    if ((j == 0 && D.imp_lo) || (j == A.ny && D.imp_hi)) {
        const double* gy = dmp + (int64_t)(j == 0 ? 0 : 2) * P;
        gu += gy[i];
        gv += gy[P + i];
    }
    const double a = ca[o], uc = u[o], vc = v[o], up = uprev[o], vp = uprev[o + CS];
    double nu, nv, h0u, h0v, h1u, h1v;
    if constexpr (MODE == 0) {
        nu = (2.0 * uc - up + a * Lu + gu * up) / (1.0 + gu);
        nv = (2.0 * vc - vp + a * Lv + gv * vp) / (1.0 + gv);
        h0u = acc0[o] + A.w * nu;
        h0v = acc0[o + CS] + A.w * nv;
        h1u = acc1[o] + D.wv * (nu - up);
        h1v = acc1[o + CS] + D.wv * (nv - vp);
    } else {
        // up / vp hold the second field u1 here
        nu = uc + D.dtw * (1.0 - gu) * up + 0.5 * a * Lu;
        nv = vc + D.dtw * (1.0 - gv) * vp + 0.5 * a * Lv;
        h0u = (base0 ? base0[o] : 0.0) + A.w0 * uc + A.w * nu;
        h0v = (base0 ? base0[o + CS] : 0.0) + A.w0 * vc + A.w * nv;
        h1u = (base1 ? base1[o] : 0.0) + D.w0v * up;
        h1v = (base1 ? base1[o + CS] : 0.0) + D.w0v * vp;
    }
    unext[o] = nu;
    unext[o + CS] = nv;
    acc0[o] = h0u;
    acc0[o + CS] = h0v;
    acc1[o] = h1u;
    acc1[o + CS] = h1v;
}

template <int V, int TY, int MODE, bool FORCE>
__global__ __launch_bounds__(64) void damped2d_kernel(const double* __restrict__ u, const double* uprev,
                                                     double* unext, const double* __restrict__ base0,
                                                     const double* __restrict__ base1, double* __restrict__ acc0,
                                                     double* __restrict__ acc1, const double* __restrict__ dmp,
                                                     const double* __restrict__ dmpx, const double* __restrict__ ca,
                                                     const double* __restrict__ cl, const double* __restrict__ cm,
                                                     const double* __restrict__ f, Damp2D D) {
    if ((int)blockIdx.x >= D.nmain) {   // the face-column blocks follow the strip tiles
        damped2d_face<MODE, FORCE>((int)blockIdx.x - D.nmain, u, uprev, unext, base0, base1, acc0, acc1, dmp, dmpx,
                                   ca, cl, cm, f, D);
        return;
    }
    const int nbx = (D.A.nx - 1 + Cols<V>::W - 1) / Cols<V>::W;
    const int nby = (D.A.jhi - D.A.jlo + 1 + TY - 1) / TY;
    int t;
    if (!xcd_tile((int)blockIdx.x, nbx * nby, t)) return;
    damped2d_body<V, TY, MODE, FORCE>(t % nbx, t / nbx, u, uprev, unext, base0, base1, acc0, acc1, dmp, dmpx, ca,
                                      cl, cm, f, D);
}

template <int V, int TY>
void damped_launch_vt(int mode, bool force, hipStream_t s, const double* u, const double* uprev, double* unext,
                      const double* base0, const double* base1, double* acc0, double* acc1, const double* dmp,
                      const double* dmpx, const double* ca, const double* cl, const double* cm, const double* f,
                      const Damp2D& Din) {
    Damp2D D = Din;
    const int nrows = D.A.jhi - D.A.jlo + 1;
    const int nbx = (D.A.nx - 1 + Cols<V>::W - 1) / Cols<V>::W;
    D.nmain = xcd_grid(nbx * ((nrows + TY - 1) / TY));
    const int nface = (D.ximp_lo + D.ximp_hi) * ((nrows + 63) / 64);
    const dim3 grid((unsigned)(D.nmain + nface));
#define ELWH_DL(M, F)                                                                                         \
    hipLaunchKernelGGL((damped2d_kernel<V, TY, M, F>), grid, dim3(64), 0, s, u, uprev, unext, base0, base1,  \
                       acc0, acc1, dmp, dmpx, ca, cl, cm, f, D)
    if (mode == 0) {
        if (force) ELWH_DL(0, true); else ELWH_DL(0, false);
    } else {
        if (force) ELWH_DL(1, true); else ELWH_DL(1, false);
    }
#undef ELWH_DL
}

}  // namespace

bool tile_valid_damped(int V, int TY) { return (V == 1 || V == 2) && (TY == 4 || TY == 8 || TY == 16); }

void launch_damped2d(int V, int TY, int mode, bool force, hipStream_t s, const double* u, const double* uprev,
                     double* unext, const double* base0, const double* base1, double* acc0, double* acc1,
                     const double* dmp, const double* dmpx, const double* ca, const double* cl, const double* cm,
                     const double* f, const Damp2D& D) {
#define ELWH_DV(VV, TT)                                                                                       \
    if (V == VV && TY == TT) {                                                                                \
        damped_launch_vt<VV, TT>(mode, force, s, u, uprev, unext, base0, base1, acc0, acc1, dmp, dmpx, ca, cl, \
                                 cm, f, D);                                                                   \
        return;                                                                                               \
    }
    ELWH_DV(1, 4) ELWH_DV(1, 8) ELWH_DV(1, 16) ELWH_DV(2, 4) ELWH_DV(2, 8) ELWH_DV(2, 16)
#undef ELWH_DV
    damped_launch_vt<1, 8>(mode, force, s, u, uprev, unext, base0, base1, acc0, acc1, dmp, dmpx, ca, cl, cm, f, D);
}

}  // namespace elwh
