// C ABI of libelwh (declared in include/elwh.h): context set-up, the filter
// and A_h applications, and the Krylov drivers.
//
// Krylov (Sec. 4.5): M A_h is symmetric, so CG runs on A_h in the M inner
// product, A_h = I - S_h and b = Pi_h 0.  The CG scalars live on the device
// (alpha and beta are formed by the reduction kernels), the host reads one
// residual per iteration off the critical path.  Conjugate residual (Remark
// of Sec. 4.5; also the fallback after a CG breakdown) and restarted GMRES
// with classical Gram-Schmidt applied twice (used for non-symmetric problems
// in Sec. 5.4) are host-driven over the same FP64 reductions.  The FP32 path
// runs CG with FP32-stepped applications and FP64 vectors and replaces the
// residual by b - A_h x from an FP64 application whenever it has fallen by
// inner_tol, keeping the search direction (reliable updates); it stops on
// that FP64 residual.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include "elwh_internal.h"

namespace elwh {
void run_filter_2d(elwh_ctx* c, const double* x, bool with_force, bool amode, bool fp32, double* out);
void run_filter_3d(elwh_ctx* c, const double* x, bool with_force, bool amode, bool fp32, double* out);

void prof_mark(elwh_ctx* c, int phase, int nsteps) {
    if (!c->prof_on) return;
    const size_t base = 3 * c->prof_used;
    if (phase == 0) {
        while (c->prof_ev.size() < base + 3) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) {
                c->prof_on = false;
                return;
            }
            c->prof_ev.push_back(e);
        }
    }
    (void)hipEventRecord(c->prof_ev[base + phase], c->stream);
    if (phase == 2) {
        if (c->prof_nsteps.size() <= c->prof_used) c->prof_nsteps.resize(c->prof_used + 1);
        c->prof_nsteps[c->prof_used] = nsteps;
        c->prof_used++;
    }
}

void run_filter(elwh_ctx* c, const double* x, bool with_force, bool amode, bool fp32, double* out) {
    if (c->mapped && c->L.dim == 3)
        run_filter_curv3d(c, x, with_force, amode, fp32, out);
    else if (c->mapped)
        run_filter_curv2d(c, x, with_force, amode, fp32, out);
    else if (c->L.dim == 2)
        run_filter_2d(c, x, with_force, amode, fp32, out);
    else
        run_filter_3d(c, x, with_force, amode, fp32, out);
    c->napply++;
}
}  // namespace elwh

using namespace elwh;

namespace {

thread_local std::string g_create_err;

enum { VX = 0, VR, VP, VQ, VB, VT, VD, VRI };

#define HIPCK(expr)                                                                   \
    do {                                                                              \
        hipError_t e_ = (expr);                                                       \
        if (e_ != hipSuccess) {                                                       \
            c->err = std::string(#expr) + ": " + hipGetErrorString(e_);               \
            return ELWH_ERR_HIP;                                                      \
        }                                                                             \
    } while (0)

#define CKST(expr)                    \
    do {                              \
        elwh_status s_ = (expr);      \
        if (s_ != ELWH_OK) return s_; \
    } while (0)

elwh_status dev_alloc(elwh_ctx* c, void** p, size_t bytes) {
    if (hipMalloc(p, bytes) != hipSuccess) {
        *p = nullptr;
        c->err = "device allocation failed (" + std::to_string(bytes) + " bytes)";
        return ELWH_ERR_ALLOC;
    }
    if (hipMemsetAsync(*p, 0, bytes, c->stream) != hipSuccess) {
        c->err = "hipMemsetAsync failed";
        return ELWH_ERR_HIP;
    }
    return ELWH_OK;
}

template <typename T>
elwh_status alloc_t(elwh_ctx* c, T** p, size_t n) {
    return dev_alloc(c, reinterpret_cast<void**>(p), n * sizeof(T));
}

void free_all(elwh_ctx* c) {
    auto f = [](void* p) {
        if (p) (void)hipFree(p);
    };
    f(c->ca); f(c->cl); f(c->cm); f(c->mw);
    f(c->fa); f(c->fl); f(c->fm);
    for (auto* p : c->cg) f(p);
    for (auto* p : c->fg) f(p);
    f(c->jac);
    for (auto* p : c->s64) f(p);
    for (auto* p : c->s32) f(p);
    f(c->acc); f(c->acc_lo); f(c->f64); f(c->f32);
    for (auto* v : c->vec) f(v);
    for (auto* v : c->basis) f(v);
    f(c->dmp); f(c->dmpx); f(c->acc1); f(c->x1);
    for (auto* v : c->basis2) f(v);
    f(c->gm_ptrs); f(c->gm_part); f(c->gm_h);
    f(c->partials); f(c->dscal);
    if (c->hscal) (void)hipHostFree(c->hscal);
    for (auto e : c->prof_ev) (void)hipEventDestroy(e);
    c->prof_ev.clear();
    if (c->ev_scal) (void)hipEventDestroy(c->ev_scal);
    c->ev_scal = nullptr;
}

// (x, y)_M into the host (synchronising).
elwh_status dot_host(elwh_ctx* c, const double* x, const double* y, double* out) {
    launch_dot_M_partial(c, x, y, c->stream);
    launch_reduce_final(c, RED_SUM, S_TMP, c->stream);
    HIPCK(hipMemcpyAsync(c->hscal, c->dscal, S_NSLOT * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCK(hipStreamSynchronize(c->stream));
    *out = c->hscal[S_TMP];
    return ELWH_OK;
}

elwh_status read_scalars(elwh_ctx* c) {
    HIPCK(hipMemcpyAsync(c->hscal, c->dscal, S_NSLOT * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCK(hipStreamSynchronize(c->stream));
    return ELWH_OK;
}

elwh_status set_scalar(elwh_ctx* c, int slot, double v) {
    HIPCK(hipStreamSynchronize(c->stream));
    c->hscal[slot] = v;
    HIPCK(hipMemcpyAsync(c->dscal + slot, c->hscal + slot, sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIPCK(hipStreamSynchronize(c->stream));
    return ELWH_OK;
}

void apply_A(elwh_ctx* c, const double* x, double* y, bool fp32) { run_filter(c, x, false, true, fp32, y); }

// b (VB) = Pi_h 0 with the packed forcing, FP64 stepping.
void compute_rhs(elwh_ctx* c) {
    double* zero = c->vec[VT];
    (void)hipMemsetAsync(zero, 0, c->L.field_elems() * sizeof(double), c->stream);
    run_filter(c, zero, true, false, false, c->vec[VB]);
}

// Device-scalar CG on A (FP64 or FP32 stepping) for rhs b, solution in x,
// work vectors r, p, q.  x holds the initial guess (x_zero: it is zero).
struct CGOut {
    int iters = 0;
    double relres = 0;
    bool converged = false;
};

// x <- alpha x, q <- alpha q with alpha = (x, b)_M / (x, q)_M (q = A_h x);
// alpha = 0 when (x, q)_M <= 0.
// Forcing into the internal layout (and FP32 copy); a mapped grid takes J f.
void pack_forcing(elwh_ctx* c, const double* f, bool fp32) {
    launch_pack(c->L, c->bc, f, c->f64, c->L.dim, c->stream);
    if (c->mapped) launch_scale_field(c->L, c->f64, c->jac, c->L.dim, c->stream);
    if (fp32) launch_convert_f32(c->L, c->f64, c->f32, c->L.dim, c->stream);
}

elwh_status scale_start(elwh_ctx* c, const double* b, double* x, double* q) {
    double xb, xq;
    CKST(dot_host(c, x, b, &xb));
    CKST(dot_host(c, x, q, &xq));
    const double alpha = (xq > 0 && std::isfinite(xb) && std::isfinite(xq)) ? xb / xq : 0.0;
    launch_axpby(c, 0.0, x, alpha, x, c->stream);
    launch_axpby(c, 0.0, q, alpha, q, c->stream);
    return ELWH_OK;
}

elwh_status cg_start(elwh_ctx* c, const double* b, double* x, bool x_zero, double* r, double* p, double* q,
                     bool fp32, double* bb_out, double* rr_out) {
    if (x_zero) {
        launch_copy(c, b, r, c->stream);
    } else {
        apply_A(c, x, q, fp32);
        if (c->opts.scale_x0) CKST(scale_start(c, b, x, q));
        launch_copy(c, b, r, c->stream);
        launch_axpby(c, -1.0, q, 1.0, r, c->stream);
    }
    launch_copy(c, r, p, c->stream);
    double bb, rr;
    CKST(dot_host(c, b, b, &bb));
    CKST(dot_host(c, r, r, &rr));
    if (!std::isfinite(bb) || !std::isfinite(rr)) {
        c->err = "non-finite right-hand side or residual";
        return ELWH_ERR_ARG;
    }
    CKST(set_scalar(c, S_RR, rr));
    CKST(set_scalar(c, S_FLAG, 0.0));
    *bb_out = bb;
    *rr_out = rr;
    return ELWH_OK;
}

// k CG iterations; returns early when ||r||_M <= tol ||b||_M.
elwh_status cg_steps(elwh_ctx* c, double* x, double* r, double* p, double* q, bool fp32, double bb, int k,
                     double tol, CGOut* out, bool record) {
    for (int it = 0; it < k; ++it) {
        apply_A(c, p, q, fp32);
        launch_dot_pq_pp_partial(c, p, q, c->stream);
        launch_reduce_final(c, RED_PQ, 0, c->stream);
        launch_cg_update_xr(c, x, r, p, q, c->stream);
        launch_reduce_final(c, RED_RR, 0, c->stream);
        CKST(read_scalars(c));
        if (c->hscal[S_FLAG] == 2.0) {
            c->err = "(p, A_h p)_M / (p, p)_M lies outside the spectrum of a stable step: the time step is unstable";
            return ELWH_ERR_UNSTABLE;
        }
        if (c->hscal[S_FLAG] != 0.0) {
            c->err = "CG breakdown: (p, A_h p)_M <= 0 (A_h not positive definite near resonance)";
            return ELWH_ERR_BREAKDOWN;
        }
        const double rr = c->hscal[S_RR];
        if (!std::isfinite(rr)) {
            c->err = "non-finite residual: the time step is unstable";
            return ELWH_ERR_UNSTABLE;
        }
        out->iters++;
        out->relres = std::sqrt(rr / bb);
        if (record) {
            c->alphas.push_back(c->hscal[S_ALPHA]);
        }
        if (tol > 0 && out->relres <= tol) {
            out->converged = true;
            return ELWH_OK;
        }
        if (record) c->betas.push_back(c->hscal[S_BETA]);
        launch_cg_update_p(c, p, r, c->stream);
    }
    return ELWH_OK;
}

// The same CG iterations with the host check taken off the critical path:
// after an iteration's scalars are copied to the host (asynchronously), the
// next direction p = r + beta p and its application q = A_h p are enqueued
// before the host waits for and checks the copy, so the GPU never idles on
// the host round trip.  A converged or failed iteration leaves p and q one
// step ahead (q valid: cg_qready), which a later call continues from; the last
// of the k iterations enqueues only the direction update.  FP64 stepping.
elwh_status cg_steps_pipelined(elwh_ctx* c, double* x, double* r, double* p, double* q, double bb, int k, double tol,
                               CGOut* out) {
    if (!c->ev_scal) HIPCK(hipEventCreateWithFlags(&c->ev_scal, hipEventDisableTiming));
    for (int it = 0; it < k; ++it) {
        if (!c->cg_qready) apply_A(c, p, q, false);
        c->cg_qready = false;
        launch_dot_pq_pp_partial(c, p, q, c->stream);
        launch_reduce_final(c, RED_PQ, 0, c->stream);
        launch_cg_update_xr(c, x, r, p, q, c->stream);
        launch_reduce_final(c, RED_RR, 0, c->stream);
        HIPCK(hipMemcpyAsync(c->hscal, c->dscal, S_NSLOT * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCK(hipEventRecord(c->ev_scal, c->stream));
        launch_cg_update_p(c, p, r, c->stream);
        if (it + 1 < k) {
            apply_A(c, p, q, false);
            c->cg_qready = true;
        }
        HIPCK(hipEventSynchronize(c->ev_scal));
        if (c->hscal[S_FLAG] == 2.0) {
            c->err = "(p, A_h p)_M / (p, p)_M lies outside the spectrum of a stable step: the time step is unstable";
            return ELWH_ERR_UNSTABLE;
        }
        if (c->hscal[S_FLAG] != 0.0) {
            c->err = "CG breakdown: (p, A_h p)_M <= 0 (A_h not positive definite near resonance)";
            return ELWH_ERR_BREAKDOWN;
        }
        const double rr = c->hscal[S_RR];
        if (!std::isfinite(rr)) {
            c->err = "non-finite residual: the time step is unstable";
            return ELWH_ERR_UNSTABLE;
        }
        out->iters++;
        out->relres = std::sqrt(rr / bb);
        c->alphas.push_back(c->hscal[S_ALPHA]);
        if (tol > 0 && out->relres <= tol) {
            out->converged = true;
            return ELWH_OK;
        }
        c->betas.push_back(c->hscal[S_BETA]);
    }
    return ELWH_OK;
}

double lanczos_cond(const std::vector<double>& a, const std::vector<double>& b) {
    const int k = (int)a.size();
    if (k == 0) return NAN;
    // symmetric tridiagonal T_k; extreme eigenvalues by bisection on Sturm counts
    std::vector<double> d(k), e(k, 0.0);
    for (int i = 0; i < k; ++i) {
        d[i] = 1.0 / a[i] + (i > 0 ? b[i - 1] / a[i - 1] : 0.0);
        if (i + 1 < k && i < (int)b.size()) e[i] = std::sqrt(b[i]) / a[i];
    }
    double lo = 1e300, hi = -1e300;
    for (int i = 0; i < k; ++i) {
        const double r = std::fabs(i > 0 ? e[i - 1] : 0.0) + std::fabs(e[i]);
        lo = std::min(lo, d[i] - r);
        hi = std::max(hi, d[i] + r);
    }
    auto count_below = [&](double x) {
        int cnt = 0;
        double q = 1.0;
        for (int i = 0; i < k; ++i) {
            const double off = i > 0 ? e[i - 1] : 0.0;
            q = d[i] - x - (i > 0 ? off * off / q : 0.0);
            if (q == 0.0) q = 1e-300;
            if (q < 0) cnt++;
        }
        return cnt;
    };
    auto kth = [&](int idx) {
        double a_ = lo, b_ = hi;
        for (int it = 0; it < 200; ++it) {
            const double m = 0.5 * (a_ + b_);
            if (count_below(m) > idx) b_ = m; else a_ = m;
        }
        return 0.5 * (a_ + b_);
    };
    const double emin = kth(0), emax = kth(k - 1);
    return emin > 0 ? emax / emin : NAN;
}

elwh_status final_residual(elwh_ctx* c, const double* x, double bb, double* out) {
    apply_A(c, x, c->vec[VQ], false);
    launch_copy(c, c->vec[VB], c->vec[VT], c->stream);
    launch_axpby(c, -1.0, c->vec[VQ], 1.0, c->vec[VT], c->stream);
    double rr;
    CKST(dot_host(c, c->vec[VT], c->vec[VT], &rr));
    *out = std::sqrt(rr / bb);
    return ELWH_OK;
}

elwh_status solve_cr(elwh_ctx* c, bool x_zero, double tol, int maxit, int* iters, double* relres) {
    double *x = c->vec[VX], *r = c->vec[VR], *p = c->vec[VP], *Ar = c->vec[VQ], *Ap = c->vec[VD];
    const double* b = c->vec[VB];
    if (x_zero) {
        launch_copy(c, b, r, c->stream);
    } else {
        apply_A(c, x, Ar, false);
        launch_copy(c, b, r, c->stream);
        launch_axpby(c, -1.0, Ar, 1.0, r, c->stream);
    }
    double bb, rr, rAr, ApAp;
    CKST(dot_host(c, b, b, &bb));
    CKST(dot_host(c, r, r, &rr));
    *relres = std::sqrt(rr / bb);
    *iters = 0;
    if (tol > 0 && *relres <= tol) return ELWH_OK;
    launch_copy(c, r, p, c->stream);
    apply_A(c, r, Ar, false);
    launch_copy(c, Ar, Ap, c->stream);
    CKST(dot_host(c, r, Ar, &rAr));
    for (int k = 1; k <= maxit; ++k) {
        CKST(dot_host(c, Ap, Ap, &ApAp));
        if (!(ApAp > 0) || !std::isfinite(rAr)) {
            c->err = std::isfinite(rAr) ? "CR breakdown" : "non-finite residual: the time step is unstable";
            return std::isfinite(rAr) ? ELWH_ERR_BREAKDOWN : ELWH_ERR_UNSTABLE;
        }
        const double alpha = rAr / ApAp;
        launch_axpby(c, alpha, p, 1.0, x, c->stream);
        launch_axpby(c, -alpha, Ap, 1.0, r, c->stream);
        CKST(dot_host(c, r, r, &rr));
        *iters = k;
        *relres = std::sqrt(rr / bb);
        if (tol > 0 && *relres <= tol) return ELWH_OK;
        apply_A(c, r, Ar, false);
        double rAr_new;
        CKST(dot_host(c, r, Ar, &rAr_new));
        if (rAr_new == 0.0) {
            // r is M-orthogonal to A_h r: the next step would not move x
            c->err = "CR breakdown: (r, A_h r)_M = 0 (A_h indefinite; MINRES does not break down here)";
            return ELWH_ERR_BREAKDOWN;
        }
        const double beta = rAr_new / rAr;
        launch_axpby(c, 1.0, r, beta, p, c->stream);
        launch_axpby(c, 1.0, Ar, beta, Ap, c->stream);
        rAr = rAr_new;
    }
    return tol > 0 ? ELWH_ERR_NOT_CONVERGED : ELWH_OK;
}

// MINRES in the M inner product (the remedy the remark in Sec. 4.4 recommends
// when A_h is slightly indefinite near resonance): x_k minimises ||b - A_h x||_M
// over x_0 + K_k(A_h, r_0).  The Lanczos process in the M inner product
// (A_h is M-self-adjoint) builds A_h V_k = V_{k+1} Tbar_k; the small
// least-squares problem min ||beta_1 e_1 - Tbar_k y|| is solved by one Givens
// rotation per column (Paige and Saunders), and x is updated through the
// direction vectors D_k = V_k R_k^{-1}.  Host-driven: one application and two
// FP64 M-dots per iteration.  Iterate in VX, right-hand side in VB; uses VR,
// VP, VQ, VD, VRI as work vectors.
elwh_status solve_minres(elwh_ctx* c, bool x_zero, double tol, int maxit, int* iters, double* relres) {
    double* x = c->vec[VX];
    const double* b = c->vec[VB];
    double* vprev = c->vec[VR];   // v_{j-1}
    double* v = c->vec[VP];       // v_j
    double* q = c->vec[VQ];       // A_h v_j, then beta_{j+1} v_{j+1}
    double* d1 = c->vec[VD];      // d_{j-1}
    double* d2 = c->vec[VRI];     // d_{j-2}, overwritten by d_j
    if (x_zero) {
        launch_copy(c, b, v, c->stream);
    } else {
        apply_A(c, x, q, false);
        launch_copy(c, b, v, c->stream);
        launch_axpby(c, -1.0, q, 1.0, v, c->stream);
    }
    double bb, rr;
    CKST(dot_host(c, b, b, &bb));
    CKST(dot_host(c, v, v, &rr));
    if (!std::isfinite(rr)) {
        c->err = "non-finite residual: the time step is unstable";
        return ELWH_ERR_UNSTABLE;
    }
    const double bn = std::sqrt(bb);
    double beta = std::sqrt(rr);   // beta_1 = ||r_0||_M
    *relres = beta / bn;
    *iters = 0;
    if ((tol > 0 && *relres <= tol) || beta == 0.0) return ELWH_OK;
    launch_axpby(c, 0.0, v, 1.0 / beta, v, c->stream);
    const size_t bytes = c->L.field_elems() * sizeof(double);
    HIPCK(hipMemsetAsync(vprev, 0, bytes, c->stream));
    HIPCK(hipMemsetAsync(d1, 0, bytes, c->stream));
    HIPCK(hipMemsetAsync(d2, 0, bytes, c->stream));
    double c2 = 1.0, s2 = 0.0, c1 = 1.0, s1 = 0.0;   // rotations G_{j-2}, G_{j-1}
    double g = beta;                                  // rotated right-hand side entry j
    for (int k = 1; k <= maxit; ++k) {
        apply_A(c, v, q, false);
        double alpha;
        CKST(dot_host(c, v, q, &alpha));
        launch_axpby(c, -alpha, v, 1.0, q, c->stream);
        if (k > 1) launch_axpby(c, -beta, vprev, 1.0, q, c->stream);
        double qq;
        CKST(dot_host(c, q, q, &qq));
        if (!std::isfinite(alpha) || !std::isfinite(qq)) {
            c->err = "non-finite Lanczos coefficient: the time step is unstable";
            return ELWH_ERR_UNSTABLE;
        }
        const double beta_next = std::sqrt(qq);
        // column k of Tbar is (beta_k, alpha_k, beta_{k+1}) in rows k-1, k, k+1
        // (no entry above the first diagonal); apply G_{k-2}, G_{k-1}, then
        // form G_k, which zeroes beta_{k+1}
        const double bk = k > 1 ? beta : 0.0;
        const double eps = s2 * bk, t = c2 * bk;
        const double delta = c1 * t + s1 * alpha;
        const double gbar = -s1 * t + c1 * alpha;
        const double gamma = std::hypot(gbar, beta_next);
        if (!(gamma > 0)) {
            c->err = "MINRES breakdown: singular Lanczos tridiagonal (A_h singular)";
            return ELWH_ERR_BREAKDOWN;
        }
        const double cs = gbar / gamma, sn = beta_next / gamma;
        const double tau = cs * g;
        g = -sn * g;
        // d_k = (v_k - delta d_{k-1} - eps d_{k-2}) / gamma, x += tau d_k
        launch_axpby(c, 1.0 / gamma, v, -eps / gamma, d2, c->stream);
        launch_axpby(c, -delta / gamma, d1, 1.0, d2, c->stream);
        launch_axpby(c, tau, d2, 1.0, x, c->stream);
        *iters = k;
        *relres = std::fabs(g) / bn;
        if ((tol > 0 && *relres <= tol) || beta_next == 0.0) return ELWH_OK;
        std::swap(d1, d2);
        launch_axpby(c, 0.0, q, 1.0 / beta_next, q, c->stream);   // v_{k+1}
        double* old = vprev;
        vprev = v;
        v = q;
        q = old;
        c2 = c1; s2 = s1; c1 = cs; s1 = sn;
        beta = beta_next;
    }
    return tol > 0 ? ELWH_ERR_NOT_CONVERGED : ELWH_OK;
}

// A residual-minimising method (CR or MINRES) from the iterate in VX, judged
// on the true residual: when its recurrence residual meets tol but
// ||b - A_h x||_M from an FP64 application does not, it restarts from x.
// relfp64 receives the last true residual (-1 when none was computed).
constexpr int kMaxReplace = 8;
typedef elwh_status (*MinResMethod)(elwh_ctx*, bool, double, int, int*, double*);

elwh_status solve_checked(elwh_ctx* c, MinResMethod method, bool x_zero, double tol, int maxit, int* iters,
                          double* relres, double* relfp64) {
    double bb;
    CKST(dot_host(c, c->vec[VB], c->vec[VB], &bb));
    *iters = 0;
    *relfp64 = -1.0;
    elwh_status st = ELWH_OK;
    for (int rep = 0;; ++rep) {
        int it = 0;
        st = method(c, x_zero && rep == 0, tol, maxit - *iters, &it, relres);
        *iters += it;
        if (st != ELWH_OK || tol <= 0) break;
        CKST(final_residual(c, c->vec[VX], bb, relfp64));
        if (*relfp64 <= tol) break;
        if (*iters >= maxit || rep + 1 >= kMaxReplace) {
            st = ELWH_ERR_NOT_CONVERGED;
            break;
        }
    }
    return st;
}

// The fallback after a CG breakdown starts from the iterate that the broken
// CG sequence started from (kept in VRI), not from the last CG iterate: close
// to a breakdown CG takes very long steps along directions with (p, A_h p)_M
// near 0, and the error they leave takes a residual-minimising method many
// more iterations to remove than the whole solve from the start does.
// (Measured on the six held-out warm-start problems at 256^2 whose CG breaks
// down: CR from the CG iterate 306, 2444, 717, 1306, 936 and over 6929
// iterations, CR from the start 213, 888, 705, 1018, 928 and 1085.)
void keep_start(elwh_ctx* c) { launch_copy(c, c->vec[VX], c->vec[VRI], c->stream); }
void back_to_start(elwh_ctx* c) { launch_copy(c, c->vec[VRI], c->vec[VX], c->stream); }

// Device buffers of the GMRES orthogonalisation for restart length m: the
// pointer table (up to 2 (m + 1) basis fields, then the two fields of w),
// the multi-dot partials and the coefficients of the two CGS passes plus
// ||w||^2.
elwh_status ensure_gm(elwh_ctx* c, int m) {
    if (c->gm_cap >= m + 1) return ELWH_OK;
    for (void* q : {(void*)c->gm_ptrs, (void*)c->gm_part, (void*)c->gm_h})
        if (q) (void)hipFree(q);
    c->gm_ptrs = nullptr;
    c->gm_part = c->gm_h = nullptr;
    c->gm_cap = 0;
    CKST(alloc_t(c, &c->gm_ptrs, (size_t)(2 * (m + 1) + 2)));
    CKST(alloc_t(c, &c->gm_part, (size_t)(m + 1) * multidot2_blocks(c)));
    CKST(alloc_t(c, &c->gm_h, (size_t)(2 * (m + 1) + 1)));
    c->gm_cap = m + 1;
    return ELWH_OK;
}

elwh_status solve_gmres(elwh_ctx* c, bool x_zero, double tol, int maxit, int* iters, double* relres) {
    const int m = c->opts.gmres_m;
    while ((int)c->basis.size() < m + 1) {
        double* v = nullptr;
        CKST(alloc_t(c, &v, (size_t)c->L.field_elems()));
        c->basis.push_back(v);
    }
    double* x = c->vec[VX];
    double* w = c->vec[VQ];
    const double* b = c->vec[VB];
    CKST(ensure_gm(c, m));
    {
        std::vector<double*> tab(c->basis.begin(), c->basis.begin() + (m + 1));
        tab.push_back(w);
        HIPCK(hipMemcpyAsync(c->gm_ptrs, tab.data(), tab.size() * sizeof(double*), hipMemcpyHostToDevice,
                             c->stream));
        HIPCK(hipStreamSynchronize(c->stream));   // tab is a host temporary
    }
    const double* const* ptrs = c->gm_ptrs;
    std::vector<double> hh(2 * (m + 1) + 1);
    double bb;
    CKST(dot_host(c, b, b, &bb));
    const double bn = std::sqrt(bb);
    int total = 0;
    bool first = true;
    std::vector<double> H((m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
    while (true) {
        double* r = c->basis[0];
        if (first && x_zero) {
            launch_copy(c, b, r, c->stream);
        } else {
            apply_A(c, x, w, false);
            launch_copy(c, b, r, c->stream);
            launch_axpby(c, -1.0, w, 1.0, r, c->stream);
        }
        first = false;
        double rr;
        CKST(dot_host(c, r, r, &rr));
        const double beta = std::sqrt(rr);
        if (!std::isfinite(beta)) {
            c->err = "non-finite residual: the time step is unstable";
            return ELWH_ERR_UNSTABLE;
        }
        *relres = beta / bn;
        *iters = total;
        if ((tol > 0 && *relres <= tol) || total >= maxit) break;
        launch_axpby(c, 0.0, r, 1.0 / beta, r, c->stream);
        std::fill(H.begin(), H.end(), 0.0);
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int jdone = 0;
        for (int j = 0; j < m; ++j) {
            apply_A(c, c->basis[j], w, false);
            total++;
            // classical Gram-Schmidt twice, coefficients on the device, one
            // host synchronisation per iteration
            for (int pass = 0; pass < 2; ++pass) {
                double* hp = c->gm_h + pass * (m + 1);
                launch_multidot2(c, ptrs, j + 1, w, nullptr, c->gm_part, hp, c->stream);
                launch_multiaxpy2(c, ptrs, j + 1, hp, w, nullptr, c->stream);
            }
            launch_multidot2(c, ptrs + (m + 1), 1, w, nullptr, c->gm_part, c->gm_h + 2 * (m + 1), c->stream);
            HIPCK(hipMemcpyAsync(hh.data(), c->gm_h, hh.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
            HIPCK(hipStreamSynchronize(c->stream));
            for (int i = 0; i <= j; ++i) H[i * m + j] += hh[i] + hh[m + 1 + i];
            const double ww = hh[2 * (m + 1)];
            const double hn = std::sqrt(ww);
            H[(j + 1) * m + j] = hn;
            for (int i = 0; i < j; ++i) {
                const double t = cs[i] * H[i * m + j] + sn[i] * H[(i + 1) * m + j];
                H[(i + 1) * m + j] = -sn[i] * H[i * m + j] + cs[i] * H[(i + 1) * m + j];
                H[i * m + j] = t;
            }
            const double rho = std::hypot(H[j * m + j], H[(j + 1) * m + j]);
            cs[j] = H[j * m + j] / rho;
            sn[j] = H[(j + 1) * m + j] / rho;
            H[j * m + j] = rho;
            H[(j + 1) * m + j] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            jdone = j + 1;
            *relres = std::fabs(g[j + 1]) / bn;
            if ((tol > 0 && *relres <= tol) || total >= maxit || hn == 0.0) break;
            launch_copy(c, w, c->basis[j + 1], c->stream);
            launch_axpby(c, 0.0, w, 1.0 / hn, c->basis[j + 1], c->stream);
        }
        for (int i = jdone - 1; i >= 0; --i) {
            double s = g[i];
            for (int k = i + 1; k < jdone; ++k) s -= H[i * m + k] * y[k];
            y[i] = s / H[i * m + i];
        }
        for (int i = 0; i < jdone; ++i) launch_axpby(c, y[i], c->basis[i], 1.0, x, c->stream);
    }
    *iters = total;
    return (tol > 0 && *relres > tol) ? ELWH_ERR_NOT_CONVERGED : ELWH_OK;
}

}  // namespace

// ============================================================================

namespace elwh {
void set_create_error(const std::string& msg) { g_create_err = msg; }

// Conjugate residual (method 1) or MINRES (method 2) in FP64 from the
// iterate in VX (right-hand side in VB), judged on the true residual, for the
// batch's fallback after a CG breakdown.
elwh_status ctx_solve_fallback(elwh_ctx* c, int method, double tol, int maxit, int* iters, double* relres) {
    double relfp64;
    return solve_checked(c, method == 2 ? solve_minres : solve_cr, false, tol, maxit, iters, relres, &relfp64);
}
}  // namespace elwh

namespace {
// Create a context; xc/yc non-null: a mapped 2-D grid with these node
// coordinates (host copies are taken here, like the materials).
elwh_status create_impl(const elwh_grid* grid_in, const double* xc, const double* yc, const double* zc, const double* rho,
                        const double* lam, const double* mu, double omega, const int* bc_in, const elwh_opts* opts,
                        elwh_ctx** out) {
    if (!out) return ELWH_ERR_ARG;
    *out = nullptr;
    elwh_opts o;
    elwh_default_opts(&o);
    if (opts) o = *opts;
    g_create_err.clear();
    if (!grid_in || !bc_in) {
        g_create_err = "null grid or bc";
        return ELWH_ERR_ARG;
    }
    const bool mapped = xc != nullptr;
    elwh_grid gbuf = *grid_in;
    int bc[6] = {ELWH_BC_DIRICHLET, ELWH_BC_DIRICHLET, ELWH_BC_DIRICHLET,
                 ELWH_BC_DIRICHLET, ELWH_BC_DIRICHLET, ELWH_BC_DIRICHLET};
    const bool mapped3 = mapped && zc != nullptr;
    for (int f = 0; f < (mapped && !mapped3 ? 4 : 2 * (gbuf.dim == 3 ? 3 : 2)); ++f) bc[f] = bc_in[f];
    if (mapped) {
        if (gbuf.dim != (mapped3 ? 3 : 2)) {
            g_create_err = mapped3 ? "3-D mapped grids need dim = 3" : "mapped grids of elwh_create_mapped are two-dimensional";
            return ELWH_ERR_ARG;
        }
        // the reference square or cube: h_a = 1/n_a
        gbuf.len[0] = gbuf.len[1] = gbuf.len[2] = 1.0;
    }
    // impedance faces: traction-type faces of the energy plus boundary damping
    int imp[2] = {0, 0}, ximp[2] = {0, 0};
    for (int f = 0; f < 6; ++f) {
        if (bc[f] != ELWH_BC_IMPEDANCE) continue;
        if (mapped || gbuf.dim != 2 || f > 3) {
            g_create_err = "impedance faces are supported on the faces of 2-D Cartesian grids";
            return ELWH_ERR_ARG;
        }
        if (o.prec != ELWH_FP64) {
            g_create_err = "impedance faces need FP64 stepping";
            return ELWH_ERR_ARG;
        }
        if (o.scheme == ELWH_SCHEME_MODIFIED) {
            g_create_err = "the modified trapezoid weights are for one-field contexts (no impedance faces)";
            return ELWH_ERR_ARG;
        }
        (f < 2 ? ximp[f] : imp[f - 2]) = 1;
        bc[f] = ELWH_BC_TRACTION_FREE;
    }
    const bool x_free_ok = ximp[0] || ximp[1];
    const elwh_grid* grid = &gbuf;
    elwh_status st = check_config(grid, bc, &o, &g_create_err, x_free_ok);
    if (st != ELWH_OK) return st;
    if (!rho || !lam || !mu) {
        g_create_err = "null material array";
        return ELWH_ERR_ARG;
    }
    elwh_ctx* c = new (std::nothrow) elwh_ctx();
    if (!c) return ELWH_ERR_ALLOC;
    c->grid = *grid;
    c->mapped = mapped;
    c->imp[0] = imp[0];
    c->imp[1] = imp[1];
    c->ximp[0] = ximp[0];
    c->ximp[1] = ximp[1];
    for (int f = 0; f < 6; ++f) c->bc[f] = f < 2 * grid->dim ? bc[f] : ELWH_BC_DIRICHLET;
    c->omega = omega;
    c->opts = o;
    c->stream = reinterpret_cast<hipStream_t>(o.stream);
    c->L = make_layout(grid);
    c->st = make_stencil(grid);
    c->mr = make_march(grid, c->bc);

    auto fail = [&](elwh_status s) {
        g_create_err = c->err.empty() ? g_create_err : c->err;
        free_all(c);
        delete c;
        return s;
    };
    const int64_t nn = c->L.nodes_caller();
    std::vector<double> hr(nn), hl(nn), hm(nn);
    if (hipMemcpyAsync(hr.data(), rho, nn * sizeof(double), hipMemcpyDefault, c->stream) != hipSuccess ||
        hipMemcpyAsync(hl.data(), lam, nn * sizeof(double), hipMemcpyDefault, c->stream) != hipSuccess ||
        hipMemcpyAsync(hm.data(), mu, nn * sizeof(double), hipMemcpyDefault, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess) {
        c->err = "copying the materials failed (device pointers expected)";
        return fail(ELWH_ERR_HIP);
    }
    MappedMetric met;
    if (mapped) {
        std::vector<double> hx(nn), hy(nn);
        if (hipMemcpyAsync(hx.data(), xc, nn * sizeof(double), hipMemcpyDefault, c->stream) != hipSuccess ||
            hipMemcpyAsync(hy.data(), yc, nn * sizeof(double), hipMemcpyDefault, c->stream) != hipSuccess ||
            hipStreamSynchronize(c->stream) != hipSuccess) {
            c->err = "copying the node coordinates failed (device pointers expected)";
            return fail(ELWH_ERR_HIP);
        }
        if (mapped3) {
            std::vector<double> hz(nn);
            if (hipMemcpyAsync(hz.data(), zc, nn * sizeof(double), hipMemcpyDefault, c->stream) != hipSuccess ||
                hipStreamSynchronize(c->stream) != hipSuccess) {
                c->err = "copying the node coordinates failed (device pointers expected)";
                return fail(ELWH_ERR_HIP);
            }
            st = make_plan_mapped3(grid, hx.data(), hy.data(), hz.data(), hr.data(), hl.data(), hm.data(), omega,
                                   c->bc, &o, &c->plan, &met, &c->err);
        } else {
            st = make_plan_mapped(grid, hx.data(), hy.data(), hr.data(), hl.data(), hm.data(), omega, c->bc, &o,
                                  &c->plan, &met, &c->err);
        }
    } else {
        st = make_plan(grid, hr.data(), hl.data(), hm.data(), omega, c->bc, &o, &c->plan, &c->err, x_free_ok);
    }
    if (st != ELWH_OK) return fail(st);

    // weights of the (K-period) trapezoid filter and the forcing factors
    // cos(omega t_n); the modified-weights scheme (remark closing Sec. 4.4)
    // forces at wbar = (2 / dt) asin(omega dt / 2) and multiplies each weight by
    // cos(omega t_n) / cos(wbar t_n)
    const int ntot = c->plan.nt * o.periods;
    const bool modified = o.scheme == ELWH_SCHEME_MODIFIED;
    const double wbar = modified ? 2.0 * std::asin(0.5 * omega * c->plan.dt) / c->plan.dt : omega;
    c->w.resize(ntot + 1);
    c->cosn.resize(ntot + 1);
    for (int n = 0; n <= ntot; ++n) {
        const double cn = std::cos(2.0 * M_PI * n / c->plan.nt);
        const double eta = (n == 0 || n == ntot) ? 0.5 : 1.0;
        const double cbar = modified ? std::cos(wbar * n * c->plan.dt) : cn;
        c->cosn[n] = cbar;
        c->w[n] = (2.0 / ntot) * eta * (cn - 0.25) * (modified ? cn / cbar : 1.0);
    }

    const Layout& L = c->L;
    const size_t CS = (size_t)L.CS, FE = (size_t)L.field_elems();
    if ((st = alloc_t(c, &c->ca, CS)) || (st = alloc_t(c, &c->cl, CS)) || (st = alloc_t(c, &c->cm, CS)) ||
        (st = alloc_t(c, &c->mw, CS)) || (st = alloc_t(c, &c->s64[0], FE)) || (st = alloc_t(c, &c->s64[1], FE)) ||
        (st = alloc_t(c, &c->acc_lo, FE)) || (st = alloc_t(c, &c->f64, FE)))
        return fail(st);
    for (auto& v : c->vec)
        if ((st = alloc_t(c, &v, FE))) return fail(st);
    // four state levels where a launch takes two or more steps (2-D; 3-D Cartesian with fuse >= 2)
    const bool four = L.dim == 2 || (!mapped && o.fuse >= 2);
    if (four && ((st = alloc_t(c, &c->s64[2], FE)) || (st = alloc_t(c, &c->s64[3], FE)))) return fail(st);
    if (o.prec == ELWH_FP32_STEP) {
        if ((st = alloc_t(c, &c->fa, CS)) || (st = alloc_t(c, &c->fl, CS)) || (st = alloc_t(c, &c->fm, CS)) ||
            (st = alloc_t(c, &c->s32[0], FE)) || (st = alloc_t(c, &c->s32[1], FE)) ||
            (st = alloc_t(c, &c->f32, FE)))
            return fail(st);
        if (four && ((st = alloc_t(c, &c->s32[2], FE)) || (st = alloc_t(c, &c->s32[3], FE))))
            return fail(st);
    }
    const int nmetric = mapped3 ? 9 : 4;
    if (mapped) {
        for (int k = 0; k < nmetric; ++k)
            if ((st = alloc_t(c, &c->cg[k], CS)) ||
                (o.prec == ELWH_FP32_STEP && (st = alloc_t(c, &c->fg[k], CS))))
                return fail(st);
        if ((st = alloc_t(c, &c->jac, CS))) return fail(st);
    }
    if ((st = alloc_t(c, &c->partials, 2 * (size_t)c->red_blocks)) || (st = alloc_t(c, &c->dscal, (size_t)S_NSLOT)))
        return fail(st);
    if (hipHostMalloc(reinterpret_cast<void**>(&c->hscal), S_NSLOT * sizeof(double), hipHostMallocDefault) !=
        hipSuccess) {
        c->err = "pinned host allocation failed";
        return fail(ELWH_ERR_ALLOC);
    }
    std::memset(c->hscal, 0, S_NSLOT * sizeof(double));

    // coefficient arrays in the padded layout, built on the host in FP64
    {
        std::vector<double> ha(CS, 0.0), hlam(CS, 0.0), hmu(CS, 0.0), hmw(CS, 0.0);
        std::vector<double> hg[9], hj;
        if (mapped) {
            for (int k = 0; k < nmetric; ++k) hg[k].assign(CS, 0.0);
            hj.assign(CS, 0.0);
        }
        const double cdt2 = c->plan.c * c->plan.dt * c->plan.dt;
        const int nzn = L.dim == 3 ? L.nz + 1 : 1;
        for (int z = 0; z < nzn; ++z)
            for (int y = 0; y <= L.ny; ++y)
                for (int x = 0; x <= L.nx; ++x) {
                    const int64_t src = ((int64_t)z * (L.ny + 1) + y) * (L.nx + 1) + x;
                    const int64_t dst = (int64_t)z * L.PS + (int64_t)y * L.P + x;
                    const double jw = mapped ? met.J[src] : 1.0;   // mass rho J, lambda/J, mu/J
                    ha[dst] = cdt2 / (hr[src] * jw);
                    hlam[dst] = hl[src] / jw;
                    hmu[dst] = hm[src] / jw;
                    if (mapped) {
                        for (int k = 0; k < nmetric; ++k) hg[k][dst] = met.g[k][src];
                        hj[dst] = jw;
                    }
                    bool unknown = true;
                    double wn = 1.0;
                    const int coord[3] = {x, y, z};
                    const int nmax[3] = {L.nx, L.ny, L.nz};
                    for (int a = 0; a < L.dim; ++a) {
                        if (coord[a] == 0) {
                            if (c->bc[2 * a] == ELWH_BC_DIRICHLET) unknown = false; else wn *= 0.5;
                        }
                        if (coord[a] == nmax[a]) {
                            if (c->bc[2 * a + 1] == ELWH_BC_DIRICHLET) unknown = false; else wn *= 0.5;
                        }
                    }
                    hmw[dst] = unknown ? wn * hr[src] * jw : 0.0;
                }
        if (hipMemcpyAsync(c->ca, ha.data(), CS * 8, hipMemcpyHostToDevice, c->stream) != hipSuccess ||
            hipMemcpyAsync(c->cl, hlam.data(), CS * 8, hipMemcpyHostToDevice, c->stream) != hipSuccess ||
            hipMemcpyAsync(c->cm, hmu.data(), CS * 8, hipMemcpyHostToDevice, c->stream) != hipSuccess ||
            hipMemcpyAsync(c->mw, hmw.data(), CS * 8, hipMemcpyHostToDevice, c->stream) != hipSuccess) {
            c->err = "uploading coefficients failed";
            return fail(ELWH_ERR_HIP);
        }
        if (mapped) {
            bool ok = hipMemcpyAsync(c->jac, hj.data(), CS * 8, hipMemcpyHostToDevice, c->stream) == hipSuccess;
            for (int k = 0; k < nmetric && ok; ++k)
                ok = hipMemcpyAsync(c->cg[k], hg[k].data(), CS * 8, hipMemcpyHostToDevice, c->stream) == hipSuccess;
            if (!ok) {
                c->err = "uploading the metric failed";
                return fail(ELWH_ERR_HIP);
            }
            if (o.prec == ELWH_FP32_STEP)
                for (int k = 0; k < nmetric; ++k) launch_convert_f32(L, c->cg[k], c->fg[k], 1, c->stream);
        }
        if (o.prec == ELWH_FP32_STEP) {
            launch_convert_f32(L, c->ca, c->fa, 1, c->stream);
            launch_convert_f32(L, c->cl, c->fl, 1, c->stream);
            launch_convert_f32(L, c->cm, c->fm, 1, c->stream);
        }
        if (hipStreamSynchronize(c->stream) != hipSuccess) {
            c->err = "stream synchronisation failed in create";
            return fail(ELWH_ERR_HIP);
        }
    }
    if (imp[0] || imp[1] || ximp[0] || ximp[1]) {
        // damping g = c dt Bt / 2 of the face rows and columns, B = 2 c / h
        // (c = c_p for the normal, c_s for the tangential component, h the
        // spacing normal to the face), Bt = B omega dt / sin(omega dt) for the
        // corrected scheme; the velocity accumulator and the second input field
        const size_t P = (size_t)L.P, NY = (size_t)L.ny + 1;
        if ((st = alloc_t(c, &c->dmp, 4 * P)) || (st = alloc_t(c, &c->dmpx, 4 * NY)) ||
            (st = alloc_t(c, &c->acc1, FE)) || (st = alloc_t(c, &c->x1, FE)))
            return fail(st);
        std::vector<double> hd(4 * P, 0.0), hdx(4 * NY, 0.0);
        const double hx = grid->len[0] / grid->n[0], hy = grid->len[1] / grid->n[1];
        const double wdt = omega * c->plan.dt;
        const double rescale = o.scheme == ELWH_SCHEME_CORRECTED ? wdt / std::sin(wdt) : 1.0;
        const double gfac = 0.5 * c->plan.c * c->plan.dt * rescale * 2.0;
        auto cs_at = [&](int64_t k) { return std::sqrt(hm[k] / hr[k]); };
        auto cp_at = [&](int64_t k) { return std::sqrt((hl[k] + 2.0 * hm[k]) / hr[k]); };
        for (int side = 0; side < 2; ++side) {
            if (imp[side]) {
                const int j = side ? L.ny : 0;
                for (int x = 0; x <= L.nx; ++x) {
                    const int64_t src = (int64_t)j * (L.nx + 1) + x;
                    hd[(2 * side) * P + x] = gfac / hy * cs_at(src);       // u tangential
                    hd[(2 * side + 1) * P + x] = gfac / hy * cp_at(src);   // v normal
                }
            }
            if (ximp[side]) {
                const int x = side ? L.nx : 0;
                for (int j = 0; j <= L.ny; ++j) {
                    const int64_t src = (int64_t)j * (L.nx + 1) + x;
                    hdx[(2 * side) * NY + j] = gfac / hx * cp_at(src);     // u normal
                    hdx[(2 * side + 1) * NY + j] = gfac / hx * cs_at(src); // v tangential
                }
            }
        }
        if (hipMemcpyAsync(c->dmp, hd.data(), 4 * P * 8, hipMemcpyHostToDevice, c->stream) != hipSuccess ||
            hipMemcpyAsync(c->dmpx, hdx.data(), 4 * NY * 8, hipMemcpyHostToDevice, c->stream) != hipSuccess ||
            hipStreamSynchronize(c->stream) != hipSuccess) {
            c->err = "uploading the damping rows failed";
            return fail(ELWH_ERR_HIP);
        }
    }
    // default tiling, then (optionally) the timed choice
    if (mapped3) {
        c->tile64 = Tile{1, 4};
        c->tile32 = Tile{1, 4};
    } else if (mapped) {
        c->tile64 = Tile{1, 8};
        c->tile32 = Tile{2, 8};
    } else if (imp[0] || imp[1] || ximp[0] || ximp[1]) {
        c->tile64 = Tile{1, 8};   // the two-field step kernel (fewer registers at V = 1)
        c->tile32 = Tile{4, 8};
    } else if (c->L.dim == 2) {
        c->tile64 = Tile{2, 8};
        c->tile32 = Tile{4, 8};
    } else if (o.fuse >= 2) {
        c->tile64 = Tile{6, 32};   // two-step launches: RB rows (plus two halo rows), TZ planes
        c->tile32 = Tile{6, 32};
    } else {
        c->tile64 = Tile{1, 16};
        c->tile32 = Tile{1, 16};
    }
    if (o.autotune) {
        if ((st = elwh_autotune(c, ELWH_FP64, 2, nullptr)) != ELWH_OK) return fail(st);
        if (o.prec == ELWH_FP32_STEP && (st = elwh_autotune(c, ELWH_FP32_STEP, 2, nullptr)) != ELWH_OK)
            return fail(st);
    }
    *out = c;
    return ELWH_OK;
}

}  // namespace

extern "C" {

void elwh_default_opts(elwh_opts* o) {
    if (!o) return;
    o->cfl = 0.8;
    o->nt = 0;
    o->periods = 1;
    o->prec = ELWH_FP64;
    o->krylov = ELWH_KRYLOV_CG;
    o->gmres_m = 30;
    o->scheme = ELWH_SCHEME_CORRECTED;
    o->compensated = 1;
    o->inner_tol = 1e-2;
    o->max_outer = 50;
    o->stream = nullptr;
    o->autotune = 1;
    o->fuse = 4;
    o->scale_x0 = 0;
    o->cr_fallback = 1;
    o->fp64_fallback = 1;
    o->fp32_switch = 0.0;
}

elwh_status elwh_plan(const elwh_grid* grid, const double* rho, const double* lam, const double* mu, double omega,
                      const int bc[6], const elwh_opts* opts, elwh_info* info) {
    elwh_opts o;
    elwh_default_opts(&o);
    if (opts) o = *opts;
    if (!bc) {
        g_create_err = "null bc";
        return ELWH_ERR_ARG;
    }
    int bcp[6];
    for (int f = 0; f < 6; ++f) bcp[f] = bc[f] == ELWH_BC_IMPEDANCE ? ELWH_BC_TRACTION_FREE : bc[f];
    const bool x_free_ok = grid && grid->dim == 2 && (bc[0] == ELWH_BC_IMPEDANCE || bc[1] == ELWH_BC_IMPEDANCE);
    Plan p;
    elwh_status st = make_plan(grid, rho, lam, mu, omega, bcp, &o, &p, &g_create_err, x_free_ok);
    if (st != ELWH_OK) return st;
    if (info) {
        std::memset(info, 0, sizeof(*info));
        info->nt = p.nt;
        info->dt = p.dt;
        info->c = p.c;
        info->lambda_bound = p.lambda_bound;
    }
    return ELWH_OK;
}

elwh_status elwh_create(const elwh_grid* grid, const double* rho, const double* lam, const double* mu,
                        double omega, const int bc[6], const elwh_opts* opts, elwh_ctx** out) {
    return create_impl(grid, nullptr, nullptr, nullptr, rho, lam, mu, omega, bc, opts, out);
}

elwh_status elwh_create_mapped(const elwh_grid* grid, const double* x, const double* y, const double* rho,
                               const double* lam, const double* mu, double omega, const int bc[4],
                               const elwh_opts* opts, elwh_ctx** out) {
    if (!x || !y) {
        if (out) *out = nullptr;
        g_create_err = "null coordinate array";
        return ELWH_ERR_ARG;
    }
    return create_impl(grid, x, y, nullptr, rho, lam, mu, omega, bc, opts, out);
}

elwh_status elwh_filter_diagnostics(int nt, int periods, double omega, int scheme, elwh_filter_diag* out) {
    return filter_diagnostics(nt, periods, omega, scheme, out, &g_create_err);
}

elwh_status elwh_create_mapped3(const elwh_grid* grid, const double* x, const double* y, const double* z,
                                const double* rho, const double* lam, const double* mu, double omega, const int bc[6],
                                const elwh_opts* opts, elwh_ctx** out) {
    if (!x || !y || !z) {
        if (out) *out = nullptr;
        g_create_err = "null coordinate array";
        return ELWH_ERR_ARG;
    }
    return create_impl(grid, x, y, z, rho, lam, mu, omega, bc, opts, out);
}

elwh_status elwh_plan_mapped3(const elwh_grid* grid, const double* x, const double* y, const double* z,
                              const double* rho, const double* lam, const double* mu, double omega, const int bc[6],
                              const elwh_opts* opts, elwh_info* info) {
    elwh_opts o;
    elwh_default_opts(&o);
    if (opts) o = *opts;
    if (!bc) {
        g_create_err = "null bc";
        return ELWH_ERR_ARG;
    }
    Plan p;
    elwh_status st = make_plan_mapped3(grid, x, y, z, rho, lam, mu, omega, bc, &o, &p, nullptr, &g_create_err);
    if (st != ELWH_OK) return st;
    if (info) {
        std::memset(info, 0, sizeof(*info));
        info->nt = p.nt;
        info->dt = p.dt;
        info->c = p.c;
        info->lambda_bound = p.lambda_bound;
    }
    return ELWH_OK;
}

elwh_status elwh_plan_mapped(const elwh_grid* grid, const double* x, const double* y, const double* rho,
                             const double* lam, const double* mu, double omega, const int bc[4],
                             const elwh_opts* opts, elwh_info* info) {
    elwh_opts o;
    elwh_default_opts(&o);
    if (opts) o = *opts;
    if (!bc) {
        g_create_err = "null bc";
        return ELWH_ERR_ARG;
    }
    int bc6[6] = {bc[0], bc[1], bc[2], bc[3], ELWH_BC_DIRICHLET, ELWH_BC_DIRICHLET};
    Plan p;
    elwh_status st = make_plan_mapped(grid, x, y, rho, lam, mu, omega, bc6, &o, &p, nullptr, &g_create_err);
    if (st != ELWH_OK) return st;
    if (info) {
        std::memset(info, 0, sizeof(*info));
        info->nt = p.nt;
        info->dt = p.dt;
        info->c = p.c;
        info->lambda_bound = p.lambda_bound;
    }
    return ELWH_OK;
}

void elwh_destroy(elwh_ctx* c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    free_all(c);
    delete c;
}

elwh_status elwh_query(const elwh_ctx* c, elwh_info* info) {
    if (!c || !info) return ELWH_ERR_ARG;
    std::memset(info, 0, sizeof(*info));
    info->nt = c->plan.nt;
    info->dt = c->plan.dt;
    info->c = c->plan.c;
    info->lambda_bound = c->plan.lambda_bound;
    info->napply = c->napply;
    return ELWH_OK;
}

const char* elwh_last_error(const elwh_ctx* c) { return c ? c->err.c_str() : g_create_err.c_str(); }

elwh_status elwh_apply_filter(elwh_ctx* c, const double* u0, const double* f, double* out) {
    if (!c || !u0 || !out) return ELWH_ERR_ARG;
    if (c->imp[0] || c->imp[1] || c->ximp[0] || c->ximp[1]) {
        c->err = "a context with impedance faces takes the two-field entry points (elwh_apply_filter2, "
                 "elwh_apply_A2, elwh_solve2)";
        return ELWH_ERR_ARG;
    }
    const bool fp32 = c->opts.prec == ELWH_FP32_STEP;
    launch_pack(c->L, c->bc, u0, c->vec[VX], c->L.dim, c->stream);
    if (f) {
        pack_forcing(c, f, fp32);
    }
    run_filter(c, c->vec[VX], f != nullptr, false, fp32, c->vec[VQ]);
    launch_unpack(c->L, c->bc, c->vec[VQ], out, c->L.dim, c->stream);
    HIPCK(hipGetLastError());
    return ELWH_OK;
}

elwh_status elwh_apply_A(elwh_ctx* c, const double* x, double* y) {
    if (!c || !x || !y) return ELWH_ERR_ARG;
    if (c->imp[0] || c->imp[1]) {
        c->err = "a context with impedance faces takes the two-field entry points (elwh_apply_filter2, "
                 "elwh_apply_A2, elwh_solve2)";
        return ELWH_ERR_ARG;
    }
    const bool fp32 = c->opts.prec == ELWH_FP32_STEP;
    launch_pack(c->L, c->bc, x, c->vec[VX], c->L.dim, c->stream);
    apply_A(c, c->vec[VX], c->vec[VQ], fp32);
    launch_unpack(c->L, c->bc, c->vec[VQ], y, c->L.dim, c->stream);
    HIPCK(hipGetLastError());
    return ELWH_OK;
}

elwh_status elwh_dot_M(elwh_ctx* c, const double* x, const double* y, double* out) {
    if (!c || !x || !y || !out) return ELWH_ERR_ARG;
    launch_pack(c->L, c->bc, x, c->vec[VT], c->L.dim, c->stream);
    launch_pack(c->L, c->bc, y, c->vec[VD], c->L.dim, c->stream);
    return dot_host(c, c->vec[VT], c->vec[VD], out);
}

}  // extern "C"

namespace {

elwh_status impedance_error(elwh_ctx* c) {
    c->err = "a context with impedance faces takes the two-field entry points (elwh_apply_filter2, "
             "elwh_apply_A2, elwh_solve2)";
    return ELWH_ERR_ARG;
}

// b = Pi_h 0 (VB) with the forcing f, FP64 stepping; *bb = ||b||_M^2.
elwh_status prepare_rhs(elwh_ctx* c, const double* f, double* bb) {
    pack_forcing(c, f, false);
    compute_rhs(c);
    CKST(dot_host(c, c->vec[VB], c->vec[VB], bb));
    if (!std::isfinite(*bb)) {
        c->err = "non-finite right-hand side";
        return ELWH_ERR_ARG;
    }
    return ELWH_OK;
}

void load_start(elwh_ctx* c, const double* x0) {
    if (x0)
        launch_pack(c->L, c->bc, x0, c->vec[VX], c->L.dim, c->stream);
    else
        (void)hipMemsetAsync(c->vec[VX], 0, c->L.field_elems() * sizeof(double), c->stream);
}

// Stepwise CG from x0 once b is in VB (bb > 0): r = b - A_h x0, p = r.
elwh_status cg_begin_rhs(elwh_ctx* c, const double* x0) {
    load_start(c, x0);
    c->alphas.clear();
    c->betas.clear();
    double rr;
    CKST(cg_start(c, c->vec[VB], c->vec[VX], x0 == nullptr, c->vec[VR], c->vec[VP], c->vec[VQ], false, &c->cg_bb,
                  &rr));
    c->cg_iters = 0;
    c->cg_active = true;
    c->cg_qready = false;
    c->cg_zero = false;
    return ELWH_OK;
}

// Zero right-hand side: the solution of A_h v = 0 is v = 0.
elwh_status cg_begin_zero(elwh_ctx* c) {
    HIPCK(hipMemsetAsync(c->vec[VX], 0, c->L.field_elems() * sizeof(double), c->stream));
    HIPCK(hipMemsetAsync(c->vec[VR], 0, c->L.field_elems() * sizeof(double), c->stream));
    c->alphas.clear();
    c->betas.clear();
    c->cg_bb = 0.0;
    c->cg_iters = 0;
    c->cg_active = true;
    c->cg_qready = false;
    c->cg_zero = true;
    return ELWH_OK;
}

void fill_plan(const elwh_ctx* c, elwh_info* info) {
    info->nt = c->plan.nt;
    info->dt = c->plan.dt;
    info->c = c->plan.c;
    info->lambda_bound = c->plan.lambda_bound;
}

// v = x and the CG record; known_relfp64 >= 0 is a true residual of the
// current x computed already (saves one application).
elwh_status cg_result_impl(elwh_ctx* c, double* v, elwh_info* info, double known_relfp64) {
    if (v) launch_unpack(c->L, c->bc, c->vec[VX], v, c->L.dim, c->stream);
    if (info) {
        std::memset(info, 0, sizeof(*info));
        info->iters = c->cg_iters;
        fill_plan(c, info);
        if (c->cg_zero) {
            info->relres = info->relres_fp64 = 0.0;
            info->cond_est = NAN;
        } else {
            double rr;
            CKST(dot_host(c, c->vec[VR], c->vec[VR], &rr));
            info->relres = std::sqrt(rr / c->cg_bb);
            if (known_relfp64 >= 0)
                info->relres_fp64 = known_relfp64;
            else
                CKST(final_residual(c, c->vec[VX], c->cg_bb, &info->relres_fp64));
            info->cond_est = lanczos_cond(c->alphas, c->betas);
        }
        info->napply = c->napply;
    }
    HIPCK(hipStreamSynchronize(c->stream));
    return ELWH_OK;
}

}  // namespace

extern "C" {

elwh_status elwh_cg_begin(elwh_ctx* c, const double* f, const double* x0) {
    if (!c || !f) return ELWH_ERR_ARG;
    if (c->imp[0] || c->imp[1]) return impedance_error(c);
    if (c->opts.prec != ELWH_FP64) {
        c->err = "the stepwise CG interface is FP64 only";
        return ELWH_ERR_ARG;
    }
    double bb;
    CKST(prepare_rhs(c, f, &bb));
    return bb > 0 ? cg_begin_rhs(c, x0) : cg_begin_zero(c);
}

elwh_status elwh_cg_iterate(elwh_ctx* c, int k, double tol, double* relres) {
    if (!c || !c->cg_active || k < 0) return ELWH_ERR_ARG;
    if (c->cg_zero) {
        if (relres) *relres = 0.0;
        return ELWH_OK;
    }
    CGOut o;
    elwh_status st = cg_steps_pipelined(c, c->vec[VX], c->vec[VR], c->vec[VP], c->vec[VQ], c->cg_bb, k, tol, &o);
    c->cg_iters += o.iters;
    if (relres) *relres = o.relres;
    return st;
}

elwh_status elwh_cg_result(elwh_ctx* c, double* v, elwh_info* info) {
    if (!c || !c->cg_active) return ELWH_ERR_ARG;
    return cg_result_impl(c, v, info, -1.0);
}

elwh_status elwh_solve(elwh_ctx* c, const double* f, const double* x0, double tol, int maxit, double* v,
                       elwh_info* info) {
    if (!c || !f || !v || maxit < 0) return ELWH_ERR_ARG;
    if (c->imp[0] || c->imp[1]) return impedance_error(c);
    c->napply = 0;
    elwh_info inf;
    std::memset(&inf, 0, sizeof(inf));
    fill_plan(c, &inf);
    elwh_status st = ELWH_OK;
    double bb;
    CKST(prepare_rhs(c, f, &bb));
    if (!(bb > 0)) {
        // A_h v = 0: v = 0 whatever the start
        HIPCK(hipMemsetAsync(c->vec[VX], 0, c->L.field_elems() * sizeof(double), c->stream));
        launch_unpack(c->L, c->bc, c->vec[VX], v, c->L.dim, c->stream);
        HIPCK(hipStreamSynchronize(c->stream));
        inf.napply = c->napply;
        if (info) *info = inf;
        return ELWH_OK;
    }

    if (c->opts.prec == ELWH_FP64 && c->opts.krylov == ELWH_KRYLOV_CG) {
        CKST(cg_begin_rhs(c, x0));
        keep_start(c);
        double rel = 0;
        st = elwh_cg_iterate(c, maxit, tol, &rel);
        // Convergence is judged on the true residual: once the recurrence
        // residual meets tol, r is replaced by b - A_h x from an FP64
        // application and CG goes on along the same search direction until the
        // true residual meets tol too (a reliable update).
        double relfp64 = -1.0;
        int replaced = 0;
        for (int rep = 0; st == ELWH_OK && tol > 0; ++rep) {
            double rr;
            CKST(final_residual(c, c->vec[VX], c->cg_bb, &relfp64));   // VT = b - A_h x
            if (relfp64 <= tol) break;
            if (c->cg_iters >= maxit || rep + 1 >= kMaxReplace) {
                st = ELWH_ERR_NOT_CONVERGED;
                break;
            }
            rr = relfp64 * relfp64 * c->cg_bb;
            launch_copy(c, c->vec[VT], c->vec[VR], c->stream);
            CKST(set_scalar(c, S_RR, rr));
            c->cg_qready = false;   // final_residual overwrote q
            relfp64 = -1.0;
            ++replaced;
            st = elwh_cg_iterate(c, maxit - c->cg_iters, tol, &rel);
        }
        if (st == ELWH_ERR_BREAKDOWN && c->opts.cr_fallback) {
            // A_h slightly indefinite: CR or MINRES from the start
            int it = 0;
            double relfb = 1.0;
            back_to_start(c);
            st = solve_checked(c, c->opts.cr_fallback == 2 ? solve_minres : solve_cr, x0 == nullptr, tol,
                               std::max(1, maxit - c->cg_iters), &it, &relfb, &relfp64);
            if (st != ELWH_OK && st != ELWH_ERR_NOT_CONVERGED) return st;
            CKST(cg_result_impl(c, v, &inf, relfp64));
            inf.cr_iters = it;
            inf.relres = relfb;
        } else {
            if (st != ELWH_OK && st != ELWH_ERR_NOT_CONVERGED) return st;
            CKST(cg_result_impl(c, v, &inf, relfp64));
        }
        inf.outer = replaced;
        if (tol > 0) st = inf.relres_fp64 <= tol ? ELWH_OK : ELWH_ERR_NOT_CONVERGED;
    } else if (c->opts.prec == ELWH_FP64) {
        load_start(c, x0);
        int it = 0;
        double rel = 0, relfp64 = -1.0;
        if (c->opts.krylov == ELWH_KRYLOV_GMRES)
            st = solve_gmres(c, x0 == nullptr, tol, maxit, &it, &rel);
        else
            st = solve_checked(c, c->opts.krylov == ELWH_KRYLOV_MINRES ? solve_minres : solve_cr, x0 == nullptr, tol,
                               maxit, &it, &rel, &relfp64);
        if (st != ELWH_OK && st != ELWH_ERR_NOT_CONVERGED) return st;
        inf.iters = it;
        inf.relres = rel;
        if (relfp64 >= 0)
            inf.relres_fp64 = relfp64;
        else
            CKST(final_residual(c, c->vec[VX], bb, &inf.relres_fp64));
        if (tol > 0) st = inf.relres_fp64 <= tol ? ELWH_OK : ELWH_ERR_NOT_CONVERGED;
        launch_unpack(c->L, c->bc, c->vec[VX], v, c->L.dim, c->stream);
    } else {
        // FP32 stepping inside CG with FP64 reliable updates.  x, r, p and
        // every inner product stay FP64; A_h p is applied with FP32 stepping.
        // A segment runs until the recursive residual has fallen by inner_tol
        // (or below the target); then r is replaced by b - A_h x from an FP64
        // application and the search direction continues from it
        // (p = r + beta p with beta = (r, r)_M / (r_k, r_k)_M of the last CG
        // step).  Restarting CG at every replacement instead discards the
        // Krylov space and costs two to three times the iterations here.
        load_start(c, x0);
        auto true_residual = [&](bool xzero, double* rr, bool first) -> elwh_status {
            if (xzero) {
                launch_copy(c, c->vec[VB], c->vec[VR], c->stream);
            } else {
                apply_A(c, c->vec[VX], c->vec[VT], false);
                if (first && c->opts.scale_x0) CKST(scale_start(c, c->vec[VB], c->vec[VX], c->vec[VT]));
                launch_copy(c, c->vec[VB], c->vec[VR], c->stream);
                launch_axpby(c, -1.0, c->vec[VT], 1.0, c->vec[VR], c->stream);
            }
            CKST(dot_host(c, c->vec[VR], c->vec[VR], rr));
            if (!std::isfinite(*rr)) {
                c->err = "non-finite residual: the time step is unstable";
                return ELWH_ERR_UNSTABLE;
            }
            return ELWH_OK;
        };
        double rr;
        CKST(true_residual(x0 == nullptr, &rr, true));
        keep_start(c);
        launch_copy(c, c->vec[VR], c->vec[VP], c->stream);
        CKST(set_scalar(c, S_RR, rr));
        CKST(set_scalar(c, S_FLAG, 0.0));
        double relfp64 = std::sqrt(rr / bb), seg = rr;
        inf.relres = relfp64;
        int outer = 0, iters = 0;
        bool finished = false;   // set when the FP64 phase ends the solve (CG breakdown)
        // FP64 first (opts.fp32_switch > 0): CG with FP64 applications down to
        // the switch residual, then a residual replacement that keeps the
        // search direction, and the FP32 segments below continue the same
        // Krylov sequence.
        const double sw = std::max(c->opts.fp32_switch, tol);
        if (c->opts.fp32_switch > 0 && tol > 0 && relfp64 > sw && maxit > 0) {
            CGOut o;
            const elwh_status si = cg_steps(c, c->vec[VX], c->vec[VR], c->vec[VP], c->vec[VQ], false, bb, maxit, sw,
                                            &o, false);
            iters += o.iters;
            inf.fp64_iters += o.iters;
            inf.relres = o.relres;
            if (si == ELWH_ERR_BREAKDOWN && c->opts.cr_fallback) {
                int it = 0;
                double relcr = 1.0, relchk = -1.0;
                back_to_start(c);
                st = solve_checked(c, c->opts.cr_fallback == 2 ? solve_minres : solve_cr, false, tol,
                                   std::max(1, maxit - iters), &it, &relcr, &relchk);
                if (st != ELWH_OK && st != ELWH_ERR_NOT_CONVERGED) return st;
                inf.cr_iters = it;
                inf.relres = relcr;
                CKST(final_residual(c, c->vec[VX], bb, &relfp64));
                st = relfp64 <= tol ? ELWH_OK : ELWH_ERR_NOT_CONVERGED;
                finished = true;
            } else if (si != ELWH_OK) {
                return si;
            } else if (o.converged) {
                // (not converged: maxit was reached, and the loop below ends)
                const double rr_new = c->hscal[S_RR], beta_k = c->hscal[S_BETA];
                const double rr_k = beta_k > 0 ? rr_new / beta_k : 0.0;
                CKST(true_residual(false, &rr, false));
                relfp64 = std::sqrt(rr / bb);
                seg = rr;
                CKST(set_scalar(c, S_BETA, rr_k > 0 ? rr / rr_k : 0.0));
                CKST(set_scalar(c, S_RR, rr));
                launch_cg_update_p(c, c->vec[VP], c->vec[VR], c->stream);
            } else {
                relfp64 = o.relres;
            }
        }
        std::vector<double> hist{relfp64};   // FP64 residual after each segment
        bool stagnated = false;
        int longest = 0;                      // iterations of the longest segment so far
        st = finished ? st : ELWH_ERR_NOT_CONVERGED;
        while (!finished) {
            if (tol > 0 && relfp64 <= tol) {
                st = ELWH_OK;
                break;
            }
            if (iters >= maxit || outer > c->opts.max_outer) {
                if (tol <= 0) st = ELWH_OK;
                break;
            }
            // stop the segment at rr <= max(inner_tol^2 seg, (tol/2)^2 bb)
            const double tseg = std::max(c->opts.inner_tol, tol > 0 ? 0.5 * tol * std::sqrt(bb / seg) : 0.0);
            // with the fallback on, a segment may take at most twice the
            // iterations of the longest earlier one (at least 64)
            int budget = maxit - iters;
            const bool capped = c->opts.fp64_fallback && tol > 0 && outer > 0 && budget > std::max(64, 2 * longest);
            if (capped) budget = std::max(64, 2 * longest);
            CGOut o;
            elwh_status si = cg_steps(c, c->vec[VX], c->vec[VR], c->vec[VP], c->vec[VQ], true, seg, budget,
                                      tseg, &o, false);
            if (si == ELWH_ERR_BREAKDOWN && c->opts.cr_fallback) {
                // conjugate residual (or MINRES) in FP64 from the start
                iters += o.iters;
                int it = 0;
                double relcr = 1.0, relchk = -1.0;
                back_to_start(c);
                st = solve_checked(c, c->opts.cr_fallback == 2 ? solve_minres : solve_cr, false, tol,
                                   std::max(1, maxit - iters), &it, &relcr, &relchk);
                if (st != ELWH_OK && st != ELWH_ERR_NOT_CONVERGED) return st;
                inf.cr_iters = it;
                inf.relres = relcr;
                CKST(final_residual(c, c->vec[VX], bb, &relfp64));
                if (tol > 0) st = relfp64 <= tol ? ELWH_OK : ELWH_ERR_NOT_CONVERGED;
                break;
            }
            if (si != ELWH_OK) return si;
            iters += o.iters;
            ++outer;
            longest = std::max(longest, o.iters);
            const double rr_new = c->hscal[S_RR], beta_k = c->hscal[S_BETA];
            inf.relres = std::sqrt(rr_new / bb);
            const double rr_k = beta_k > 0 ? rr_new / beta_k : 0.0;
            CKST(true_residual(false, &rr, false));
            relfp64 = std::sqrt(rr / bb);
            seg = rr;
            hist.push_back(relfp64);
            if (c->opts.fp64_fallback && tol > 0 && relfp64 > tol && iters < maxit &&
                ((capped && !o.converged) || (hist.size() >= 3 && relfp64 > 0.5 * hist[hist.size() - 3]))) {
                stagnated = true;   // a segment over its cap, or less than a halving over two segments
                break;
            }
            if (!o.converged) continue;   // out of iterations: the loop head ends it
            CKST(set_scalar(c, S_BETA, rr_k > 0 ? rr / rr_k : 0.0));
            CKST(set_scalar(c, S_RR, rr));
            launch_cg_update_p(c, c->vec[VP], c->vec[VR], c->stream);
        }
        if (stagnated) {
            // FP32 applications no longer improve x: FP64 CG from x (r = b - A_h x)
            const int keep = c->opts.scale_x0;
            c->opts.scale_x0 = 0;
            double bb2 = 0, rr2 = 0;
            keep_start(c);   // a new CG sequence starts here
            const elwh_status s0 = cg_start(c, c->vec[VB], c->vec[VX], false, c->vec[VR], c->vec[VP], c->vec[VQ],
                                            false, &bb2, &rr2);
            c->opts.scale_x0 = keep;
            CKST(s0);
            c->cg_qready = false;
            // The pipelined recurrence stops on its own residual, which can sit
            // well below the true one: when b - A_h x is still above tol, CG
            // restarts from x (r = b - A_h x), at most kMaxReplace times.
            for (int rep = 0;; ++rep) {
                CGOut o2;
                st = cg_steps_pipelined(c, c->vec[VX], c->vec[VR], c->vec[VP], c->vec[VQ], bb2, maxit - iters, tol,
                                        &o2);
                inf.fp64_iters += o2.iters;
                iters += o2.iters;
                inf.relres = o2.relres;
                if (st == ELWH_ERR_BREAKDOWN && c->opts.cr_fallback) {
                    int it = 0;
                    double relcr = 1.0, relchk = -1.0;
                    back_to_start(c);
                    st = solve_checked(c, c->opts.cr_fallback == 2 ? solve_minres : solve_cr, false, tol,
                                       std::max(1, maxit - iters), &it, &relcr, &relchk);
                    inf.cr_iters = it;
                    inf.relres = relcr;
                    if (st != ELWH_OK && st != ELWH_ERR_NOT_CONVERGED) return st;
                    CKST(final_residual(c, c->vec[VX], bb, &relfp64));
                    break;
                }
                if (st != ELWH_OK && st != ELWH_ERR_NOT_CONVERGED) return st;
                CKST(final_residual(c, c->vec[VX], bb, &relfp64));
                if (relfp64 <= tol || st != ELWH_OK || iters >= maxit || rep + 1 >= kMaxReplace) break;
                ++outer;
                c->opts.scale_x0 = 0;
                keep_start(c);
                const elwh_status s1 = cg_start(c, c->vec[VB], c->vec[VX], false, c->vec[VR], c->vec[VP],
                                                c->vec[VQ], false, &bb2, &rr2);
                c->opts.scale_x0 = keep;
                CKST(s1);
                c->cg_qready = false;
            }
            st = relfp64 <= tol ? ELWH_OK : ELWH_ERR_NOT_CONVERGED;
        }
        inf.iters = iters;
        inf.outer = outer;
        inf.relres_fp64 = relfp64;
        launch_unpack(c->L, c->bc, c->vec[VX], v, c->L.dim, c->stream);
    }
    HIPCK(hipStreamSynchronize(c->stream));
    inf.napply = c->napply;
    if (info) *info = inf;
    return st;
}

elwh_status elwh_profile_enable(elwh_ctx* c, int on) {
    if (!c) return ELWH_ERR_ARG;
    HIPCK(hipStreamSynchronize(c->stream));
    c->prof_on = on != 0;
    c->prof_used = 0;
    return ELWH_OK;
}

elwh_status elwh_profile_read(elwh_ctx* c, double* step_ms, int* nstep, double* init_ms, int* ninit) {
    if (!c) return ELWH_ERR_ARG;
    HIPCK(hipStreamSynchronize(c->stream));
    double ts = 0, ti = 0;
    int ns = 0, ni = 0;
    for (size_t k = 0; k < c->prof_used; ++k) {
        float m1 = 0.f, m2 = 0.f;
        HIPCK(hipEventElapsedTime(&m1, c->prof_ev[3 * k], c->prof_ev[3 * k + 1]));
        HIPCK(hipEventElapsedTime(&m2, c->prof_ev[3 * k + 1], c->prof_ev[3 * k + 2]));
        ti += m1;
        ni++;
        ts += m2;
        ns += c->prof_nsteps[k];
    }
    c->prof_used = 0;
    if (step_ms) *step_ms = ts;
    if (nstep) *nstep = ns;
    if (init_ms) *init_ms = ti;
    if (ninit) *ninit = ni;
    return ELWH_OK;
}

elwh_status elwh_set_tile(elwh_ctx* c, int prec, int vec, int rows) {
    if (!c) return ELWH_ERR_ARG;
    const bool fp32 = prec == ELWH_FP32_STEP;
    const bool ok = c->mapped ? (c->L.dim == 3 ? tile_valid_curv3(fp32, vec, rows) : tile_valid_curv(fp32, vec, rows))
                              : (c->L.dim == 2 ? tile_valid_2d(fp32, vec, rows)
                                               : (c->opts.fuse >= 2 ? tile_valid_3d_k2(fp32, vec, rows)
                                                                    : tile_valid_3d(fp32, vec, rows)));
    if (!ok) {
        c->err = "unsupported tile";
        return ELWH_ERR_ARG;
    }
    Tile& t = fp32 ? c->tile32 : c->tile64;
    t.V = vec;
    t.TY = rows;
    return ELWH_OK;
}

}  // extern "C"

namespace {
void run_filter_twofield(elwh_ctx* c, const double* x0, const double* z1, bool with_force, bool amode, double s_in,
                         double s_out, double* out0, double* out1);
// dim, prec, variant (bit 0: compensated accumulator, bits 1-2: steps per
// 2-D launch minus one, bit 3: mapped grid, bit 4: two-field step), nx, ny, nz
using TuneKey = std::tuple<int, int, int, int, int, int>;
std::mutex g_tune_mu;
std::map<TuneKey, Tile> g_tune;

std::string device_arch() {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');
    return colon == std::string::npos ? a : a.substr(0, colon);
}

bool file_lookup(const TuneKey& k, const std::string& arch, Tile* t) {
    const char* path = std::getenv("ELWH_TUNE_CACHE");
    if (!path) return false;
    FILE* fp = std::fopen(path, "r");
    if (!fp) return false;
    char line[512], a[64];
    bool found = false;
    while (std::fgets(line, sizeof line, fp)) {
        int dim, prec, comp, nx, ny, nz, V, rows;
        double us;
        if (std::sscanf(line, "{\"arch\": \"%63[^\"]\", \"dim\": %d, \"prec\": %d, \"variant\": %d, \"n\": [%d, %d, %d], "
                              "\"V\": %d, \"rows\": %d, \"us\": %lf}",
                        a, &dim, &prec, &comp, &nx, &ny, &nz, &V, &rows, &us) == 10 &&
            arch == a && k == TuneKey(dim, prec, comp, nx, ny, nz)) {
            t->V = V;
            t->TY = rows;
            found = true;
        }
    }
    std::fclose(fp);
    return found;
}

void file_store(const TuneKey& k, const std::string& arch, const Tile& t, double us) {
    const char* path = std::getenv("ELWH_TUNE_CACHE");
    if (!path) return;
    FILE* fp = std::fopen(path, "a");
    if (!fp) return;
    std::fprintf(fp,
                 "{\"arch\": \"%s\", \"dim\": %d, \"prec\": %d, \"variant\": %d, \"n\": [%d, %d, %d], \"V\": %d, "
                 "\"rows\": %d, \"us\": %.3f}\n",
                 arch.c_str(), std::get<0>(k), std::get<1>(k), std::get<2>(k), std::get<3>(k), std::get<4>(k),
                 std::get<5>(k), t.V, t.TY, us);
    std::fclose(fp);
}
}  // namespace

extern "C" {

elwh_status elwh_autotune(elwh_ctx* c, int prec, int reps, double* best_step_us) {
    if (!c || reps < 1) return ELWH_ERR_ARG;
    const bool fp32 = prec == ELWH_FP32_STEP;
    if (fp32 && c->opts.prec != ELWH_FP32_STEP) {
        c->err = "FP32 tiling needs an FP32 context";
        return ELWH_ERR_ARG;
    }
    // a context with impedance faces runs the two-field step kernel: tune that
    const bool twofield = !fp32 && (c->imp[0] || c->imp[1] || c->ximp[0] || c->ximp[1]);
    const int steps = !c->mapped && !twofield ? (c->L.dim == 2 ? c->opts.fuse : std::min(c->opts.fuse, 2)) : 1;
    const int comp = (fp32 && c->opts.compensated ? 1 : 0) | ((steps - 1) << 1) | (c->mapped ? 8 : 0) |
                     (twofield ? 16 : 0);
    const TuneKey key(c->L.dim, fp32 ? 1 : 0, comp, c->L.nx, c->L.ny, c->L.nz);
    Tile& dst = fp32 ? c->tile32 : c->tile64;
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            dst = it->second;
            if (best_step_us) *best_step_us = -1.0;
            return ELWH_OK;
        }
    }
    const std::string arch = device_arch();
    Tile ft;
    if (file_lookup(key, arch, &ft)) {
        dst = ft;
        std::lock_guard<std::mutex> g(g_tune_mu);
        g_tune[key] = ft;
        if (best_step_us) *best_step_us = -1.0;
        return ELWH_OK;
    }
    std::vector<Tile> cands;
    if (twofield) {
        for (int V : {1, 2})
            for (int TY : {4, 8, 16})
                if (tile_valid_damped(V, TY)) cands.push_back(Tile{V, TY});
    } else if (c->mapped && c->L.dim == 3) {
        cands.push_back(Tile{1, 4});   // one tiling: a thread per node
    } else if (c->mapped) {
        for (int V : {1, 2})
            for (int TY : {8, 16})
                if (tile_valid_curv(fp32, V, TY)) cands.push_back(Tile{V, TY});
    } else if (c->L.dim == 2) {
        for (int V : {1, 2, 4})
            for (int TY : {4, 8, 10, 12, 16})
                if (tile_valid_2d(fp32, V, TY)) cands.push_back(Tile{V, TY});
    } else if (steps >= 2) {
        // two-step tilings, and single steps (RB 1) where they are faster
        for (int RB : {2, 4, 6})
            for (int TZ : {8, 16, 32, 64}) cands.push_back(Tile{RB, TZ});
        for (int TZ : {16, 32}) cands.push_back(Tile{1, TZ});
    } else {
        for (int RB : {1, 2, 4})
            for (int TZ : {8, 16, 32}) cands.push_back(Tile{RB, TZ});
    }
    double* in = c->vec[VT];
    double* out = c->vec[VD];
    HIPCK(hipMemsetAsync(in, 0, c->L.field_elems() * sizeof(double), c->stream));
    hipEvent_t e0, e1;
    HIPCK(hipEventCreate(&e0));
    HIPCK(hipEventCreate(&e1));
    const bool prof = c->prof_on;
    c->prof_on = false;
    const int napply = c->napply;
    double best = 1e300;
    Tile bt = dst;
    // three round-robin passes over the candidates, each candidate's fastest
    // pass counts: a single pass can be skewed by clock ramps and warm-up
    std::vector<double> fastest(cands.size(), 1e300);
    auto once = [&]() {
        if (twofield)
            run_filter_twofield(c, in, in, false, true, 1.0, 1.0, out, c->acc1);
        else
            apply_A(c, in, out, fp32);
    };
    bool ok = true;
    for (int pass = 0; pass < 3 && ok; ++pass) {
        for (size_t ci = 0; ci < cands.size(); ++ci) {
            dst = cands[ci];
            if (pass == 0) once();   // warm-up (first launch of this instantiation)
            (void)hipEventRecord(e0, c->stream);
            for (int r = 0; r < reps; ++r) once();
            (void)hipEventRecord(e1, c->stream);
            if (hipEventSynchronize(e1) != hipSuccess) {
                ok = false;
                break;
            }
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            fastest[ci] = std::min(fastest[ci], 1e3 * ms / reps / (c->plan.nt * c->opts.periods));
        }
    }
    for (size_t ci = 0; ci < cands.size(); ++ci)
        if (fastest[ci] < best) {
            best = fastest[ci];
            bt = cands[ci];
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->prof_on = prof;
    c->napply = napply;
    dst = bt;
    HIPCK(hipGetLastError());
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        g_tune[key] = bt;
    }
    file_store(key, arch, bt, best);
    if (best_step_us) *best_step_us = best;
    return ELWH_OK;
}

elwh_status elwh_get_tile(const elwh_ctx* c, int prec, int* vec, int* rows) {
    if (!c || !vec || !rows) return ELWH_ERR_ARG;
    const Tile& t = prec == ELWH_FP32_STEP ? c->tile32 : c->tile64;
    *vec = t.V;
    *rows = t.TY;
    return ELWH_OK;
}

}  // extern "C"

// ============================================================================
// Two-field operator for impedance y faces (the remark of Sec. 3): the filter
// acts on the pair (u0, u1) of initial displacement and velocity; GMRES on
// A_h = I - S_h of the stacked unknown z = [u0; u1 / omega] in the M inner
// product of each half.

namespace {

elwh_status twofield_ready(elwh_ctx* c) {
    if (c->mapped || c->L.dim != 2 || c->opts.prec != ELWH_FP64) {
        c->err = "the two-field operator runs on 2-D Cartesian grids in FP64";
        return ELWH_ERR_ARG;
    }
    // a context without impedance faces: allocate the two-field buffers (zero
    // damping tables) at the first two-field call
    const size_t P = (size_t)c->L.P, FE = (size_t)c->L.field_elems();
    if (!c->dmp) CKST(alloc_t(c, &c->dmp, 4 * P));
    if (!c->dmpx) CKST(alloc_t(c, &c->dmpx, 4 * ((size_t)c->L.ny + 1)));
    if (!c->acc1) CKST(alloc_t(c, &c->acc1, FE));
    if (!c->x1) CKST(alloc_t(c, &c->x1, FE));
    return ELWH_OK;
}

// out0 = sum w_n u^n, out1 = s_out sum w_n v^n for u^0 = x0 and the second
// field u1 = s_in z1 (amode: x0 - ..., z1 - ...), v^n the centred velocity.
void run_filter_twofield(elwh_ctx* c, const double* x0, const double* z1, bool with_force, bool amode, double s_in,
                         double s_out, double* out0, double* out1) {
    hipStream_t s = c->stream;
    Damp2D D;
    D.A = make_args2d(c);
    D.imp_lo = c->imp[0];
    D.imp_hi = c->imp[1];
    D.ximp_lo = c->ximp[0];
    D.ximp_hi = c->ximp[1];
    D.hx = c->grid.len[0] / c->grid.n[0];
    D.hy = c->grid.len[1] / c->grid.n[1];
    const Tile t = tile_valid_damped(c->tile64.V, c->tile64.TY) ? c->tile64 : Tile{2, 8};
    const int N = c->plan.nt * c->opts.periods;
    const double sgn = amode ? -1.0 : 1.0, dt = c->plan.dt;
    D.A.w0 = sgn * c->w[0];
    D.A.w = sgn * c->w[1];
    D.A.fc = c->cosn[0];
    D.w0v = sgn * c->w[0] * s_in * s_out;
    D.dtw = dt * s_in;
    D.wv = 0.0;
    prof_mark(c, 0);
    launch_damped2d(t.V, t.TY, 1, with_force, s, x0, z1, c->s64[1], amode ? x0 : nullptr, amode ? z1 : nullptr,
                    out0, out1, c->dmp, c->dmpx, c->ca, c->cl, c->cm, c->f64, D);
    prof_mark(c, 1);
    const double* prev = x0;
    double* cur = c->s64[1];
    for (int n = 1; n <= N; ++n) {
        // u^{n+1} over u^{n-1} when that is a state buffer, else a free one
        double* nxt = nullptr;
        for (double* b : c->s64)
            if (b == prev) nxt = b;
        if (!nxt)
            for (double* b : c->s64)
                if (b != cur && b != prev) {
                    nxt = b;
                    break;
                }
        D.A.w = n < N ? sgn * c->w[n + 1] : 0.0;   // the step past the window adds velocity only
        D.A.fc = c->cosn[n];
        D.wv = sgn * c->w[n] * s_out / (2.0 * dt);
        launch_damped2d(t.V, t.TY, 0, with_force, s, cur, prev, nxt, nullptr, nullptr, out0, out1, c->dmp, c->dmpx,
                        c->ca, c->cl, c->cm, c->f64, D);
        prev = cur;
        cur = nxt;
    }
    prof_mark(c, 2, N);
    c->napply++;
}

// Pair helpers: a two-field vector is two field vectors in the internal layout.
struct Pair {
    double* a;
    double* b;
};

elwh_status dot2(elwh_ctx* c, Pair x, Pair y, double* out) {
    double d0, d1;
    CKST(dot_host(c, x.a, y.a, &d0));
    CKST(dot_host(c, x.b, y.b, &d1));
    *out = d0 + d1;
    return ELWH_OK;
}

void axpby2(elwh_ctx* c, double a, Pair x, double b, Pair y) {
    launch_axpby(c, a, x.a, b, y.a, c->stream);
    launch_axpby(c, a, x.b, b, y.b, c->stream);
}

void copy2(elwh_ctx* c, Pair x, Pair y) {
    launch_copy(c, x.a, y.a, c->stream);
    launch_copy(c, x.b, y.b, c->stream);
}

void apply_A2(elwh_ctx* c, Pair x, Pair y) {
    run_filter_twofield(c, x.a, x.b, false, true, c->omega, 1.0 / c->omega, y.a, y.b);
}

// Restarted GMRES with classical Gram-Schmidt twice on the stacked system
// A_h z = b (z in x, b in b; x holds the start, x_zero: it is zero).
elwh_status solve_gmres2(elwh_ctx* c, Pair x, Pair b, Pair w, bool x_zero, double tol, int maxit, int* iters,
                         double* relres) {
    const int m = c->opts.gmres_m;
    const size_t FE = (size_t)c->L.field_elems();
    while ((int)c->basis2.size() < 2 * (m + 1)) {
        double* v = nullptr;
        CKST(alloc_t(c, &v, FE));
        c->basis2.push_back(v);
    }
    CKST(ensure_gm(c, m));
    {
        std::vector<double*> tab(c->basis2.begin(), c->basis2.begin() + 2 * (m + 1));
        tab.push_back(w.a);
        tab.push_back(w.b);
        HIPCK(hipMemcpyAsync(c->gm_ptrs, tab.data(), tab.size() * sizeof(double*), hipMemcpyHostToDevice,
                             c->stream));
        HIPCK(hipStreamSynchronize(c->stream));   // tab is a host temporary
    }
    const double* const* ptrs = c->gm_ptrs;
    std::vector<double> hh(2 * (m + 1) + 1);
    auto V = [&](int j) { return Pair{c->basis2[2 * j], c->basis2[2 * j + 1]}; };
    double bb;
    CKST(dot2(c, b, b, &bb));
    const double bn = std::sqrt(bb);
    if (!(bn > 0)) {
        // b = 0: the solution is zero whatever the start
        HIPCK(hipMemsetAsync(x.a, 0, FE * sizeof(double), c->stream));
        HIPCK(hipMemsetAsync(x.b, 0, FE * sizeof(double), c->stream));
        *iters = 0;
        *relres = 0.0;
        if (std::isfinite(bb)) return ELWH_OK;
        c->err = "non-finite right-hand side: the time step is unstable";
        return ELWH_ERR_UNSTABLE;
    }
    int total = 0;
    bool first = true;
    std::vector<double> H((m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
    while (true) {
        const Pair r = V(0);
        if (first && x_zero) {
            copy2(c, b, r);
        } else {
            apply_A2(c, x, w);
            copy2(c, b, r);
            axpby2(c, -1.0, w, 1.0, r);
        }
        first = false;
        double rr;
        CKST(dot2(c, r, r, &rr));
        const double beta = std::sqrt(rr);
        if (!std::isfinite(beta)) {
            c->err = "non-finite residual: the time step is unstable";
            return ELWH_ERR_UNSTABLE;
        }
        *relres = beta / bn;
        *iters = total;
        if ((tol > 0 && *relres <= tol) || total >= maxit) break;
        axpby2(c, 0.0, r, 1.0 / beta, r);
        std::fill(H.begin(), H.end(), 0.0);
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int jdone = 0;
        for (int j = 0; j < m; ++j) {
            apply_A2(c, V(j), w);
            total++;
            // classical Gram-Schmidt twice, coefficients kept on the device;
            // one host synchronisation per iteration
            for (int pass = 0; pass < 2; ++pass) {
                double* hp = c->gm_h + pass * (m + 1);
                launch_multidot2(c, ptrs, j + 1, w.a, w.b, c->gm_part, hp, c->stream);
                launch_multiaxpy2(c, ptrs, j + 1, hp, w.a, w.b, c->stream);
            }
            launch_multidot2(c, ptrs + 2 * (m + 1), 1, w.a, w.b, c->gm_part, c->gm_h + 2 * (m + 1), c->stream);
            HIPCK(hipMemcpyAsync(hh.data(), c->gm_h, hh.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
            HIPCK(hipStreamSynchronize(c->stream));
            for (int i = 0; i <= j; ++i) H[i * m + j] += hh[i] + hh[m + 1 + i];
            const double ww = hh[2 * (m + 1)];
            const double hn = std::sqrt(ww);
            H[(j + 1) * m + j] = hn;
            for (int i = 0; i < j; ++i) {
                const double tt = cs[i] * H[i * m + j] + sn[i] * H[(i + 1) * m + j];
                H[(i + 1) * m + j] = -sn[i] * H[i * m + j] + cs[i] * H[(i + 1) * m + j];
                H[i * m + j] = tt;
            }
            const double rho = std::hypot(H[j * m + j], H[(j + 1) * m + j]);
            cs[j] = H[j * m + j] / rho;
            sn[j] = H[(j + 1) * m + j] / rho;
            H[j * m + j] = rho;
            H[(j + 1) * m + j] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            jdone = j + 1;
            *relres = std::fabs(g[j + 1]) / bn;
            if ((tol > 0 && *relres <= tol) || total >= maxit || hn == 0.0) break;
            copy2(c, w, V(j + 1));
            axpby2(c, 0.0, w, 1.0 / hn, V(j + 1));
        }
        for (int i = jdone - 1; i >= 0; --i) {
            double sum = g[i];
            for (int k = i + 1; k < jdone; ++k) sum -= H[i * m + k] * y[k];
            y[i] = sum / H[i * m + i];
        }
        for (int i = 0; i < jdone; ++i) axpby2(c, y[i], V(i), 1.0, x);
    }
    *iters = total;
    return (tol > 0 && *relres > tol) ? ELWH_ERR_NOT_CONVERGED : ELWH_OK;
}

}  // namespace

extern "C" {

elwh_status elwh_apply_filter2(elwh_ctx* c, const double* u0, const double* u1, const double* f, double* out0,
                               double* out1) {
    if (!c || !u0 || !u1 || !out0 || !out1) return ELWH_ERR_ARG;
    CKST(twofield_ready(c));
    launch_pack(c->L, c->bc, u0, c->vec[VX], c->L.dim, c->stream);
    launch_pack(c->L, c->bc, u1, c->x1, c->L.dim, c->stream);
    if (f) pack_forcing(c, f, false);
    run_filter_twofield(c, c->vec[VX], c->x1, f != nullptr, false, 1.0, 1.0, c->vec[VQ], c->acc1);
    launch_unpack(c->L, c->bc, c->vec[VQ], out0, c->L.dim, c->stream);
    launch_unpack(c->L, c->bc, c->acc1, out1, c->L.dim, c->stream);
    HIPCK(hipGetLastError());
    return ELWH_OK;
}

elwh_status elwh_apply_A2(elwh_ctx* c, const double* x0, const double* x1, double* y0, double* y1) {
    if (!c || !x0 || !x1 || !y0 || !y1) return ELWH_ERR_ARG;
    CKST(twofield_ready(c));
    launch_pack(c->L, c->bc, x0, c->vec[VX], c->L.dim, c->stream);
    launch_pack(c->L, c->bc, x1, c->x1, c->L.dim, c->stream);
    run_filter_twofield(c, c->vec[VX], c->x1, false, true, 1.0, 1.0, c->vec[VQ], c->acc1);
    launch_unpack(c->L, c->bc, c->vec[VQ], y0, c->L.dim, c->stream);
    launch_unpack(c->L, c->bc, c->acc1, y1, c->L.dim, c->stream);
    HIPCK(hipGetLastError());
    return ELWH_OK;
}

elwh_status elwh_solve2(elwh_ctx* c, const double* f, const double* x0, const double* x1, double tol, int maxit,
                        double* v0, double* v1, elwh_info* info) {
    if (!c || !f || !v0 || !v1 || maxit < 0) return ELWH_ERR_ARG;
    CKST(twofield_ready(c));
    c->napply = 0;
    const size_t FE = (size_t)c->L.field_elems();
    const Pair x{c->vec[VX], c->vec[VP]}, b{c->vec[VB], c->vec[VD]}, w{c->vec[VQ], c->vec[VR]};
    double* zero = c->vec[VT];
    HIPCK(hipMemsetAsync(zero, 0, FE * sizeof(double), c->stream));
    pack_forcing(c, f, false);
    run_filter_twofield(c, zero, zero, true, false, c->omega, 1.0 / c->omega, b.a, b.b);   // b = Pi_h [0; 0]
    const bool xz = x0 == nullptr && x1 == nullptr;
    if (x0)
        launch_pack(c->L, c->bc, x0, x.a, c->L.dim, c->stream);
    else
        HIPCK(hipMemsetAsync(x.a, 0, FE * sizeof(double), c->stream));
    if (x1) {
        launch_pack(c->L, c->bc, x1, x.b, c->L.dim, c->stream);
        launch_axpby(c, 0.0, x.b, 1.0 / c->omega, x.b, c->stream);
    } else {
        HIPCK(hipMemsetAsync(x.b, 0, FE * sizeof(double), c->stream));
    }
    int it = 0;
    double rel = 1.0;
    elwh_status st = solve_gmres2(c, x, b, w, xz, tol, maxit, &it, &rel);
    if (st != ELWH_OK && st != ELWH_ERR_NOT_CONVERGED) return st;
    // the true residual with one more application
    double bb, rr;
    CKST(dot2(c, b, b, &bb));
    apply_A2(c, x, w);
    axpby2(c, 1.0, b, -1.0, w);
    CKST(dot2(c, w, w, &rr));
    launch_unpack(c->L, c->bc, x.a, v0, c->L.dim, c->stream);
    launch_axpby(c, 0.0, x.b, c->omega, x.b, c->stream);
    launch_unpack(c->L, c->bc, x.b, v1, c->L.dim, c->stream);
    HIPCK(hipStreamSynchronize(c->stream));
    if (info) {
        std::memset(info, 0, sizeof(*info));
        info->iters = it;
        info->nt = c->plan.nt;
        info->napply = c->napply;
        info->dt = c->plan.dt;
        info->c = c->plan.c;
        info->lambda_bound = c->plan.lambda_bound;
        info->relres = rel;
        info->relres_fp64 = bb > 0 ? std::sqrt(rr / bb) : 0.0;
        info->cond_est = NAN;
    }
    return st;
}

}  // extern "C"
