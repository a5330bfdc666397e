/*
 * elwh.h -- C ABI of libelwh.so: the El-WaveHoltz filter operator and its
 * Krylov solve on one AMD Instinct MI355X (gfx950).
 *
 * Method: D. Appelo, F. Garcia, A. Alvarez Loya, O. Runborg, "El-WaveHoltz:
 * A Time-Domain Iterative Solver for Time-Harmonic Elastic Waves",
 * arXiv:2205.12344.  Section numbers below refer to that paper.
 *
 * Problem (Sec. 2.1, 2.2): find the real displacement v with
 *     omega^2 rho v + div T(v) = f   in a box,
 * T(v) = lambda (div v) I + 2 mu sym(grad v), with homogeneous Dirichlet or
 * traction-free faces.  The library discretises it on a uniform Cartesian
 * grid with the second-order conservative finite-difference operator of
 * Sec. 4.1 (free faces closed from a discrete energy) and finds v as the
 * fixed point of the WaveHoltz filter (Sec. 3, eq. el_WHI_OP) applied with
 * the time-corrected explicit leapfrog of Sec. 4.3, by CG (or GMRES or
 * conjugate residual) on A_h = I - S_h in the M inner product (Sec. 4.5).
 * With the corrected scheme the result equals the direct discretisation of
 * the Helmholtz equation, (omega^2 M + L_h) v = W f.
 *
 * Conventions for every entry point
 *  - Array arguments are DEVICE pointers (e.g. torch.Tensor.data_ptr() of a
 *    CUDA tensor) to float64 data, owned by the caller; no call keeps or
 *    frees them.  Materials are copied at create; fields are read or written
 *    during the call only.
 *  - Field layout: [component][z][y][x] over the full (n+1)^dim node grid,
 *    x fastest, no padding; 2-D fields are [2][ny+1][nx+1], 3-D fields
 *    [3][nz+1][ny+1][nx+1].  Material arrays are one component.
 *  - Faces are ordered -x,+x,-y,+y,-z,+z (2-D uses the first four).
 *    Dirichlet-face nodes hold 0: inputs there are ignored, outputs there
 *    are written as 0.  Traction-free faces are supported on the +-y faces in
 *    2-D and the +-z faces in 3-D; the x faces (and y faces in 3-D) must be
 *    Dirichlet.  Impedance (absorbing) faces: any face in 2-D, two-field
 *    entry points only.
 *  - Calls are asynchronous on the context's stream unless stated otherwise.
 *    One context must not be used from two threads at once.
 *  - Errors are returned as elwh_status; nothing aborts or throws across the
 *    ABI.  elwh_last_error() returns a message for the last failure.
 */
#ifndef ELWH_H
#define ELWH_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct elwh_ctx elwh_ctx;

typedef enum {
    ELWH_OK = 0,
    ELWH_ERR_ARG = 1,            /* invalid argument (shape, NaN/Inf, non-positive material, ...) */
    ELWH_ERR_ALLOC = 2,          /* device or host allocation failed */
    ELWH_ERR_HIP = 3,            /* a HIP runtime call failed */
    ELWH_ERR_UNSTABLE = 4,       /* energy growth: the time step violates stability */
    ELWH_ERR_NOT_CONVERGED = 5,  /* Krylov tolerance not met within maxit */
    ELWH_ERR_BREAKDOWN = 6       /* (p, A p)_M <= 0: A_h indefinite near resonance (Sec. 4.4 Remark) */
} elwh_status;

/* ELWH_BC_IMPEDANCE: an absorbing face T(u) n = -Z u_t (Z = rho c_p on the
 * normal, rho c_s on the tangential component); on any face of 2-D
 * Cartesian grids with FP64 stepping, and only through the two-field entry
 * points elwh_apply_filter2 / elwh_apply_A2 / elwh_solve2 (the one-field
 * ones return ELWH_ERR_ARG on such a context). */
enum { ELWH_BC_DIRICHLET = 0, ELWH_BC_TRACTION_FREE = 1, ELWH_BC_IMPEDANCE = 2 };
enum { ELWH_FP64 = 0, ELWH_FP32_STEP = 1 };
enum { ELWH_KRYLOV_CG = 0, ELWH_KRYLOV_GMRES = 1, ELWH_KRYLOV_CR = 2, ELWH_KRYLOV_MINRES = 3 };
/* ELWH_SCHEME_MODIFIED: the standard (uncorrected) leapfrog with the modified
 * trapezoid weights of the remark closing Sec. 4.4.  The stepping is forced at
 * wbar = (2 / dt) asin(omega dt / 2), whose discrete time-harmonic solution
 * solves the Helmholtz system at omega exactly, and the filter weights are
 * w_n cos(omega t_n) / cos(wbar t_n), so the fixed point carries no time
 * error either.  Needs N_T >= 4 (else ELWH_ERR_ARG); a weight grows large when
 * a time level falls close to a zero of cos(wbar t), the risk the remark
 * names.  One-field contexts only. */
enum { ELWH_SCHEME_CORRECTED = 0, ELWH_SCHEME_STANDARD = 1, ELWH_SCHEME_MODIFIED = 2 };

/* dim = 2 or 3; n[a] = cells along axis a (nodes n[a]+1, n[a] >= 2);
 * len[a] = box length, h[a] = len[a]/n[a].  Unused entries are ignored. */
typedef struct {
    int dim;
    int n[3];
    double len[3];
} elwh_grid;

typedef struct {
    double cfl;        /* time-step safety factor on 2/sqrt(G), G the Gershgorin
                          bound of rho^-1 Ltilde (default 0.8) */
    int nt;            /* steps per period; 0 = the rule N_T = max(3, ceil(T/dt*)) */
    int periods;       /* K of the K-period filter, eq. many_periods_filter (default 1) */
    int prec;          /* ELWH_FP64, or ELWH_FP32_STEP: FP32 state and stencil,
                          FP64 accumulator, FP64 Krylov vectors and inner
                          products, FP64 residual replacements */
    int krylov;        /* ELWH_KRYLOV_CG (default), _GMRES, _CR, _MINRES (the
                          remedy the remark in Sec. 4.4 recommends for an
                          indefinite A_h); with ELWH_FP32_STEP only CG (else
                          ELWH_ERR_ARG) */
    int gmres_m;       /* GMRES restart length (default 30) */
    int scheme;        /* ELWH_SCHEME_CORRECTED (default, Sec. 4.3), _STANDARD or _MODIFIED */
    int compensated;   /* FP32 path: TwoSum-compensated FP64 accumulator, the
                          compensation word held in FP32 between launches
                          (default 1) */
    double inner_tol;  /* FP32 path: reduction of the recursive residual between two
                          FP64 residual replacements (default 1e-2) */
    int max_outer;     /* FP32 path: maximum residual replacements (default 50) */
    void* stream;      /* hipStream_t the context works on; NULL = the null stream */
    int autotune;      /* 1 (default): pick the step-kernel tiling by timing at create */
    int fuse;          /* time steps per step-kernel launch: 2-D Cartesian 1 to 4,
                          3-D Cartesian 1 or 2 (larger values act as 2, and
                          the tiling may still choose single steps); the
                          batch takes two-step launches for any value >= 2;
                          default 4; mapped grids and the two-field step
                          always step singly */
    int scale_x0;      /* CG paths: 1 = replace a given x0 by alpha x0 with
                          alpha = (x0, b)_M / (x0, A_h x0)_M, the factor that
                          minimises the A_h-norm error along x0 (0 when
                          (x0, A_h x0)_M <= 0), so the start is never worse than
                          x0 = 0 in that norm; costs no extra application
                          (default 0) */
    int cr_fallback;   /* CG paths: when CG breaks down ((p, A_h p)_M <= 0: A_h
                          slightly indefinite near resonance, the remark of
                          Sec. 4.4), solve again in FP64 from the iterate the
                          broken CG sequence started from (x0 or 0; in the FP32
                          path after a stagnation, where its FP64 CG began; the
                          last CG iterate is not used: near a breakdown CG
                          steps far along nearly A_h-null directions) with
                          1 (default) = the conjugate residual method, which
                          minimises the same residual norm as MINRES but can
                          itself break down when (r, A_h r)_M = 0 (reported as
                          ELWH_ERR_BREAKDOWN), or 2 = MINRES, the method the
                          remark recommends, which does not break down on a
                          nonsingular A_h; 0 = return ELWH_ERR_BREAKDOWN */
    int fp64_fallback; /* FP32 path: 1 (default) = when the FP64-recomputed
                          residual has not halved over the last two segments
                          (FP32 applications no longer improve x), finish with
                          FP64 CG from the current iterate (info.fp64_iters);
                          0 = stay with FP32 applications until maxit */
    double fp32_switch;/* FP32 path: the relative residual below which FP32
                          stepping takes over.  0 (default) = FP32 applications
                          from the start; s > 0 = FP64 CG until ||r||_M <=
                          s ||b||_M, then (after a residual replacement that keeps
                          the search direction) FP32 segments.  An FP32
                          application perturbs A_h by a relative eps (about
                          1e-5 at N_T = 63); an inexact Krylov method tolerates a
                          perturbation of about tol ||b|| / ||r|| at a residual r,
                          so s = tol / eps spends the FP32 error only where it
                          costs no accuracy. */
} elwh_opts;

typedef struct {
    int iters;          /* Krylov iterations */
    int outer;          /* FP64 residual replacements: FP32 path, and FP64 CG when the
                           true residual lagged the recurrence at tol; else 0 */
    int nt;             /* steps per period N_T */
    int napply;         /* operator applications (each periods*N_T steps) */
    double dt;          /* time step T / N_T */
    double c;           /* correction factor (wt/omega)^2, 1 for the standard scheme */
    double lambda_bound;/* Gershgorin bound G used by the time-step rule */
    double relres;      /* last Krylov residual ||r||_M / ||b||_M (recurrence) */
    double relres_fp64; /* final ||b - A_h v||_M / ||b||_M recomputed with an FP64 apply */
    double cond_est;    /* Lanczos condition estimate from the CG coefficients (CG only) */
    int cr_iters;       /* CR or MINRES iterations after a CG breakdown (cr_fallback), else 0;
                           not included in iters */
    int fp64_iters;     /* FP32 path: FP64 CG iterations after a stagnation (fp64_fallback), else 0;
                           included in iters */
} elwh_info;

/* Fill *opts with the defaults listed above.  Never fails. */
void elwh_default_opts(elwh_opts* opts);

/*
 * Time-step plan, host only (no GPU use): the Gershgorin bound G of
 * rho^-1 Ltilde over all unknown rows, dt* = cfl*2/sqrt(G),
 * N_T = max(3, ceil(T/dt*)) (or opts->nt), dt = T/N_T, and the correction
 * factor c = (sin(omega dt/2)/(omega dt/2))^2 of Sec. 4.3.
 * rho, lam, mu are HOST pointers (one component, node layout).
 * Writes info->nt, dt, c, lambda_bound.  Errors: ELWH_ERR_ARG.
 */
elwh_status elwh_plan(const elwh_grid* grid, const double* rho, const double* lam,
                      const double* mu, double omega, const int bc[6],
                      const elwh_opts* opts, elwh_info* info);

/*
 * Create a context for one problem (Sec. 2.1 data: rho, lambda, mu > 0 and
 * finite; omega > 0).  rho, lam, mu are DEVICE pointers, copied.  Computes
 * the plan (elwh_plan), uploads the coefficient arrays in the library's
 * padded internal layout and allocates all workspaces.  opts may be NULL.
 * Synchronous.  Errors: ELWH_ERR_ARG, ELWH_ERR_ALLOC, ELWH_ERR_HIP; on error
 * *out is NULL.
 */
elwh_status elwh_create(const elwh_grid* grid, const double* rho, const double* lam,
                        const double* mu, double omega, const int bc[6],
                        const elwh_opts* opts, elwh_ctx** out);

/*
 * Mapped (curvilinear) 2-D grids (Sec. 4.1; the annular sectors of the
 * iterations-vs-frequency experiment, Sec. 5.5).  The domain is the image of
 * the unit square under a smooth one-to-one map (q, r) -> (x, y); x and y
 * hold the physical coordinates of the (n[0]+1) x (n[1]+1) nodes of the
 * uniform (q, r) grid, in the node layout with q along the fast axis
 * (grid->dim must be 2; grid->len is ignored: h_q = 1/n[0], h_r = 1/n[1]).
 *
 * The operator is J times the stress divergence in conservation form on the
 * square, discretised from a non-negative discrete energy: compact
 * D+(Kbar D-) terms along q and r and central D0(K D0) cross terms, with
 * the 2x2 blocks K^ab = J [lam g_a g_b^T + mu (g_a . g_b) I + mu g_b g_a^T],
 * g_q = grad q, g_r = grad r.  The metric terms come from second-order
 * differences of the node coordinates (one-sided over three nodes on the
 * edges of the square).  The mass is rho J and the forcing J f, so the
 * solution satisfies omega^2 rho v + div T(v) = f discretely on the mapped
 * grid, and every other entry point (elwh_apply_filter, elwh_apply_A,
 * elwh_dot_M with M = rho J, the solvers, K periods, FP32 stepping, the
 * stepwise CG) works unchanged on the context.  Fields keep the node
 * layout [2][n[1]+1][n[0]+1] with Cartesian components (u, v) along x and y.
 *
 * bc: the four sides of the square (-q, +q, -r, +r).  The q sides must be
 * Dirichlet; each r side is Dirichlet or traction-free, closed from the same
 * energy with trapezoid weight 1/2 on its nodes and q-edges and the
 * one-sided r difference in its cross terms (M weights rho J / 2 there).
 * Every time step is one launch (opts->fuse is ignored).  x, y, rho, lam, mu
 * are DEVICE pointers, copied.  Errors: ELWH_ERR_ARG (also for a map with
 * J <= 0 at some node, i.e. folded or left-handed, or non-finite
 * coordinates), ELWH_ERR_ALLOC, ELWH_ERR_HIP; on error *out is NULL.  The
 * batched solver does not take mapped grids.
 */
elwh_status elwh_create_mapped(const elwh_grid* grid, const double* x, const double* y,
                               const double* rho, const double* lam, const double* mu,
                               double omega, const int bc[4], const elwh_opts* opts,
                               elwh_ctx** out);

/*
 * Mapped (curvilinear) 3-D grids (Sec. 4.1 in three dimensions; the partial
 * toroidal shell of Sec. 5.11).  The domain is the image of the unit cube
 * under a smooth one-to-one map (q, r, s) -> (x, y, z); x, y, z hold the
 * physical coordinates of the (n[0]+1) x (n[1]+1) x (n[2]+1) nodes of the
 * uniform (q, r, s) grid in the node layout (q fastest; grid->dim must be 3,
 * grid->len is ignored: h_a = 1/n[a]).  With G_a = J grad a (G_q = x_r x x_s,
 * G_r = x_s x x_q, G_s = x_q x x_r from second-order differences of the node
 * coordinates, one-sided over three nodes on the faces of the cube) and the
 * 3x3 blocks K^ab = (1/J) [lam G_a G_b^T + mu (G_a . G_b) I + mu G_b G_a^T],
 * L_h is minus the gradient of the discrete energy
 *   1/2 sum_a sum_{a-edges} w_e (D+a U)^T Kbar^aa (D+a U)
 *   + sum_{a < b} sum_{unknown nodes} w_n (Dh_a U)^T K^ab (Dh_b U)
 * (Kbar the two-node mean, Dh central or one-sided into the domain on a free
 * face, w = 1/2 on a free face); mass rho J, forcing J f, so the solution
 * satisfies omega^2 rho v + div T(v) = f discretely.  bc: the six faces
 * (-q, +q, -r, +r, -s, +s); the q and r faces must be Dirichlet, each s face
 * Dirichlet or traction-free (the free radial surfaces of the shell).  The
 * filter, A_h, the solvers, K periods, FP32 stepping and elwh_dot_M (M = w
 * rho J) work unchanged; one time step per launch, one thread per node.
 * x, y, z, rho, lam, mu are DEVICE pointers, copied.  Errors: ELWH_ERR_ARG
 * (also for a folded or left-handed map: J <= 0 at some node),
 * ELWH_ERR_ALLOC, ELWH_ERR_HIP; on error *out is NULL.
 * elwh_plan_mapped3 is the host-only plan (HOST pointers): G is the
 * Gershgorin bound of (w rho J)^-1 L_h over the unknown rows.
 */
elwh_status elwh_create_mapped3(const elwh_grid* grid, const double* x, const double* y, const double* z,
                                const double* rho, const double* lam, const double* mu, double omega, const int bc[6],
                                const elwh_opts* opts, elwh_ctx** out);
elwh_status elwh_plan_mapped3(const elwh_grid* grid, const double* x, const double* y, const double* z,
                              const double* rho, const double* lam, const double* mu, double omega, const int bc[6],
                              const elwh_opts* opts, elwh_info* info);

/* elwh_plan for a mapped grid: HOST pointers, no GPU use; G is the
 * Gershgorin bound of (rho J)^-1 L_h over the interior rows.  Errors as
 * elwh_create_mapped (ELWH_ERR_ARG only). */
elwh_status elwh_plan_mapped(const elwh_grid* grid, const double* x, const double* y,
                             const double* rho, const double* lam, const double* mu,
                             double omega, const int bc[4], const elwh_opts* opts,
                             elwh_info* info);

/*
 * Accuracy of the discrete filter (App. B), host only, no GPU use.  For N_T
 * steps per period and K = periods, the trapezoid filter multiplies a mode
 * cos(n theta) of the time stepping by beta_h(theta) = sum_n w_n cos(n theta)
 * (w_n the weights of elwh_apply_filter); A_h = I - S_h has the eigenvalue
 * 1 - beta_h, which is negative where beta_h > 1.  With the rescaled
 * frequency r = theta / (omega dt) (r = 1 at resonance, where beta_h = 1):
 *   r_star     the leftmost r < 1 with beta_h(r) = 1 (bisection); beta_h >= 1
 *              on [r_star, 1]; r_star = 1 when double precision resolves no
 *              such band
 *   gap        1 - r_star (App. B bounds it by 0.022 dt^2 in the time unit
 *              T = 2 pi, i.e. dt = 2 pi / N_T, for one period)
 *   beta_max, r_max   the largest beta_h on [r_star, 1] and where it occurs
 *   lambda_lo, lambda_hi   the band of spatial frequencies lambda (modes
 *              with -L_h phi = lambda^2 M phi) that land in [r_star, 1]:
 *              sin(theta/2) = sin(omega dt/2) lambda / omega for the
 *              corrected scheme (lambda_hi = omega), sin(theta/2) =
 *              lambda dt / 2 for the standard one (scheme: ELWH_SCHEME_*).
 * An eigenvalue lambda_j of the medium inside [lambda_lo, lambda_hi] makes
 * A_h indefinite: CG may break down there and the conjugate residual method
 * (opts.krylov, or the cr_fallback of elwh_solve) is the remedy of the
 * remark in Sec. 4.4.  Errors: ELWH_ERR_ARG (nt < 3, periods outside
 * [1, 1000], omega <= 0, unknown scheme).
 */
typedef struct {
    double r_star, gap, beta_max, r_max, lambda_lo, lambda_hi;
} elwh_filter_diag;

elwh_status elwh_filter_diagnostics(int nt, int periods, double omega, int scheme,
                                    elwh_filter_diag* out);

/*
 * Two-field operator for impedance faces (the remark after eq.
 * many_periods_filter in Sec. 3; the paper leaves such boundaries to future
 * work).  With an absorbing face the initial velocity of the time-harmonic
 * solution is not zero and the filter acts on the pair
 *     Pi_h [u0; u1] = [sum_n w_n u^n; sum_n w_n v^n],
 * u^n the corrected leapfrog (Sec. 4.3) started from displacement u0 and
 * velocity u1, v^n = (u^{n+1} - u^{n-1}) / (2 dt) its centred velocity
 * (v^0 = u1; one step past the window gives v^{K N_T}), w_n the trapezoid
 * weights of elwh_apply_filter.  An impedance face is a traction-type face of
 * the discrete energy (Sec. 4.1) whose rows carry the damping B = 2 c / h
 * (c = c_p for the normal, c_s for the tangential component, h the spacing
 * normal to the face; the two faces' terms add at a corner), stepped as
 *     (1 + g) u^{n+1} = 2 u^n - (1 - g) u^{n-1} + a (Ltilde u^n - f cos(omega t_n)),
 * g = c dt Bt / 2 with Bt = B omega dt / sin(omega dt) for the corrected
 * scheme (Bt = B for the standard one), so that the fixed point reproduces
 * the time-harmonic solution without time error: with the corrected scheme
 *     u0 = Re v,   u1 = -(sin(omega dt) / dt) Im v,
 * v the complex solution of (omega^2 M + L_h - i omega D) v = W f, D = M B
 * (the direct discretisation of omega^2 rho v + div T(v) = f with the
 * impedance condition T(v) n + i omega Z v = 0).  Without impedance faces
 * these entry points apply the same operator (the fixed point has u1 = 0).
 * FP64, 2-D Cartesian contexts only.  All arrays are DEVICE fields in the
 * layout above.
 *
 * elwh_apply_filter2  out0, out1 = Pi_h [u0; u1] with forcing f (NULL: S_h).
 * elwh_apply_A2       [y0; y1] = [x0; x1] - S_h [x0; x1].  In both calls the
 *                     inputs are copied before any output is written, so
 *                     inputs and outputs may alias.
 * elwh_solve2         the fixed point by restarted GMRES (opts.gmres_m, CGS2)
 *                     on A_h z = Pi_h [0; 0] for the stacked z = [u0; u1 /
 *                     omega] in the M inner product of each half, from
 *                     [x0; x1] (NULL: zero), until the recurrence residual is
 *                     <= tol times ||b|| or maxit applications; writes the
 *                     displacement v0 and the velocity v1, info->iters,
 *                     relres and relres_fp64 (the true residual recomputed
 *                     with one more application).  Synchronises the stream.
 * Errors: ELWH_ERR_ARG (NULL pointer, mapped, 3-D or FP32 context),
 * ELWH_ERR_NOT_CONVERGED (v0, v1 hold the last iterate), ELWH_ERR_UNSTABLE,
 * ELWH_ERR_ALLOC, ELWH_ERR_HIP.
 */
elwh_status elwh_apply_filter2(elwh_ctx* ctx, const double* u0, const double* u1, const double* f, double* out0,
                               double* out1);
elwh_status elwh_apply_A2(elwh_ctx* ctx, const double* x0, const double* x1, double* y0, double* y1);
elwh_status elwh_solve2(elwh_ctx* ctx, const double* f, const double* x0, const double* x1, double tol, int maxit,
                        double* v0, double* v1, elwh_info* info);

/* Release every device and host resource of ctx (NULL is a no-op). */
void elwh_destroy(elwh_ctx* ctx);

/* Plan and sizes of a context (nt, dt, c, lambda_bound; other fields 0). */
elwh_status elwh_query(const elwh_ctx* ctx, elwh_info* info);

/* Text of the last error on ctx (or of the last failed create when ctx is
 * NULL); valid until the next call on that context. */
const char* elwh_last_error(const elwh_ctx* ctx);

/*
 * out = Pi_h u0  (Sec. 3 eq. el_WHI_OP, trapezoid rule): u0 is the initial
 * displacement (zero initial velocity), f the forcing amplitude of
 * -f cos(omega t) (eq. elastic-time), NULL for f = 0 (then out = S_h u0).
 * The time stepping is the corrected leapfrog of Sec. 4.3 started with
 * u^{-1} = u^1 (the even-in-time start); the accumulation
 * sum_n w_n u^n is fused into each step.  In the FP32 path the stepping is
 * FP32 and the accumulation FP64.  u0 and out may alias.
 */
elwh_status elwh_apply_filter(elwh_ctx* ctx, const double* u0, const double* f, double* out);

/* y = A_h x = x - S_h x  (Sec. 4.5 eq. amat_non_sym).  x and y may alias. */
elwh_status elwh_apply_A(elwh_ctx* ctx, const double* x, double* y);

/*
 * Solve A_h v = b, b = Pi_h 0 with forcing f (Sec. 4.5), by the Krylov
 * method in opts (CG in the M inner product by default), from x0 (NULL =
 * zero guess) until the true residual ||b - A_h v||_M, recomputed with an
 * FP64 application (info->relres_fp64), is <= tol ||b||_M, or maxit
 * iterations.  Every method iterates until its own recurrence residual
 * (info->relres) meets tol and then checks the true one; when that is still
 * above tol the residual is replaced by the true one and the iteration goes
 * on (CG keeps its search direction; CR and MINRES restart from the
 * iterate; GMRES restarts anyway).  tol <= 0 runs exactly maxit iterations
 * and returns ELWH_OK.  When ||b||_M = 0 the solution is v = 0: it is
 * returned with ELWH_OK and no iteration, whatever x0.  FP32 path: CG with
 * FP32-stepped applications and FP64 vectors; whenever the recursive
 * residual has fallen by inner_tol, it is replaced by b - A_h x from an FP64
 * application and CG continues along the same search direction (a reliable
 * update); the solve stops on the FP64 residual.  Returns when done
 * (synchronises the stream).
 * Errors: ELWH_ERR_NOT_CONVERGED (v holds the last iterate),
 * ELWH_ERR_BREAKDOWN, ELWH_ERR_ARG, ELWH_ERR_HIP.
 */
elwh_status elwh_solve(elwh_ctx* ctx, const double* f, const double* x0, double tol,
                       int maxit, double* v, elwh_info* info);

/*
 * Stepwise CG in the M inner product (the loop of elwh_solve, exposed for
 * timing and for resume-by-restart):
 *   elwh_cg_begin    b = Pi_h 0 with f; r = b - A_h x0; p = r (when
 *                    ||b||_M = 0: x = 0, and elwh_cg_iterate returns at once)
 *   elwh_cg_iterate  k iterations (one A_h apply each, FP64 reductions,
 *                    fused vector updates); writes the current ||r||_M/||b||_M;
 *                    stops early (returns ELWH_OK) once it is <= tol
 *   elwh_cg_result   v = x; recomputes the FP64 residual into info
 * FP64 path only.  elwh_cg_iterate synchronises the stream.
 */
elwh_status elwh_cg_begin(elwh_ctx* ctx, const double* f, const double* x0);
elwh_status elwh_cg_iterate(elwh_ctx* ctx, int k, double tol, double* relres);
elwh_status elwh_cg_result(elwh_ctx* ctx, double* v, elwh_info* info);

/*
 * (x, y)_M = sum over unknown dofs of w_i rho_i x_i y_i, the inner product
 * of Sec. 4.5 (w = trapezoid weight, 1/2 per free face).  Deterministic
 * FP64 two-pass reduction.  Writes the HOST double *out; synchronises.
 */
elwh_status elwh_dot_M(elwh_ctx* ctx, const double* x, const double* y, double* out);

/*
 * elwh_dot_M_noalloc: the same M inner product as elwh_dot_M, for callers
 * that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): it needs no context and
 * makes no hipMalloc, hipFree or other allocating call.
 *   grid    dim 2 or 3, n[a] >= 2 cells per axis, at most 2^31 nodes per
 *           component (ELWH_ERR_ARG beyond); len is not used
 *   rho     DEVICE array, node layout (one component); the weight of node i
 *           is rho_i times 1/2 per traction-type face (free or impedance) it
 *           lies on, 0 on Dirichlet faces -- the M of elwh_create.  On a
 *           mapped grid pass rho J to get the M of elwh_create_mapped.
 *   bc      the faces, as in elwh_create (the first 2*dim entries are read)
 *   x, y    DEVICE fields in the caller layout [dim][nodes]
 *   stream  hipStream_t to run on (NULL: the null stream)
 *   out     HOST double; the call synchronises the stream
 * The two reduction passes keep their 512 partial sums and the result in a
 * fixed 4.5 KiB device array of the library (one per GPU, held until the
 * process ends), so the result is deterministic and does not depend on the
 * grid size; every call on one GPU shares that array, so calls that overlap
 * on one GPU (other streams or host threads) race.  Errors: ELWH_ERR_ARG,
 * ELWH_ERR_HIP; the message is elwh_last_error(NULL).
 */
elwh_status elwh_dot_M_noalloc(const elwh_grid* grid, const double* rho, const int bc[6], const double* x,
                               const double* y, void* stream, double* out);

/*
 * Measurement aid (not part of the method): the STREAM triad a = b + s c
 * over n doubles (n a multiple of 4, arrays 32-byte aligned, DEVICE
 * pointers), one 32-byte vector per thread, asynchronous on stream.  Timed
 * over arrays far larger than the 256 MiB Infinity Cache it gives the HBM
 * bandwidth a plain streaming kernel reaches (24 bytes per element).
 * Errors: ELWH_ERR_ARG, ELWH_ERR_HIP.
 */
elwh_status elwh_stream_triad(double* a, const double* b, const double* c, double s, long long n, void* stream);

/*
 * Kernel timing for measurement.  While enabled, every fused-step launch of
 * the filter (Sec. 4.3 step + trapezoid accumulation; the half-step launch
 * is counted separately) is bracketed by a pair of HIP events on the
 * context's stream.  elwh_profile_read synchronises the stream and returns
 * the summed kernel time in milliseconds and the launch counts since the
 * last read or enable, then resets them.  Enabling also resets.
 * Errors: ELWH_ERR_ARG (NULL ctx), ELWH_ERR_HIP.
 */
elwh_status elwh_profile_enable(elwh_ctx* ctx, int on);
elwh_status elwh_profile_read(elwh_ctx* ctx, double* step_ms, int* nstep, double* init_ms, int* ninit);

/*
 * Tiling of the fused step kernel for precision prec (ELWH_FP64 or
 * ELWH_FP32_STEP): 2-D: vec nodes per lane along x (1 or 2, FP32 also 4)
 * and rows (4, 8, 16; with vec = 1 also 10, 12) marched per wavefront;
 * 3-D: vec = y rows per workgroup, one wavefront each, and rows = z planes
 * marched per wavefront:
 * (1, 2, 4, 8) x (4, 8, 16, 32) for single-step launches (opts.fuse = 1),
 * (2, 4, 6) x (8, 16, 32, 64) for two-step launches (fuse >= 2; the workgroup
 * adds two halo rows), where vec = 1 with rows 4 to 32 makes every step a
 * single-step launch (the FP64 choice on large cubes).  The tiling changes
 * speed only, never results.
 * elwh_autotune times every supported tiling on reps operator applications
 * (HIP events), in three round-robin passes, and keeps the tiling with the
 * fastest pass (contexts with impedance faces time the two-field step);
 * results are cached per process by
 * (dim, precision, accumulator, grid size) and, when the environment
 * variable ELWH_TUNE_CACHE names a file, in that file as JSON lines keyed by
 * (arch, dim, precision, accumulator, grid size).  Synchronous.
 * Errors: ELWH_ERR_ARG (unsupported tiling), ELWH_ERR_HIP.
 */
elwh_status elwh_set_tile(elwh_ctx* ctx, int prec, int vec, int rows);
elwh_status elwh_get_tile(const elwh_ctx* ctx, int prec, int* vec, int* rows);
elwh_status elwh_autotune(elwh_ctx* ctx, int prec, int reps, double* best_step_us);

/*
 * Ragged batch of independent 2-D problems (sizes, media, omega and N_T may
 * all differ), solved together: each batched step ("tick") advances every
 * unfinished problem by opts->fuse >= 4 ? 4 : 2 steps of its own filter
 * application where that many are left (one step where not, and always
 * for opts->fuse = 1), in one multi-step and one single-step launch over
 * all problems; a problem whose application ends runs its CG update on the
 * device in the same tick and starts its next application at the next one;
 * converged problems drop out.  The CG phase is captured as a hipGraph of several steps and
 * replayed (elwh_batch_set_graph(b, 0) runs the same launches eagerly).
 * Each problem's solve is the one of elwh_solve (Sec. 4.5): CG on A_h in the
 * M inner product with b = Pi_h 0; FP64, or (opts->prec = ELWH_FP32_STEP)
 * FP32-stepped CG with FP64 residual replacements.
 *
 * elwh_batch_create: nprob problems; grids[i], rho[i], lam[i], mu[i]
 *   (DEVICE pointers, copied), omega[i], bc[6*i .. 6*i+5]; opts shared
 *   (opts->stream is the caller's stream; the batch works on its own stream
 *   and orders itself after / before the caller's stream).  Picks the batch
 *   tiling by timing when opts->autotune.  Errors: ELWH_ERR_ARG (also for a
 *   3-D problem), ELWH_ERR_ALLOC, ELWH_ERR_HIP.
 * elwh_batch_solve (with ELWH_PROGRESS=1 in the environment it prints a progress
 *   line to stderr at most every 10 s): f[i], x0[i] (x0 or any x0[i] may be NULL: zero guess),
 *   v[i] outputs (DEVICE pointers, caller layout); tol, maxit per problem as
 *   in elwh_solve; infos (nullable) receives nprob records.  Synchronous.
 *   Returns ELWH_OK when every problem converged, else the first failure.
 * elwh_batch_stats: wall seconds of the last solve, number of batched steps
 *   (ticks), and the FP64 / FP32 tilings {vec, rows}.
 */
typedef struct elwh_batch elwh_batch;
elwh_status elwh_batch_create(int nprob, const elwh_grid* grids, const double* const* rho,
                              const double* const* lam, const double* const* mu, const double* omega,
                              const int* bc, const elwh_opts* opts, elwh_batch** out);
elwh_status elwh_batch_solve(elwh_batch* b, const double* const* f, const double* const* x0, double tol,
                             int maxit, double* const* v, elwh_info* infos);
elwh_status elwh_batch_set_graph(elwh_batch* b, int on);
elwh_status elwh_batch_info(const elwh_batch* b, int i, elwh_info* info);
elwh_status elwh_batch_stats(const elwh_batch* b, double* seconds, long long* ticks, int* tile64,
                             int* tile32);
const char* elwh_batch_last_error(const elwh_batch* b);
void elwh_batch_destroy(elwh_batch* b);

/*
 * Learned warm start (not part of the paper: an initial guess x0 for the
 * solve).  A convolutional encoder-decoder over an H x W pixel grid
 * (H, W multiples of 16): five resolution levels of two 3x3 convolutions
 * with bias and SiLU (widths 32, 64, 96, 128, 128), 2x2 average pooling,
 * nearest upsampling with skip concatenation, and a 3x3 output convolution
 * to 2 channels; 1 644 578 parameters.  Convolutions are GEMMs on MFMA over
 * a BF16 im2col matrix (FP32 accumulation); master weights, activations,
 * gradients and the Adam state are FP32.  Tensors are NHWC float32 device
 * arrays: inputs x [B][H][W][7], outputs y [B][H][W][2], loss weights
 * w [B][H][W].  The flat parameter vector holds, per layer in order,
 * W[(ky*3+kx)*cin + ci][cout] then bias[cout].
 *
 * Mapping to a problem of n x n cells with H = W = n (Dirichlet sides and
 * bottom, free top): pixel (py, px) is node (i = px, j = py + 1).
 *   elwh_ws_features  x = (log rho / 0.2, log mu / 0.2, log(lambda/mu) / 0.5,
 *                     f_x / max|f|, f_y / max|f|, 5 omega / n, omega / 60),
 *                     w = M weight of the node (0 on Dirichlet nodes)
 *   elwh_ws_from_field targets y = v omega^2 / (max|f| k), k the output scale
 *   elwh_ws_normalize  y[b] /= its w-weighted RMS over both components (the
 *                     solver rescales the guess optimally, so the network
 *                     learns shapes; asynchronous)
 *   elwh_ws_predict   forward pass, then x0 = y max|f| k / omega^2 on the
 *                     unknown nodes (0 elsewhere), written to x0[b] (caller
 *                     layout [2][n+1][n+1])
 * Field arguments are host arrays of DEVICE pointers (one per sample);
 * omega_dev is a device array of B doubles.
 *   elwh_ws_loss_grad  L = (1/B) sum_b ||y_hat - y||_w^2 / ||y||_w^2 and its
 *                      gradient (copied to grad_host when non-null)
 *   elwh_ws_train_step one Adam step (beta 0.9, 0.999, eps 1e-8) at rate lr
 *   elwh_ws_params     read (get) / write (set) the FP32 parameters (setting
 *                      resets the Adam state) and the output scale k
 * Calls run on the given stream; forward/train/loss_grad/params synchronise
 * when they return host data.  Errors: ELWH_ERR_ARG, ELWH_ERR_ALLOC,
 * ELWH_ERR_HIP.
 */
typedef struct elwh_ws elwh_ws;
elwh_status elwh_ws_create(int max_batch, int H, int W, unsigned long long seed, void* stream, elwh_ws** out);
void elwh_ws_destroy(elwh_ws* ws);
const char* elwh_ws_last_error(const elwh_ws* ws);
long long elwh_ws_num_params(const elwh_ws* ws);
elwh_status elwh_ws_params(elwh_ws* ws, float* get, const float* set, double* out_scale_get,
                           const double* out_scale_set);
elwh_status elwh_ws_forward(elwh_ws* ws, int B, const float* x, float* y);
elwh_status elwh_ws_loss_grad(elwh_ws* ws, int B, const float* x, const float* y, const float* w, float* loss,
                              float* grad_host);
elwh_status elwh_ws_train_step(elwh_ws* ws, int B, const float* x, const float* y, const float* w, float lr,
                               float* loss);
elwh_status elwh_ws_features(elwh_ws* ws, int B, int n, const double* const* rho, const double* const* lam,
                             const double* const* mu, const double* const* f, const double* omega_dev, float* x,
                             float* w);
elwh_status elwh_ws_from_field(elwh_ws* ws, int B, int n, const double* const* f, const double* const* v,
                               const double* omega_dev, float* y);
elwh_status elwh_ws_normalize(elwh_ws* ws, int B, float* y, const float* w);
elwh_status elwh_ws_predict(elwh_ws* ws, int B, int n, const float* x, const double* const* f,
                            const double* omega_dev, double* const* x0);

#ifdef __cplusplus
}
#endif
#endif /* ELWH_H */
