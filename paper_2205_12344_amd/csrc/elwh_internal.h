// Internal declarations of libelwh: context, padded device layout, kernel
// launchers.  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/elwh.h"

namespace elwh {

// ---------------------------------------------------------------------------
// Padded internal layout.  One component of a field is stored as
// (nz+1) planes x (ny+1) rows x P elements, P = nx+4 rounded up to 64 so
// every row starts 512-byte (FP64) / 256-byte (FP32) aligned and a 4-wide
// vector starting at any node stays in its row.  2-D fields have one plane.
// Padding and Dirichlet nodes always hold zero.
// ---------------------------------------------------------------------------
struct Layout {
    int dim = 2;
    int nx = 0, ny = 0, nz = 0;      // cells
    int64_t P = 0;                   // row pitch (elements)
    int64_t PS = 0;                  // plane stride = (ny+1) * P
    int64_t CS = 0;                  // component stride = (nz+1) * PS
    int ncomp() const { return dim; }
    int64_t nodes_caller() const {
        return (int64_t)(nx + 1) * (ny + 1) * (dim == 3 ? (nz + 1) : 1);
    }
    int64_t field_elems() const { return CS * dim; }
};

// Stencil constants shared by the kernels (FP64; FP32 kernels convert).
struct Stencil {
    double cxx2, cyy2, czz2;   // 1/(2 h_a^2): compact terms with summed face pairs
    double cxy, cxz, cyz;      // 1/(4 h_a h_b): central mixed terms
    double cyyf, czzf;         // 1/h_y^2, 1/h_z^2: free-face normal compact term
    double cfxy, cfxz, cfyz;   // 1/(2 h_a h_b): free-face one-sided mixed terms
};

// Which rows/planes are unknowns along the marching axis (y in 2-D, z in 3-D).
struct March {
    int lo, hi;            // first and last unknown index along the axis
    int free_lo, free_hi;  // traction-free face at index 0 / at index n
};

// Device scalar slots used by the device-side CG updates.
// S_FLAG: 1 = CG breakdown ((p, A p)_M <= 0), 2 = unstable step (Rayleigh
// quotient (p, A p)_M / (p, p)_M outside a stable step's spectrum)
enum { S_RR = 0, S_PQ, S_RRNEW, S_ALPHA, S_BETA, S_BB, S_TMP, S_FLAG, S_PP, S_NSLOT = 16 };

// Tiling of the fused step kernels: V nodes per lane along x, TY rows (2-D)
// or TZ planes (3-D) marched per wavefront.
struct Tile {
    int V = 1, TY = 8;
};

// Kernel arguments of the 2-D fused step.
struct Args2D {
    int nx, ny;
    int64_t P, CS;
    int jlo, jhi, free_lo, free_hi;
    double cxx2, cyy2, cxy, cyyf, cfx;
    double w, w0, fc;
    double wk[4], fck[4];     // K-step launch: weight of u^{n+s}, forcing factor of step n+s-1 (s = 1..K)
    int final_;
};

// Two-field step on a 2-D grid with impedance y faces (kernels2d_damped.hip).
struct Damp2D {
    Args2D A;                 // geometry, stencil constants, w (of u^{n+1}), w0 (of u^0), fc
    double wv;                // weight of the centred velocity of level n (step launch)
    double w0v;               // weight of the second field (start launch)
    double dtw;               // dt times the scale of the second field (start launch)
    int imp_lo, imp_hi;       // the -y / +y face is an impedance face
    int ximp_lo, ximp_hi;     // the -x / +x face is an impedance face (its column is computed)
    double hx, hy;            // grid spacings (the x-face rows)
    int nmain;                // blocks of the strip march; face-column blocks follow (set at launch)
};

// Batched problem descriptor (device copy built by the host per phase).
struct BProb2D {
    Args2D A;                 // geometry and stencil constants
    int nbx, nblk, off;       // single-step launch: blocks along x, blocks, first block
    int nbx2, nblk2, off2;    // multi-step launch (K = 2 or 4): the same for its tiling
    int nsteps;               // steps per application (K N_T)
    const double* w;          // filter weights w_n (sign +1), n = 0..nsteps
    const double* cosn;       // forcing factors cos(2 pi n / N_T)
    void* s[4];               // state buffers (FP64 or FP32)
    const double* src;        // u^0 of the application
    double* out;              // accumulator = result of the application (q in CG)
    float* lo;               // compensation
    const void *ca, *cl, *cm, *f;
    const double* m;          // M weights
    double *cx, *cr, *cp;     // CG iterate, residual, direction
    double* vec[8];           // the problem's FP64 work vectors
};

// Per-problem device state of the ragged CG.
struct BState {
    int n, end, active, status, iters, maxit;
    int ic, ip;               // state buffers holding u^n and u^{n-1} (ip = -1: u^{n-1} = src)
    double rr, pq, alpha, beta, bb, tol2;
};

// For a stable step every eigenvalue of A_h = I - S_h lies in [-3/2, 7/2]
// (|beta_h(theta)| <= sum |w_n| <= 5/2), so a Rayleigh quotient
// (p, A_h p)_M / (p, p)_M outside [kStableRayleighLo, kStableRayleighHi]
// reveals an unstable time step; CG tests it at every iteration.
constexpr double kStableRayleighLo = -2.0, kStableRayleighHi = 4.0;

struct Plan {
    int nt = 0;
    double dt = 0, c = 1, lambda_bound = 0, T = 0;
};

}  // namespace elwh

struct elwh_ctx {
    elwh::Layout L;
    elwh::Stencil st;
    elwh::March mr;
    elwh::Plan plan;
    elwh_grid grid;
    int bc[6];
    double omega;
    elwh_opts opts;
    hipStream_t stream = nullptr;
    std::string err;

    // filter weights (sign +1) and forcing factors cos(2 pi n / N_T), n = 0..K N_T
    std::vector<double> w, cosn;

    // FP64 coefficient arrays (one component each): a = c dt^2 / rho, lambda, mu
    double *ca = nullptr, *cl = nullptr, *cm = nullptr;
    double* mw = nullptr;          // M weights w_node * rho (0 at Dirichlet / padding)
    // FP32 copies (FP32 path)
    float *fa = nullptr, *fl = nullptr, *fm = nullptr;
    // mapped 2-D grids: ca = c dt^2 / (rho J), cl = lambda / J, cm = mu / J,
    // metric arrays cg = (J grad q, J grad r) (FP32 copies fg), and J itself
    // (the forcing enters as J f)
    bool mapped = false;
    // (3-D mapped grids: nine metric arrays, G_q, G_r, G_s by component)
    double* cg[9] = {};
    float* fg[9] = {};
    double* jac = nullptr;

    // FP64 state buffers (2 time levels), accumulator and its compensation
    // (four for 2-D: the step-pair kernel writes two new levels beside the two it reads)
    double *s64[4] = {nullptr, nullptr, nullptr, nullptr};
    float *s32[4] = {nullptr, nullptr, nullptr, nullptr};
    double* acc = nullptr;
    float* acc_lo = nullptr;       // FP32 compensation word of the accumulator
    // forcing (internal layout) in FP64 and FP32
    double* f64 = nullptr;
    float* f32 = nullptr;
    // general FP64 work vectors (internal layout): x, r, p, q, b, tmp, tmp2
    double* vec[8] = {};
    // GMRES basis (allocated on demand)
    std::vector<double*> basis;
    // reduction partials and device scalars
    double* partials = nullptr;
    double* dscal = nullptr;
    double* hscal = nullptr;       // pinned host mirror
    int red_blocks = 1024;

    // tiling of the fused step kernels (set by elwh_set_tile / elwh_autotune)
    elwh::Tile tile64, tile32;

    // kernel profiling: three events per filter application (start, after the
    // half step, after the last step) on the context's stream
    bool prof_on = false;
    std::vector<hipEvent_t> prof_ev;   // pool, reused
    std::vector<int> prof_nsteps;      // step launches per recorded application
    size_t prof_used = 0;              // applications recorded since the last read

    // impedance y faces (two-field path): flags, damping rows g (4 x P: u and v
    // of the -y face, then of the +y face), the velocity accumulator and the
    // second field of the input, GMRES basis of the two-field solve
    int imp[2] = {0, 0};
    int ximp[2] = {0, 0};              // impedance -x / +x faces
    double* dmp = nullptr;
    double* dmpx = nullptr;
    double* acc1 = nullptr;
    double* x1 = nullptr;
    std::vector<double*> basis2;
    double** gm_ptrs = nullptr;        // device copy of the basis2 pointers, then the pair w
    double* gm_part = nullptr;         // multidot partials
    double* gm_h = nullptr;            // device Gram-Schmidt coefficients and ||w||^2
    int gm_cap = 0;                    // pairs the three buffers above hold

    // CG state of the stepwise interface
    bool cg_active = false;
    bool cg_qready = false;            // q = A_h p already computed for the next CG iteration
    hipEvent_t ev_scal = nullptr;      // marks the device-to-host copy of the CG scalars
    int cg_iters = 0;
    double cg_bb = 0;
    bool cg_zero = false;              // ||b||_M = 0: the solution is x = 0
    std::vector<double> alphas, betas;
    int napply = 0;
};

namespace elwh {

// ---- host plan (plan.cpp) --------------------------------------------------
// Metric terms of a mapped 2-D grid (Sec. 4.1) in the caller's node layout:
// J = x_q y_r - x_r y_q and g = (J grad q, J grad r) = (y_r, -x_r, -y_q, x_q),
// from second-order differences of the node coordinates.
// 3-D: J = x_q . (x_r x x_s) and G_q = x_r x x_s, G_r = x_s x x_q,
// G_s = x_q x x_r (g[3a + i] = component i of G_a).
struct MappedMetric {
    std::vector<double> J, g[9];
};
elwh_status mapped_metric(int nq, int nr, const double* x, const double* y, MappedMetric* m, std::string* err);
elwh_status mapped_metric3(int nq, int nr, int ns, const double* x, const double* y, const double* z,
                           MappedMetric* m, std::string* err);
elwh_status make_plan_mapped3(const elwh_grid* g, const double* x, const double* y, const double* z,
                              const double* rho, const double* lam, const double* mu, double omega, const int bc[6],
                              const elwh_opts* o, Plan* out, MappedMetric* met, std::string* err);
elwh_status make_plan_mapped(const elwh_grid* g, const double* x, const double* y, const double* rho,
                             const double* lam, const double* mu, double omega, const int bc[6], const elwh_opts* o,
                             Plan* out, MappedMetric* met, std::string* err);
elwh_status filter_diagnostics(int nt, int periods, double omega, int scheme, elwh_filter_diag* out,
                               std::string* err);
elwh_status make_plan(const elwh_grid* g, const double* rho, const double* lam, const double* mu,
                      double omega, const int bc[6], const elwh_opts* o, Plan* out, std::string* err,
                      bool x_free_ok = false);
// x_free_ok: traction-type x faces are allowed (2-D impedance x faces of the
// two-field path); otherwise only the marching axis takes them.
elwh_status check_config(const elwh_grid* g, const int bc[6], const elwh_opts* o, std::string* err,
                         bool x_free_ok = false);
Layout make_layout(const elwh_grid* g);
Stencil make_stencil(const elwh_grid* g);
March make_march(const elwh_grid* g, const int bc[6]);

// ---- profiling hooks (api.hip) ---------------------------------------------
// phase 0: before the half step; 1: after it; 2: after the last step
// (nsteps = number of step launches of this application).
void prof_mark(elwh_ctx* c, int phase, int nsteps = 0);
bool tile_valid_2d(bool fp32, int V, int TY);
// Conjugate residual (method 1) or MINRES (method 2), FP64 applications, from
// the iterate in vec[0] with the right-hand side in vec[4], on the context's
// stream, restarted while the true residual misses tol (api.hip).
elwh_status ctx_solve_fallback(elwh_ctx* c, int method, double tol, int maxit, int* iters, double* relres);
// The message elwh_last_error(NULL) returns (calls without a context).
void set_create_error(const std::string& msg);
bool tile_valid_3d(bool fp32, int V, int TZ);
// Two-step 3-D launches (kernels3d_k2.hip): RB y rows per workgroup plus two
// halo rows, TZ planes; reads u^n (u), u^{n-1} (uprev), writes u^{n+1} (outA)
// and u^{n+2} (outB), four distinct buffers.
bool tile_valid_3d_k2(bool fp32, int RB, int TZ);
struct Args3D;
template <typename T>
void launch_step3d_k2(int RB, int TZ, bool force, bool comp, hipStream_t s, const T* u, const T* uprev, T* outA,
                      T* outB, double* acc, float* acclo, const T* ca, const T* cl, const T* cm, const T* f,
                      const Args3D& A);
bool tile_valid_curv(bool fp32, int V, int TY);
bool tile_valid_curv3(bool fp32, int V, int TY);
// One filter application on a mapped 2-D grid (kernels2d_curv.hip).
void run_filter_curv2d(elwh_ctx* c, const double* x, bool with_force, bool amode, bool fp32, double* out);
// One filter application on a mapped 3-D grid (kernels3d_curv.hip).
void run_filter_curv3d(elwh_ctx* c, const double* x, bool with_force, bool amode, bool fp32, double* out);
// Two-field step of the impedance path (kernels2d_damped.hip).  mode 1 (start):
// u = u^0, uprev = the second field, base0/base1 the A_h bases or null;
// mode 0: u = u^n, uprev = u^{n-1} (unext may alias it), acc0/acc1 updated.
// dmp: four rows of P values, the damping g of (u, v) on the -y, then +y face;
// dmpx: four columns of ny + 1 values, the same on the -x, then +x face.
bool tile_valid_damped(int V, int TY);
void launch_damped2d(int V, int TY, int mode, bool force, hipStream_t s, const double* u, const double* uprev,
                     double* unext, const double* base0, const double* base1, double* acc0, double* acc1,
                     const double* dmp, const double* dmpx, const double* ca, const double* cl, const double* cm,
                     const double* f, const Damp2D& D);
Args2D make_args2d(const elwh_ctx* c);
// dst[comp][node] *= w[node] over the padded layout (blas.hip).
void launch_scale_field(const Layout& L, double* dst, const double* w, int ncomp, hipStream_t s);

// K = 2..4 time steps per launch (kernels2d_multi.hip): reads u^n (u) and
// u^{n-1} (uprev), writes u^{n+K-1} (outA) and u^{n+K} (outB), four distinct
// buffers; A.wk[s-1] weighs u^{n+s}, A.fck[s-1] is the forcing factor of
// step n+s-1.
template <typename T>
void launch_multi2d(int K, int V, int TY, bool force, bool comp, hipStream_t s, int nrows, const T* u,
                    const T* uprev, T* outA, T* outB, double* acc, float* acclo, const T* ca, const T* cl,
                    const T* cm, const T* f, const Args2D& A);

// ---- kernels (kernels2d.hip / kernels3d.hip / blas.hip) --------------------
// Copy a caller-layout field (ncomp components) into the padded layout,
// zeroing Dirichlet nodes (mask from bc); T = float or double destination.
void launch_pack(const Layout& L, const int bc[6], const double* src, double* dst, int ncomp,
                 hipStream_t s);
void launch_pack_f32(const Layout& L, const int bc[6], const double* src, float* dst, int ncomp,
                     hipStream_t s);
void launch_unpack(const Layout& L, const int bc[6], const double* src, double* dst, int ncomp,
                   hipStream_t s);
void launch_convert_f32(const Layout& L, const double* src, float* dst, int ncomp, hipStream_t s);

// One filter application in the padded layout.
//   x     : u^0 (FP64, padded), read only
//   f     : forcing (FP64 / FP32 per path) or null
//   out   : sum_n s w_n u^n, plus x when amode (then s = -1): A_h x
// Uses the context's state buffers and accumulator.
void run_filter(elwh_ctx* c, const double* x, bool with_force, bool amode, bool fp32, double* out);

// FP64 vector kernels over the padded layout (length = field_elems()).
void launch_dot_M_partial(const elwh_ctx* c, const double* x, const double* y, hipStream_t s);
// Partials of (p, q)_M and (p, p)_M in one pass (for RED_PQ).
void launch_dot_pq_pp_partial(const elwh_ctx* c, const double* p, const double* q, hipStream_t s);
void launch_reduce_final(const elwh_ctx* c, int mode, int slot, hipStream_t s);
void launch_cg_update_xr(const elwh_ctx* c, double* x, double* r, const double* p, const double* q,
                         hipStream_t s);
void launch_cg_update_p(const elwh_ctx* c, double* p, const double* r, hipStream_t s);
void launch_axpby(const elwh_ctx* c, double a, const double* x, double b, double* y, hipStream_t s);
void launch_copy(const elwh_ctx* c, const double* x, double* y, hipStream_t s);
// GMRES orthogonalisation with device coefficients (blas.hip).  Two-field
// (wb != null): V is a device array of 2k field pointers, vector i = (V[2i],
// V[2i+1]); one-field (wb == null): k pointers, vector i = V[i].
// launch_multidot2: out[i] = (vector i, w)_M for i < k (partials:
// k * multidot2_blocks(c) doubles); launch_multiaxpy2: w -= sum_i h[i]
// vector i, h on the device.
int multidot2_blocks(const elwh_ctx* c);
void launch_multidot2(const elwh_ctx* c, const double* const* V, int k, const double* wa, const double* wb,
                      double* partials, double* out, hipStream_t s);
void launch_multiaxpy2(const elwh_ctx* c, const double* const* V, int k, const double* h, double* wa, double* wb,
                       hipStream_t s);

enum { RED_SUM = 0, RED_PQ = 1, RED_RR = 2 };

// ---- ragged batch (kernels2d.hip) --------------------------------------------
// Steps per multi-step launch of a batch tick (kb): 4 when the options ask
// for four steps per launch, 2 for two or three, 0 for single steps only.
inline int batch_kb(int fuse) { return fuse >= 4 ? 4 : (fuse >= 2 ? 2 : 0); }
bool batch_tile_valid(bool fp32, int V, int TY, int kb);
int batch_cols(int V);
Args2D make_args2d(const elwh_ctx* c);
void launch_batch_step(bool fp32, int V, int TY, bool force, bool comp, int nblocks, hipStream_t s,
                       const BProb2D* pr, const BState* st, int np, double sgn, int amode, int kb);
// problems with kb or more steps left (kb = 2, 4) take a kb-step launch
void launch_batch_advance(hipStream_t s, const BProb2D* pr, BState* st, int np, int single, int kb, int fp32);
// computed columns per wavefront of the kb-step tiling (kb = 2 or 4)
int batch_cols_k(int V, int kb);
// kb-step tick of every active problem with at least kb steps left in its
// application (kernels2d_multi.hip); nblocks2 = tiles of the kb-step tiling.
void launch_batch_multi(bool fp32, int V, int TY, int kb, bool force, bool comp, int nblocks2, hipStream_t s,
                        const BProb2D* pr, const BState* st, int np, double sgn, int amode);
// CG update kernels of the ragged batch for the nplist problems listed in
// plist (device array of problem indices); arrive: one zeroed counter per
// problem (left zero by every launch).
void launch_batch_cg(hipStream_t s, int mode, const BProb2D* pr, BState* st, int np, const int* plist, int nplist,
                     double* partials, int* arrive, int* n_active);
void launch_batch_lincomb(hipStream_t s, const BProb2D* pr, int np, const int* mask, int idst, int ia,
                          double alpha, int ib, double beta, const double* betav = nullptr);
void launch_batch_dot(hipStream_t s, const BProb2D* pr, int np, const int* mask, int ia, int ib,
                      double* partials, double* out);
constexpr int BATCH_RED_BLOCKS = 64;

}  // namespace elwh
