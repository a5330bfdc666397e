// Ragged batch of 2-D El-WaveHoltz problems (C ABI in include/elwh.h).
//
// Every problem keeps its own context (coefficients, state buffers, work
// vectors, filter weights and N_T).  One "tick" is one batched step launch
// that advances every active problem by one time step of its own filter
// application, followed by the device-side CG updates of the problems whose
// application ended in that tick (Sec. 4.5: alpha = (r,r)_M/(p,A p)_M,
// x += alpha p, r -= alpha A p, beta, p = r + beta p, all in FP64 with
// per-problem two-pass reductions).  A problem that converges drops out; the
// others continue.  The CG phase is captured as a hipGraph of several ticks
// and replayed until no problem is active; the host reads one counter per
// replay.  FP32 batches run the same batched CG with FP32-stepped
// applications and FP64 vectors, in segments: after each segment the
// residual of every unfinished problem is replaced by b - A_h x from an FP64
// application and its search direction continues (stop on that residual).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "elwh_internal.h"

using namespace elwh;

namespace {
enum { VX = 0, VR, VP, VQ, VB, VT, VD, VRI };
constexpr int GRAPH_TICKS = 32;   // ticks per graph replay (one host check of the active count each)
constexpr int kBatchMaxReplace = 8;   // true-residual checks of the FP64 CG per solve
}  // namespace

struct elwh_batch {
    int np = 0;
    std::vector<elwh_ctx*> ctx;
    elwh_opts opts;
    hipStream_t stream = nullptr;   // own stream (graph capture needs a non-null stream)
    hipStream_t user = nullptr;     // caller's stream
    std::string err;
    bool use_graph = true;
    Tile tile[2];                   // [0] FP64, [1] FP32
    std::vector<BProb2D> h_pr;
    std::vector<int> full_blk, full_blk2;   // tiles of each problem in the two tilings of the phase
    BProb2D* d_pr = nullptr;
    std::vector<BState> h_st;
    BState* d_st = nullptr;
    int* d_mask = nullptr;
    int* d_plist = nullptr;         // problems the CG kernels of a tick visit (the live ones)
    int* d_arrive = nullptr;        // per-problem block counters of the CG reductions (kept zero)
    int nplist = 0;
    int gnplist[2] = {0, 0};
    int* d_active = nullptr;
    int* h_active = nullptr;        // pinned
    double* d_partials = nullptr;
    double* d_dots = nullptr;
    double* h_dots = nullptr;       // pinned
    std::vector<double*> d_w, d_cos;
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    int gblocks[2] = {0, 0}, gblocks2[2] = {0, 0};
    std::vector<elwh_info> info;
    double seconds = 0;
    long long ticks = 0;
};

namespace {

thread_local std::string g_batch_err;

#define BCK(expr)                                                               \
    do {                                                                        \
        hipError_t e_ = (expr);                                                 \
        if (e_ != hipSuccess) {                                                 \
            b->err = std::string(#expr) + ": " + hipGetErrorString(e_);         \
            return ELWH_ERR_HIP;                                                \
        }                                                                       \
    } while (0)
#define BST(expr)                     \
    do {                              \
        elwh_status s_ = (expr);      \
        if (s_ != ELWH_OK) return s_; \
    } while (0)

// Descriptors of every problem for one phase (precision fp32), vector roles
// given by indices into the context's work vectors.
elwh_status set_phase(elwh_batch* b, bool fp32, int isrc, int iout, int ix, int ir, int ip, int* nblocks,
                      int* nblocks2 = nullptr) {
    const Tile& t = b->tile[fp32 ? 1 : 0];
    const int W = batch_cols(t.V), W2 = batch_cols_k(t.V, batch_kb(b->opts.fuse));
    int off = 0, off2 = 0;
    b->h_pr.resize(b->np);
    for (int p = 0; p < b->np; ++p) {
        elwh_ctx* c = b->ctx[p];
        BProb2D& q = b->h_pr[p];
        std::memset(&q, 0, sizeof(q));
        q.A = make_args2d(c);
        q.nbx = (q.A.nx - 1 + W - 1) / W;
        const int nrows = q.A.jhi - q.A.jlo + 1;
        q.nblk = q.nbx * ((nrows + t.TY - 1) / t.TY);
        q.off = off;
        off += q.nblk;
        q.nbx2 = (q.A.nx - 1 + W2) / W2;
        q.nblk2 = q.nbx2 * ((nrows + t.TY - 1) / t.TY);
        q.off2 = off2;
        off2 += q.nblk2;
        q.nsteps = c->plan.nt * c->opts.periods;
        q.w = b->d_w[p];
        q.cosn = b->d_cos[p];
        if (fp32) {
            for (int k = 0; k < 4; ++k) q.s[k] = c->s32[k];
            q.ca = c->fa;
            q.cl = c->fl;
            q.cm = c->fm;
            q.f = c->f32;
        } else {
            for (int k = 0; k < 4; ++k) q.s[k] = c->s64[k];
            q.ca = c->ca;
            q.cl = c->cl;
            q.cm = c->cm;
            q.f = c->f64;
        }
        q.src = c->vec[isrc];
        q.out = c->vec[iout];
        q.lo = c->acc_lo;
        q.m = c->mw;
        q.cx = ix >= 0 ? c->vec[ix] : nullptr;
        q.cr = ir >= 0 ? c->vec[ir] : nullptr;
        q.cp = ip >= 0 ? c->vec[ip] : nullptr;
        for (int k = 0; k < 8; ++k) q.vec[k] = c->vec[k];
    }
    *nblocks = off;
    if (nblocks2) *nblocks2 = off2;
    b->full_blk.resize(b->np);
    b->full_blk2.resize(b->np);
    for (int p = 0; p < b->np; ++p) {
        b->full_blk[p] = b->h_pr[p].nblk;
        b->full_blk2[p] = b->h_pr[p].nblk2;
    }
    BCK(hipMemcpyAsync(b->d_pr, b->h_pr.data(), sizeof(BProb2D) * b->np, hipMemcpyHostToDevice, b->stream));
    BCK(hipStreamSynchronize(b->stream));   // h_pr is rewritten by the next phase
    return ELWH_OK;
}

// The problems still active (h_st) as the device list the CG kernels visit.
elwh_status list_active(elwh_batch* b) {
    std::vector<int> pl;
    for (int p = 0; p < b->np; ++p)
        if (b->h_st[p].active) pl.push_back(p);
    b->nplist = (int)pl.size();
    if (!pl.empty())
        BCK(hipMemcpyAsync(b->d_plist, pl.data(), sizeof(int) * pl.size(), hipMemcpyHostToDevice, b->stream));
    BCK(hipStreamSynchronize(b->stream));
    return ELWH_OK;
}

// Keep the tiles of the problems still active (h_st) and give the others
// none, so the step launches of the remaining ticks cover only live
// problems; the launch sizes shrink with the active set.
elwh_status retile_active(elwh_batch* b, int* nblocks, int* nblocks2) {
    int off = 0, off2 = 0;
    for (int p = 0; p < b->np; ++p) {
        BProb2D& q = b->h_pr[p];
        const bool live = b->h_st[p].active != 0;
        q.off = off;
        q.nblk = live ? b->full_blk[p] : 0;
        off += q.nblk;
        q.off2 = off2;
        q.nblk2 = live ? b->full_blk2[p] : 0;
        off2 += q.nblk2;
    }
    *nblocks = off;
    *nblocks2 = off2;
    BCK(hipMemcpyAsync(b->d_pr, b->h_pr.data(), sizeof(BProb2D) * b->np, hipMemcpyHostToDevice, b->stream));
    BCK(hipStreamSynchronize(b->stream));
    return ELWH_OK;
}

elwh_status upload_states(elwh_batch* b) {
    BCK(hipMemcpyAsync(b->d_st, b->h_st.data(), sizeof(BState) * b->np, hipMemcpyHostToDevice, b->stream));
    BCK(hipStreamSynchronize(b->stream));
    return ELWH_OK;
}

elwh_status download_states(elwh_batch* b) {
    BCK(hipMemcpyAsync(b->h_st.data(), b->d_st, sizeof(BState) * b->np, hipMemcpyDeviceToHost, b->stream));
    BCK(hipStreamSynchronize(b->stream));
    return ELWH_OK;
}

elwh_status upload_mask(elwh_batch* b, const std::vector<int>& mask) {
    BCK(hipMemcpyAsync(b->d_mask, mask.data(), sizeof(int) * b->np, hipMemcpyHostToDevice, b->stream));
    BCK(hipStreamSynchronize(b->stream));
    return ELWH_OK;
}

// Ticks of one application: the half step, then kb-step ticks while kb or
// more steps are left, single steps otherwise.
int ticks_per_application(int nsteps, int kb) {
    const int rest = nsteps - 1;
    return 1 + (kb >= 2 ? rest / kb + rest % kb : rest);
}

// One filter application per selected problem: out = Pi_h src (with the
// forcing) or A_h src.  Ragged: runs max N_T ticks.
elwh_status run_apply(elwh_batch* b, bool fp32, bool force, bool amode, int isrc, int iout,
                      const std::vector<int>& sel) {
    int nblocks = 0, nblocks2 = 0;
    BST(set_phase(b, fp32, isrc, iout, -1, -1, -1, &nblocks, &nblocks2));
    const int kb = batch_kb(b->opts.fuse);
    int maxticks = 0;
    for (int p = 0; p < b->np; ++p) {
        BState& s = b->h_st[p];
        s.n = 0;
        s.end = 0;
        s.active = sel[p] ? 1 : 0;
        if (sel[p]) maxticks = std::max(maxticks, ticks_per_application(b->h_pr[p].nsteps, kb));
    }
    BST(upload_states(b));
    const Tile& t = b->tile[fp32 ? 1 : 0];
    const bool comp = fp32 && b->opts.compensated;
    const double sgn = amode ? -1.0 : 1.0;
    for (int k = 0; k < maxticks; ++k) {
        launch_batch_step(fp32, t.V, t.TY, force, comp, nblocks, b->stream, b->d_pr, b->d_st, b->np, sgn,
                          amode ? 1 : 0, kb);
        if (kb)
            launch_batch_multi(fp32, t.V, t.TY, kb, force, comp, nblocks2, b->stream, b->d_pr, b->d_st, b->np, sgn,
                               amode ? 1 : 0);
        launch_batch_advance(b->stream, b->d_pr, b->d_st, b->np, 1, kb, fp32 ? 1 : 0);
        b->ticks++;
    }
    BCK(hipGetLastError());
    return ELWH_OK;
}

elwh_status dots(elwh_batch* b, const std::vector<int>& sel, int ia, int ib, std::vector<double>& out) {
    int nb = 0;
    BST(set_phase(b, false, VT, VQ, -1, -1, -1, &nb));
    BST(upload_mask(b, sel));
    launch_batch_dot(b->stream, b->d_pr, b->np, b->d_mask, ia, ib, b->d_partials, b->d_dots);
    BCK(hipMemcpyAsync(b->h_dots, b->d_dots, sizeof(double) * b->np, hipMemcpyDeviceToHost, b->stream));
    BCK(hipStreamSynchronize(b->stream));
    out.assign(b->h_dots, b->h_dots + b->np);
    for (int p = 0; p < b->np; ++p)
        if (!sel[p]) out[p] = 0.0;
    return ELWH_OK;
}

elwh_status lincomb(elwh_batch* b, const std::vector<int>& sel, int idst, int ia, double alpha, int ib,
                    double beta, const std::vector<double>* betas = nullptr) {
    int nb = 0;
    BST(set_phase(b, false, VT, VQ, -1, -1, -1, &nb));
    BST(upload_mask(b, sel));
    if (betas) {
        // per-problem coefficients staged in the dot-product buffer (free here)
        BCK(hipMemcpyAsync(b->d_dots, betas->data(), sizeof(double) * b->np, hipMemcpyHostToDevice, b->stream));
    }
    launch_batch_lincomb(b->stream, b->d_pr, b->np, b->d_mask, idst, ia, alpha, ib, beta, betas ? b->d_dots : nullptr);
    BCK(hipGetLastError());
    if (betas) BCK(hipStreamSynchronize(b->stream));
    return ELWH_OK;
}

// x <- alpha x, q <- alpha q per selected problem, alpha = (x, b)_M / (x, q)_M
// (q = A_h x in VQ), 0 when (x, q)_M <= 0.
elwh_status scale_start(elwh_batch* b, const std::vector<int>& sel) {
    std::vector<double> xb, xq, alpha(b->np, 0.0);
    BST(dots(b, sel, VX, VB, xb));
    BST(dots(b, sel, VX, VQ, xq));
    for (int p = 0; p < b->np; ++p)
        if (sel[p] && xq[p] > 0 && std::isfinite(xb[p]) && std::isfinite(xq[p])) alpha[p] = xb[p] / xq[p];
    BST(lincomb(b, sel, VX, VX, 0.0, VX, 0.0, &alpha));
    BST(lincomb(b, sel, VQ, VQ, 0.0, VQ, 0.0, &alpha));
    return ELWH_OK;
}

// Problems whose CG broke down ((p, A_h p)_M <= 0) are solved with the
// conjugate residual method (or MINRES) in FP64 from the iterate their CG
// sequence started from (kept in VRI: the last CG iterate before a breakdown
// carries error along nearly A_h-null directions that takes a residual-
// minimising method far longer to remove than a fresh start), one after the
// other on the batch stream; their FP64 residual is then recomputed.
elwh_status cr_fallback(elwh_batch* b, std::vector<int>& status, std::vector<int>& iters, std::vector<int>& cr_iters,
                        std::vector<double>& relres, std::vector<double>& relfp64, const std::vector<double>& bb,
                        double tol, int maxit) {
    std::vector<int> sel(b->np, 0), broken(b->np, 0);
    bool any = false;
    for (int p = 0; p < b->np; ++p) broken[p] = status[p] == ELWH_ERR_BREAKDOWN;
    BST(lincomb(b, broken, VX, VRI, 1.0, -1, 0.0));
    for (int p = 0; p < b->np; ++p) {
        if (!broken[p]) continue;
        int it = 0;
        double rel = 1.0;
        elwh_status st = ctx_solve_fallback(b->ctx[p], b->opts.cr_fallback, tol, std::max(1, maxit - iters[p]), &it,
                                            &rel);
        if (st != ELWH_OK && st != ELWH_ERR_NOT_CONVERGED && st != ELWH_ERR_BREAKDOWN) {
            b->err = elwh_last_error(b->ctx[p]);
            return st;
        }
        cr_iters[p] = it;
        relres[p] = rel;
        status[p] = (tol <= 0 && st == ELWH_ERR_NOT_CONVERGED) ? ELWH_OK : st;
        sel[p] = 1;
        any = true;
    }
    if (!any) return ELWH_OK;
    std::vector<double> rr;
    BST(run_apply(b, false, false, true, VX, VQ, sel));
    BST(lincomb(b, sel, VT, VB, 1.0, VQ, -1.0));
    BST(dots(b, sel, VT, VT, rr));
    for (int p = 0; p < b->np; ++p)
        if (sel[p]) relfp64[p] = bb[p] > 0 ? std::sqrt(rr[p] / bb[p]) : 0.0;
    return ELWH_OK;
}

void enqueue_ticks(elwh_batch* b, bool fp32, int nblocks, int nblocks2, int nticks) {
    const Tile& t = b->tile[fp32 ? 1 : 0];
    const bool comp = fp32 && b->opts.compensated;
    const int kb = batch_kb(b->opts.fuse);
    for (int k = 0; k < nticks; ++k) {
        launch_batch_step(fp32, t.V, t.TY, false, comp, nblocks, b->stream, b->d_pr, b->d_st, b->np, -1.0, 1, kb);
        if (kb)
            launch_batch_multi(fp32, t.V, t.TY, kb, false, comp, nblocks2, b->stream, b->d_pr, b->d_st, b->np, -1.0,
                               1);
        launch_batch_advance(b->stream, b->d_pr, b->d_st, b->np, 0, kb, fp32 ? 1 : 0);
        for (int mode = 0; mode < 3; ++mode)
            launch_batch_cg(b->stream, mode, b->d_pr, b->d_st, b->np, b->d_plist, b->nplist, b->d_partials,
                            b->d_arrive, b->d_active);
    }
}

elwh_status graph_for(elwh_batch* b, bool fp32, int nblocks, int nblocks2) {
    const int k = fp32 ? 1 : 0;
    if (b->gexec[k] && b->gblocks[k] == nblocks && b->gblocks2[k] == nblocks2 && b->gnplist[k] == b->nplist)
        return ELWH_OK;
    if (b->gexec[k]) {
        (void)hipGraphExecDestroy(b->gexec[k]);
        b->gexec[k] = nullptr;
    }
    hipGraph_t g;
    BCK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    enqueue_ticks(b, fp32, nblocks, nblocks2, GRAPH_TICKS);
    BCK(hipStreamEndCapture(b->stream, &g));
    hipError_t e = hipGraphInstantiate(&b->gexec[k], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        b->err = std::string("hipGraphInstantiate: ") + hipGetErrorString(e);
        b->gexec[k] = nullptr;
        return ELWH_ERR_HIP;
    }
    b->gblocks[k] = nblocks;
    b->gblocks2[k] = nblocks2;
    b->gnplist[k] = b->nplist;
    return ELWH_OK;
}

// Ragged CG phase: the states (active, rr, bb, tol2, maxit) are set by the caller.
elwh_status run_cg(elwh_batch* b, bool fp32, int ix, int ir, int ip, int iq, long long max_ticks) {
    int nblocks = 0, nblocks2 = 0;
    BST(set_phase(b, fp32, ip, iq, ix, ir, ip, &nblocks, &nblocks2));
    int nact = 0;
    for (int p = 0; p < b->np; ++p) {
        BState& s = b->h_st[p];
        s.n = 0;
        s.end = 0;
        nact += s.active;
    }
    BST(upload_states(b));
    BST(list_active(b));
    *b->h_active = nact;
    BCK(hipMemcpyAsync(b->d_active, b->h_active, sizeof(int), hipMemcpyHostToDevice, b->stream));
    BCK(hipStreamSynchronize(b->stream));
    if (nact == 0) return ELWH_OK;
    if (b->use_graph) BST(graph_for(b, fp32, nblocks, nblocks2));
    long long ticks = 0;
    // optional progress lines on stderr (ELWH_PROGRESS=1), at most every 10 s
    static const bool progress = [] {
        const char* e = std::getenv("ELWH_PROGRESS");
        return e && e[0] == '1';
    }();
    auto last = std::chrono::steady_clock::now();
    int live = nact;
    while (true) {
        if (b->use_graph) {
            BCK(hipGraphLaunch(b->gexec[fp32 ? 1 : 0], b->stream));
        } else {
            enqueue_ticks(b, fp32, nblocks, nblocks2, GRAPH_TICKS);
        }
        ticks += GRAPH_TICKS;
        b->ticks += GRAPH_TICKS;
        BCK(hipMemcpyAsync(b->h_active, b->d_active, sizeof(int), hipMemcpyDeviceToHost, b->stream));
        BCK(hipStreamSynchronize(b->stream));
        if (*b->h_active <= 0) break;
        if (*b->h_active < live) {
            // problems finished: drop their tiles from the launches (and
            // re-capture the graph for the smaller grids)
            live = *b->h_active;
            BST(download_states(b));
            BST(retile_active(b, &nblocks, &nblocks2));
            BST(list_active(b));
            if (b->use_graph) BST(graph_for(b, fp32, nblocks, nblocks2));
        }
        if (progress && std::chrono::steady_clock::now() - last > std::chrono::seconds(10)) {
            last = std::chrono::steady_clock::now();
            std::fprintf(stderr, "[elwh batch] %s CG: %lld ticks, %d of %d problems active\n", fp32 ? "FP32" : "FP64",
                         ticks, *b->h_active, b->np);
        }
        if (ticks >= max_ticks) {
            b->err = "batched CG exceeded its tick budget";
            break;
        }
    }
    BST(download_states(b));
    return ELWH_OK;
}

void free_batch(elwh_batch* b) {
    for (auto* c : b->ctx) elwh_destroy(c);
    for (auto* p : b->d_w) if (p) (void)hipFree(p);
    for (auto* p : b->d_cos) if (p) (void)hipFree(p);
    auto f = [](void* p) {
        if (p) (void)hipFree(p);
    };
    f(b->d_pr); f(b->d_st); f(b->d_mask); f(b->d_plist); f(b->d_arrive); f(b->d_active); f(b->d_partials);
    f(b->d_dots);
    if (b->h_active) (void)hipHostFree(b->h_active);
    if (b->h_dots) (void)hipHostFree(b->h_dots);
    for (auto& g : b->gexec)
        if (g) (void)hipGraphExecDestroy(g);
    if (b->stream) (void)hipStreamDestroy(b->stream);
}

elwh_status autotune_batch(elwh_batch* b, bool fp32) {
    std::vector<int> all(b->np, 1);
    std::vector<Tile> cands;
    for (int V : {1, 2, 4})
        for (int TY : {4, 8, 10, 16})
            if (batch_tile_valid(fp32, V, TY, batch_kb(b->opts.fuse))) cands.push_back(Tile{V, TY});
    for (int p = 0; p < b->np; ++p)
        BCK(hipMemsetAsync(b->ctx[p]->vec[VT], 0, b->ctx[p]->L.field_elems() * sizeof(double), b->stream));
    hipEvent_t e0, e1;
    BCK(hipEventCreate(&e0));
    BCK(hipEventCreate(&e1));
    double best = 1e300;
    Tile bt = b->tile[fp32 ? 1 : 0];
    for (const Tile& t : cands) {
        b->tile[fp32 ? 1 : 0] = t;
        BST(run_apply(b, fp32, false, true, VT, VD, all));   // warm-up
        (void)hipEventRecord(e0, b->stream);
        BST(run_apply(b, fp32, false, true, VT, VD, all));
        (void)hipEventRecord(e1, b->stream);
        BCK(hipEventSynchronize(e1));
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (ms < best) {
            best = ms;
            bt = t;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    b->tile[fp32 ? 1 : 0] = bt;
    return ELWH_OK;
}

}  // namespace

extern "C" {

elwh_status elwh_batch_create(int nprob, const elwh_grid* grids, const double* const* rho, const double* const* lam,
                              const double* const* mu, const double* omega, const int* bc, const elwh_opts* opts,
                              elwh_batch** out) {
    if (!out) return ELWH_ERR_ARG;
    *out = nullptr;
    g_batch_err.clear();
    if (nprob < 1 || nprob > 4096 || !grids || !rho || !lam || !mu || !omega || !bc) {
        g_batch_err = "bad batch arguments";
        return ELWH_ERR_ARG;
    }
    elwh_opts o;
    elwh_default_opts(&o);
    if (opts) o = *opts;
    elwh_batch* b = new (std::nothrow) elwh_batch();
    if (!b) return ELWH_ERR_ALLOC;
    b->np = nprob;
    b->opts = o;
    b->user = reinterpret_cast<hipStream_t>(o.stream);
    auto fail = [&](elwh_status s, const std::string& msg) {
        g_batch_err = msg;
        free_batch(b);
        delete b;
        return s;
    };
    if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess)
        return fail(ELWH_ERR_HIP, "stream creation failed");
    elwh_opts co = o;
    co.stream = b->stream;
    co.autotune = 0;
    for (int p = 0; p < nprob; ++p) {
        if (grids[p].dim != 2) return fail(ELWH_ERR_ARG, "batches hold 2-D problems");
        for (int f = 0; f < 6; ++f)
            if (bc[6 * p + f] == ELWH_BC_IMPEDANCE)
                return fail(ELWH_ERR_ARG, "impedance faces need the two-field solve (elwh_solve2), not the batch");
        elwh_ctx* c = nullptr;
        const elwh_status st = elwh_create(&grids[p], rho[p], lam[p], mu[p], omega[p], bc + 6 * p, &co, &c);
        if (st != ELWH_OK) return fail(st, "problem " + std::to_string(p) + ": " + elwh_last_error(nullptr));
        b->ctx.push_back(c);
    }
    auto dalloc = [&](void** ptr, size_t bytes) { return hipMalloc(ptr, bytes) == hipSuccess; };
    bool ok = dalloc(reinterpret_cast<void**>(&b->d_pr), sizeof(BProb2D) * nprob) &&
              dalloc(reinterpret_cast<void**>(&b->d_st), sizeof(BState) * nprob) &&
              dalloc(reinterpret_cast<void**>(&b->d_mask), sizeof(int) * nprob) &&
              dalloc(reinterpret_cast<void**>(&b->d_plist), sizeof(int) * nprob) &&
              dalloc(reinterpret_cast<void**>(&b->d_arrive), sizeof(int) * nprob) &&
              dalloc(reinterpret_cast<void**>(&b->d_active), sizeof(int)) &&
              dalloc(reinterpret_cast<void**>(&b->d_partials), 2 * sizeof(double) * nprob * BATCH_RED_BLOCKS) &&
              dalloc(reinterpret_cast<void**>(&b->d_dots), sizeof(double) * nprob) &&
              hipHostMalloc(reinterpret_cast<void**>(&b->h_active), sizeof(int), hipHostMallocDefault) == hipSuccess &&
              hipHostMalloc(reinterpret_cast<void**>(&b->h_dots), sizeof(double) * nprob, hipHostMallocDefault) ==
                  hipSuccess;
    if (!ok) return fail(ELWH_ERR_ALLOC, "batch allocation failed");
    if (hipMemsetAsync(b->d_arrive, 0, sizeof(int) * nprob, b->stream) != hipSuccess)
        return fail(ELWH_ERR_HIP, "clearing the reduction counters failed");
    for (int p = 0; p < nprob; ++p) {
        elwh_ctx* c = b->ctx[p];
        double *w = nullptr, *cs = nullptr;
        const size_t n = c->w.size();
        if (!dalloc(reinterpret_cast<void**>(&w), n * sizeof(double)) ||
            !dalloc(reinterpret_cast<void**>(&cs), n * sizeof(double)))
            return fail(ELWH_ERR_ALLOC, "batch allocation failed");
        b->d_w.push_back(w);
        b->d_cos.push_back(cs);
        if (hipMemcpyAsync(w, c->w.data(), n * sizeof(double), hipMemcpyHostToDevice, b->stream) != hipSuccess ||
            hipMemcpyAsync(cs, c->cosn.data(), n * sizeof(double), hipMemcpyHostToDevice, b->stream) != hipSuccess)
            return fail(ELWH_ERR_HIP, "uploading weights failed");
    }
    b->h_st.assign(nprob, BState{});
    b->info.assign(nprob, elwh_info{});
    // untuned tiles: supported by the single-step and the kb-step batch kernels
    const Tile t0 = batch_kb(o.fuse) == 4 ? Tile{1, 10} : Tile{2, 8};
    b->tile[0] = t0;
    b->tile[1] = t0;
    if (o.autotune) {
        if (autotune_batch(b, false) != ELWH_OK) return fail(ELWH_ERR_HIP, b->err);
        if (o.prec == ELWH_FP32_STEP && autotune_batch(b, true) != ELWH_OK) return fail(ELWH_ERR_HIP, b->err);
    }
    if (hipStreamSynchronize(b->stream) != hipSuccess) return fail(ELWH_ERR_HIP, "synchronisation failed");
    *out = b;
    return ELWH_OK;
}

void elwh_batch_destroy(elwh_batch* b) {
    if (!b) return;
    (void)hipStreamSynchronize(b->stream);
    free_batch(b);
    delete b;
}

const char* elwh_batch_last_error(const elwh_batch* b) { return b ? b->err.c_str() : g_batch_err.c_str(); }

elwh_status elwh_batch_set_graph(elwh_batch* b, int on) {
    if (!b) return ELWH_ERR_ARG;
    b->use_graph = on != 0;
    return ELWH_OK;
}

elwh_status elwh_batch_info(const elwh_batch* b, int i, elwh_info* info) {
    if (!b || !info || i < 0 || i >= b->np) return ELWH_ERR_ARG;
    *info = b->info[i];
    return ELWH_OK;
}

elwh_status elwh_batch_stats(const elwh_batch* b, double* seconds, long long* ticks, int* tile64, int* tile32) {
    if (!b) return ELWH_ERR_ARG;
    if (seconds) *seconds = b->seconds;
    if (ticks) *ticks = b->ticks;
    if (tile64) {
        tile64[0] = b->tile[0].V;
        tile64[1] = b->tile[0].TY;
    }
    if (tile32) {
        tile32[0] = b->tile[1].V;
        tile32[1] = b->tile[1].TY;
    }
    return ELWH_OK;
}

elwh_status elwh_batch_solve(elwh_batch* b, const double* const* f, const double* const* x0, double tol, int maxit,
                             double* const* v, elwh_info* infos) {
    if (!b || !f || !v || maxit < 0) return ELWH_ERR_ARG;
    const auto t0 = std::chrono::steady_clock::now();
    b->ticks = 0;
    const int np = b->np;
    const bool fp32 = b->opts.prec == ELWH_FP32_STEP;
    // order after the caller's pending work
    hipEvent_t ev;
    BCK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    BCK(hipEventRecord(ev, b->user));
    BCK(hipStreamWaitEvent(b->stream, ev, 0));
    std::vector<int> all(np, 1);
    for (int p = 0; p < np; ++p) {
        elwh_ctx* c = b->ctx[p];
        if (!f[p] || !v[p]) {
            (void)hipEventDestroy(ev);
            b->err = "null forcing or output pointer";
            return ELWH_ERR_ARG;
        }
        launch_pack(c->L, c->bc, f[p], c->f64, 2, b->stream);
        if (fp32) launch_convert_f32(c->L, c->f64, c->f32, 2, b->stream);
        if (x0 && x0[p])
            launch_pack(c->L, c->bc, x0[p], c->vec[VX], 2, b->stream);
        else
            BCK(hipMemsetAsync(c->vec[VX], 0, c->L.field_elems() * sizeof(double), b->stream));
        BCK(hipMemsetAsync(c->vec[VT], 0, c->L.field_elems() * sizeof(double), b->stream));
        c->napply = 0;
    }
    // b = Pi_h 0 with the forcing (FP64)
    BST(run_apply(b, false, true, false, VT, VB, all));
    std::vector<double> bb, rr;
    BST(dots(b, all, VB, VB, bb));
    std::vector<int> iters(np, 0), outer(np, 0), status(np, ELWH_ERR_NOT_CONVERGED), cr_iters(np, 0),
        fp64_iters(np, 0);
    std::vector<double> relres(np, 1.0), relfp64(np, 1.0);
    std::vector<int> has_x(np, 0);
    for (int p = 0; p < np; ++p) has_x[p] = (x0 && x0[p]) ? 1 : 0;
    for (int p = 0; p < np; ++p) {
        if (!std::isfinite(bb[p])) {
            (void)hipEventDestroy(ev);
            b->err = "non-finite right-hand side";
            return ELWH_ERR_ARG;
        }
        if (bb[p] > 0) continue;
        // A_h v = 0: the solution is v = 0 whatever the start
        has_x[p] = 0;
        BCK(hipMemsetAsync(b->ctx[p]->vec[VX], 0, b->ctx[p]->L.field_elems() * sizeof(double), b->stream));
    }
    long long max_nsteps = 0;
    for (auto* c : b->ctx) max_nsteps = std::max<long long>(max_nsteps, (long long)c->plan.nt * c->opts.periods);
    const long long tick_budget = (long long)(maxit + 2) * max_nsteps + 64;

    // Convergence is judged on the true residual, recomputed with an FP64
    // apply: a problem of sel whose recurrence residual met tol but whose true
    // residual did not has r replaced by b - A_h x and continues FP64 CG along
    // the same search direction (a reliable update), like elwh_solve.  Sets
    // relfp64 of every problem in sel; the iterations go to iters (and to
    // extra, when given).
    auto true_residual_continue = [&](const std::vector<int>& sel, std::vector<int>* extra) -> elwh_status {
        for (int rep = 0;; ++rep) {
            BST(run_apply(b, false, false, true, VX, VQ, sel));
            BST(lincomb(b, sel, VT, VB, 1.0, VQ, -1.0));
            BST(dots(b, sel, VT, VT, rr));
            std::vector<int> more(np, 0);
            bool any = false;
            for (int p = 0; p < np; ++p) {
                if (!sel[p]) continue;
                relfp64[p] = bb[p] > 0 ? std::sqrt(rr[p] / bb[p]) : 0.0;
                if (tol <= 0 || !(bb[p] > 0) || status[p] != ELWH_OK || relfp64[p] <= tol) continue;
                if (iters[p] >= maxit || rep + 1 >= kBatchMaxReplace) {
                    status[p] = ELWH_ERR_NOT_CONVERGED;
                    continue;
                }
                more[p] = 1;
                any = true;
            }
            if (!any) return ELWH_OK;
            // r = b - A_h x; p = r + beta p with beta = (r, r)_M / (r_k, r_k)_M, r_k
            // the residual before the last CG step (rr_k = rr / beta of that step)
            std::vector<double> beta(np, 0.0);
            for (int p = 0; p < np; ++p) {
                const BState& s = b->h_st[p];
                if (more[p] && s.beta > 0 && s.rr > 0) beta[p] = rr[p] / (s.rr / s.beta);
            }
            BST(lincomb(b, more, VR, VT, 1.0, -1, 0.0));
            BST(lincomb(b, more, VP, VR, 1.0, VP, 0.0, &beta));
            for (int p = 0; p < np; ++p) {
                BState& s = b->h_st[p];
                const int keep_iters = iters[p];
                std::memset(&s, 0, sizeof(s));
                if (!more[p]) continue;
                s.rr = rr[p];
                s.bb = bb[p];
                s.tol2 = tol * tol;
                s.maxit = std::max(1, maxit - keep_iters);
                s.status = ELWH_ERR_NOT_CONVERGED;
                s.active = 1;
            }
            BST(run_cg(b, false, VX, VR, VP, VQ, tick_budget));
            for (int p = 0; p < np; ++p) {
                if (!more[p]) continue;
                outer[p]++;
                iters[p] += b->h_st[p].iters;
                if (extra) (*extra)[p] += b->h_st[p].iters;
                status[p] = b->h_st[p].status;
                if (status[p] == ELWH_ERR_NOT_CONVERGED && iters[p] < maxit) status[p] = ELWH_OK;
                relres[p] = std::sqrt(b->h_st[p].rr / bb[p]);
            }
        }
    };

    if (!fp32) {
        // r = b - A x0, p = r
        bool anyx = false;
        for (int p = 0; p < np; ++p) anyx |= has_x[p] != 0;
        if (anyx) {
            BST(run_apply(b, false, false, true, VX, VQ, has_x));
            if (b->opts.scale_x0) BST(scale_start(b, has_x));
            BST(lincomb(b, has_x, VR, VB, 1.0, VQ, -1.0));
        }
        std::vector<int> nox(np);
        for (int p = 0; p < np; ++p) nox[p] = !has_x[p];
        BST(lincomb(b, nox, VR, VB, 1.0, -1, 0.0));
        BST(lincomb(b, all, VP, VR, 1.0, -1, 0.0));
        BST(lincomb(b, all, VRI, VX, 1.0, -1, 0.0));   // the start, for a fallback after a breakdown
        BST(dots(b, all, VR, VR, rr));
        for (int p = 0; p < np; ++p) {
            BState& s = b->h_st[p];
            std::memset(&s, 0, sizeof(s));
            s.rr = rr[p];
            s.bb = bb[p];
            s.tol2 = tol > 0 ? tol * tol : -1.0;
            s.maxit = maxit;
            s.status = ELWH_ERR_NOT_CONVERGED;
            const bool done = !(bb[p] > 0) || (tol > 0 && rr[p] <= s.tol2 * bb[p]) || maxit == 0;
            s.active = done ? 0 : 1;
            if (done) s.status = ELWH_OK;
        }
        BST(run_cg(b, false, VX, VR, VP, VQ, tick_budget));
        for (int p = 0; p < np; ++p) {
            iters[p] = b->h_st[p].iters;
            status[p] = b->h_st[p].status;
            if (tol <= 0 && status[p] == ELWH_ERR_NOT_CONVERGED) status[p] = ELWH_OK;
            relres[p] = bb[p] > 0 ? std::sqrt(b->h_st[p].rr / bb[p]) : 0.0;
        }
        BST(true_residual_continue(all, nullptr));
        if (b->opts.cr_fallback) BST(cr_fallback(b, status, iters, cr_iters, relres, relfp64, bb, tol, maxit));
    } else {
        // FP32 stepping inside CG with FP64 reliable updates (as elwh_solve):
        // x, r, p stay FP64; each segment runs device-driven CG with FP32
        // applications until the recursive residual has fallen by inner_tol
        // (or below the target); then r is replaced by b - A_h x from an FP64
        // application and the search direction continues from it.
        bool anyx = false;
        for (int p = 0; p < np; ++p) anyx |= has_x[p] != 0;
        if (anyx) {
            BST(run_apply(b, false, false, true, VX, VQ, has_x));
            if (b->opts.scale_x0) BST(scale_start(b, has_x));
            BST(lincomb(b, has_x, VR, VB, 1.0, VQ, -1.0));
        }
        std::vector<int> nox(np);
        for (int p = 0; p < np; ++p) nox[p] = !has_x[p];
        BST(lincomb(b, nox, VR, VB, 1.0, -1, 0.0));
        BST(lincomb(b, all, VP, VR, 1.0, -1, 0.0));
        BST(lincomb(b, all, VRI, VX, 1.0, -1, 0.0));   // the start, for a fallback after a breakdown
        BST(dots(b, all, VR, VR, rr));
        std::vector<double> seg = rr, rr_k(np, 0.0), beta(np, 0.0);
        std::vector<int> done_p(np, 0), stag(np, 0), longest(np, 0), capped(np, 0);
        std::vector<std::vector<double>> hist(np);   // FP64 residual after each segment
        for (int p = 0; p < np; ++p) {
            relfp64[p] = bb[p] > 0 ? std::sqrt(rr[p] / bb[p]) : 0.0;
            relres[p] = relfp64[p];
        }
        // FP64 first (opts.fp32_switch > 0): FP64 CG down to the switch
        // residual, then a residual replacement that keeps the search
        // direction; the FP32 segments below continue the same Krylov sequence
        if (b->opts.fp32_switch > 0 && tol > 0 && maxit > 0) {
            const double sw = std::max(b->opts.fp32_switch, tol);
            std::vector<int> ph(np, 0), repl(np, 0);
            bool anyph = false;
            for (int p = 0; p < np; ++p) {
                BState& s = b->h_st[p];
                std::memset(&s, 0, sizeof(s));
                if (!(bb[p] > 0) || !(relfp64[p] > sw)) continue;
                ph[p] = 1;
                anyph = true;
                s.active = 1;
                s.rr = rr[p];
                s.bb = bb[p];
                s.tol2 = sw * sw;
                s.maxit = maxit;
                s.status = ELWH_ERR_NOT_CONVERGED;
            }
            if (anyph) {
                BST(run_cg(b, false, VX, VR, VP, VQ, tick_budget));
                for (int p = 0; p < np; ++p) {
                    if (!ph[p]) continue;
                    const BState& s = b->h_st[p];
                    iters[p] += s.iters;
                    fp64_iters[p] += s.iters;
                    relres[p] = std::sqrt(s.rr / bb[p]);
                    if (s.status == ELWH_ERR_BREAKDOWN || s.status == ELWH_ERR_UNSTABLE) {
                        status[p] = s.status;   // (a breakdown goes to the CR fallback below)
                    } else if (s.status == ELWH_OK) {
                        repl[p] = 1;
                        rr_k[p] = s.beta > 0 ? s.rr / s.beta : 0.0;
                    } else {
                        relfp64[p] = relres[p];   // out of iterations: the loop head ends it
                    }
                }
                BST(run_apply(b, false, false, true, VX, VQ, repl));
                BST(lincomb(b, repl, VR, VB, 1.0, VQ, -1.0));
                BST(dots(b, repl, VR, VR, rr));
                for (int p = 0; p < np; ++p) {
                    if (!repl[p]) continue;
                    relfp64[p] = std::sqrt(rr[p] / bb[p]);
                    seg[p] = rr[p];
                    beta[p] = rr_k[p] > 0 ? rr[p] / rr_k[p] : 0.0;
                }
                BST(lincomb(b, repl, VP, VR, 1.0, VP, 0.0, &beta));
            }
        }
        for (int p = 0; p < np; ++p) hist[p].push_back(relfp64[p]);
        for (int o = 0;; ++o) {
            std::vector<int> pending(np, 0);
            bool any = false;
            for (int p = 0; p < np; ++p) {
                if (status[p] != ELWH_ERR_NOT_CONVERGED || done_p[p]) continue;
                if (!(bb[p] > 0) || (tol > 0 && relfp64[p] <= tol)) {
                    status[p] = ELWH_OK;
                } else if (!std::isfinite(relfp64[p])) {
                    status[p] = ELWH_ERR_UNSTABLE;
                } else if (iters[p] >= maxit || o > b->opts.max_outer) {
                    status[p] = tol > 0 ? ELWH_ERR_NOT_CONVERGED : ELWH_OK;
                    done_p[p] = 1;
                } else if (b->opts.fp64_fallback && tol > 0 &&
                           (stag[p] == 2 || (hist[p].size() >= 3 && relfp64[p] > 0.5 * hist[p][hist[p].size() - 3]))) {
                    stag[p] = 1;   // a segment over its cap, or less than a halving over two segments: FP64 below
                    done_p[p] = 1;
                } else {
                    pending[p] = 1;
                    any = true;
                }
            }
            if (!any) break;
            for (int p = 0; p < np; ++p) {
                BState& s = b->h_st[p];
                std::memset(&s, 0, sizeof(s));
                s.active = pending[p];
                s.rr = seg[p];
                s.bb = 1.0;
                const double stop = tol > 0 ? 0.25 * tol * tol * bb[p] : 0.0;
                s.tol2 = std::max(b->opts.inner_tol * b->opts.inner_tol * seg[p], stop);
                s.maxit = std::max(1, maxit - iters[p]);
                // with the fallback on, a segment may take at most twice the
                // iterations of the longest earlier one (at least 64)
                const int cap = std::max(64, 2 * longest[p]);
                capped[p] = b->opts.fp64_fallback && tol > 0 && o > 0 && s.maxit > cap;
                if (capped[p]) s.maxit = cap;
                s.status = ELWH_ERR_NOT_CONVERGED;
            }
            BST(run_cg(b, true, VX, VR, VP, VQ, tick_budget));
            for (int p = 0; p < np; ++p) {
                if (!pending[p]) continue;
                const BState& s = b->h_st[p];
                iters[p] += s.iters;
                outer[p] = o + 1;
                longest[p] = std::max(longest[p], s.iters);
                if (capped[p] && s.status == ELWH_ERR_NOT_CONVERGED) stag[p] = 2;   // segment over its cap
                relres[p] = std::sqrt(s.rr / bb[p]);
                rr_k[p] = s.beta > 0 ? s.rr / s.beta : 0.0;
                if (s.status == ELWH_ERR_BREAKDOWN || s.status == ELWH_ERR_UNSTABLE) {
                    status[p] = s.status;
                    pending[p] = 0;
                }
            }
            // residual replacement: r = b - A_h x (FP64), p = r + beta p
            BST(run_apply(b, false, false, true, VX, VQ, pending));
            BST(lincomb(b, pending, VR, VB, 1.0, VQ, -1.0));
            BST(dots(b, pending, VR, VR, rr));
            for (int p = 0; p < np; ++p) {
                if (!pending[p]) continue;
                relfp64[p] = std::sqrt(rr[p] / bb[p]);
                seg[p] = rr[p];
                beta[p] = rr_k[p] > 0 ? rr[p] / rr_k[p] : 0.0;
                hist[p].push_back(relfp64[p]);
            }
            BST(lincomb(b, pending, VP, VR, 1.0, VP, 0.0, &beta));
        }
        // problems whose FP32 segments stopped improving x: FP64 CG from x
        bool anystag = false;
        for (int p = 0; p < np; ++p) {
            if (stag[p] != 1) stag[p] = 0;   // over a cap but finished otherwise
            anystag |= stag[p] != 0;
        }
        if (anystag) {
            BST(lincomb(b, stag, VRI, VX, 1.0, -1, 0.0));   // a new CG sequence starts here
            BST(run_apply(b, false, false, true, VX, VQ, stag));
            BST(lincomb(b, stag, VR, VB, 1.0, VQ, -1.0));
            BST(lincomb(b, stag, VP, VR, 1.0, -1, 0.0));
            BST(dots(b, stag, VR, VR, rr));
            for (int p = 0; p < np; ++p) {
                BState& s = b->h_st[p];
                std::memset(&s, 0, sizeof(s));
                if (!stag[p]) continue;
                s.rr = rr[p];
                s.bb = bb[p];
                s.tol2 = tol * tol;
                s.maxit = std::max(1, maxit - iters[p]);
                s.status = ELWH_ERR_NOT_CONVERGED;
                s.active = rr[p] <= s.tol2 * bb[p] ? 0 : 1;
                if (!s.active) s.status = ELWH_OK;
            }
            BST(run_cg(b, false, VX, VR, VP, VQ, tick_budget));
            for (int p = 0; p < np; ++p) {
                if (!stag[p]) continue;
                fp64_iters[p] += b->h_st[p].iters;
                iters[p] += b->h_st[p].iters;
                status[p] = b->h_st[p].status;
                relres[p] = std::sqrt(b->h_st[p].rr / bb[p]);
            }
            // judged on the true residual, as the FP64 path
            BST(true_residual_continue(stag, &fp64_iters));
        }
        if (b->opts.cr_fallback) BST(cr_fallback(b, status, iters, cr_iters, relres, relfp64, bb, tol, maxit));
    }
    for (int p = 0; p < np; ++p) launch_unpack(b->ctx[p]->L, b->ctx[p]->bc, b->ctx[p]->vec[VX], v[p], 2, b->stream);
    BCK(hipEventRecord(ev, b->stream));
    BCK(hipStreamWaitEvent(b->user, ev, 0));
    BCK(hipStreamSynchronize(b->stream));
    (void)hipEventDestroy(ev);
    b->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    elwh_status worst = ELWH_OK;
    for (int p = 0; p < np; ++p) {
        elwh_info& in = b->info[p];
        std::memset(&in, 0, sizeof(in));
        elwh_ctx* c = b->ctx[p];
        in.iters = iters[p];
        in.outer = outer[p];
        in.nt = c->plan.nt;
        in.dt = c->plan.dt;
        in.c = c->plan.c;
        in.lambda_bound = c->plan.lambda_bound;
        in.relres = relres[p];
        in.relres_fp64 = relfp64[p];
        in.cond_est = NAN;
        in.cr_iters = cr_iters[p];
        in.fp64_iters = fp64_iters[p];
        if (infos) infos[p] = in;
        if (status[p] != ELWH_OK && worst == ELWH_OK) worst = (elwh_status)status[p];
        if (status[p] == ELWH_ERR_BREAKDOWN || status[p] == ELWH_ERR_UNSTABLE) worst = (elwh_status)status[p];
    }
    if (worst != ELWH_OK && b->err.empty()) b->err = "at least one problem did not converge";
    return worst;
}

}  // extern "C"
