"""GPU parity: the HIP path (through the C ABI) against the CPU FP64 oracle on
the same seeded inputs.

Bars.  FP64: rel-L2 <= 1e-12 per application (the stated FP64 tolerance).
FP32 stepping: rel-L2 <= fp32_bound(N_T) = 2 u32 sqrt(N_T) N_T / (2 pi)
+ 8 u32 per application, u32 = 2^-24: one rounding per step, accumulated as
a random walk over N_T steps and amplified by at most 1/sin(theta_min) ~
N_T/(2 pi), the bound of the leapfrog's discrete Green's function for the
slowest mode of one period; plus the FP32 rounding of the inputs u^0, f and
of the coefficients a, lambda, mu (each a relative perturbation of at most
u32 of a map of norm below 2), which dominates at very small N_T.  Solves:
the stated residuals."""

import math
import sys

import numpy as np
import pytest

from oracle import direct, krylov
from oracle import stepping as S
from oracle.operator import Operator
from oracle.problem import Problem
from paper_2205_12344_amd import inputs

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
U32 = 2.0 ** -24


def fp32_bound(nt):
    return 2.0 * U32 * math.sqrt(nt) * nt / (2 * math.pi) + 8.0 * U32


def _say(*a):
    print("[gpu-test]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def E():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_12344_amd import elwh
    return elwh


def _media(shape, seed, s=0.25):
    rng = np.random.default_rng(seed)
    rho = np.exp(s * rng.standard_normal(shape))
    mu = np.exp(s * rng.standard_normal(shape))
    lam = mu * np.clip(2 * np.exp(s * rng.standard_normal(shape)), 1, 3)
    return rho, lam, mu


def _rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def _oracle(dim, n, length, bc, rho, lam, mu, omega, **kw):
    prob = Problem(dim, n, length=length, bc=bc)
    op = Operator(prob, rho, lam, mu)
    wh = S.WaveHoltz(op, omega, **kw)
    return prob, op, wh


# 2-D grids: ragged in x (62 computed columns per wavefront) and in y (16 rows
# per block), free faces on y, one-column and two-row extremes
CASES_2D = [
    ((130, 37), (0, 0, 0, 1), (1.0, 0.8)),
    ((63, 16), (0, 0, 0, 0), (1.0, 1.0)),
    ((64, 33), (0, 0, 1, 0), (0.9, 1.1)),
    ((125, 20), (0, 0, 1, 1), (1.0, 0.5)),
    ((2, 40), (0, 0, 0, 1), (1.0, 1.0)),
    ((50, 2), (0, 0, 1, 1), (1.0, 1.0)),
]


@pytest.mark.parametrize("n,bc,length", CASES_2D)
@pytest.mark.parametrize("force", [False, True])
@pytest.mark.parametrize("fuse", [2, 1, 3, 4])
def test_filter_2d_fp64(E, n, bc, length, force, fuse):
    _say("filter2d fp64", n, bc, force, "fuse", fuse)
    rho, lam, mu = _media((n[1] + 1, n[0] + 1), sum(n))
    om = 9.3
    prob, op, wh = _oracle(2, n, length, bc, rho, lam, mu, om)
    rng = np.random.default_rng(7)
    u0 = rng.standard_normal(prob.field_shape) * prob.unknown_mask()
    f = rng.standard_normal(prob.field_shape) * prob.unknown_mask() if force else None
    ref = prob.scatter(wh.apply_filter(prob.gather(u0), prob.gather(f) if force else None))
    ctx = E.Context(2, n, rho, lam, mu, om, bc, length=length, fuse=fuse)
    assert ctx.info()["nt"] == wh.nt
    got = ctx.apply_filter(u0, f).cpu().numpy()
    assert _rel(got, ref) <= FP64_TOL
    # A_h x = x - S_h x
    gotA = ctx.apply_A(u0).cpu().numpy()
    refA = prob.scatter(wh.apply_A(prob.gather(u0)))
    assert _rel(gotA, refA) <= FP64_TOL


CASES_3D = [
    ((70, 9, 37), (0, 0, 0, 0, 0, 0), (1.0, 0.7, 1.2)),
    ((20, 11, 18), (0, 0, 0, 0, 0, 1), (1.0, 1.0, 1.0)),
    ((33, 6, 17), (0, 0, 0, 0, 1, 1), (1.0, 1.0, 0.8)),
    ((2, 2, 2), (0, 0, 0, 0, 1, 0), (1.0, 1.0, 1.0)),
]


@pytest.mark.parametrize("n,bc,length", CASES_3D)
@pytest.mark.parametrize("force", [False, True])
@pytest.mark.parametrize("fuse", [2, 1])
def test_filter_3d_fp64(E, n, bc, length, force, fuse):
    _say("filter3d fp64", n, bc, force, "steps per launch", fuse)
    shape = (n[2] + 1, n[1] + 1, n[0] + 1)
    rho, lam, mu = _media(shape, sum(n) + 1)
    om = 6.1
    prob, op, wh = _oracle(3, n, length, bc, rho, lam, mu, om)
    rng = np.random.default_rng(8)
    u0 = rng.standard_normal(prob.field_shape) * prob.unknown_mask()
    f = rng.standard_normal(prob.field_shape) * prob.unknown_mask() if force else None
    ref = prob.scatter(wh.apply_filter(prob.gather(u0), prob.gather(f) if force else None))
    ctx = E.Context(3, n, rho, lam, mu, om, bc, length=length, fuse=fuse)
    assert ctx.info()["nt"] == wh.nt
    got = ctx.apply_filter(u0, f).cpu().numpy()
    assert _rel(got, ref) <= FP64_TOL


@pytest.mark.parametrize("dim", [2, 3])
def test_filter_fp32_stepping(E, dim):
    n = (90, 41) if dim == 2 else (40, 13, 22)
    bc = (0, 0, 0, 1) if dim == 2 else (0, 0, 0, 0, 0, 1)
    _say("filter fp32", dim, n)
    shape = tuple(n[a] + 1 for a in reversed(range(dim)))
    rho, lam, mu = _media(shape, 31 + dim)
    om = 7.0
    prob, op, wh = _oracle(dim, n, None, bc, rho, lam, mu, om)
    rng = np.random.default_rng(9)
    u0 = rng.standard_normal(prob.field_shape) * prob.unknown_mask()
    f = rng.standard_normal(prob.field_shape) * prob.unknown_mask()
    ref = prob.scatter(wh.apply_filter(prob.gather(u0), prob.gather(f)))
    runs = {}
    for comp in (1, 0):
        for fuse in ((2, 1, 3, 4) if dim == 2 else (2, 1)):
            ctx = E.Context(dim, n, rho, lam, mu, om, bc, prec=E.FP32_STEP, compensated=comp, fuse=fuse)
            got = runs[comp, fuse] = ctx.apply_filter(u0, f).cpu().numpy()
            err = _rel(got, ref)
            _say("  fp32 compensated", comp, "fuse", fuse, "nt", wh.nt, "rel err", err, "bound", fp32_bound(wh.nt))
            assert err <= fp32_bound(wh.nt)
    # The FP32 states do not depend on how the accumulator is summed, so the
    # compensated and plain results differ only by the plain FP64 summation's
    # rounding (about N_T * 2^-53 of the terms): a compensation word read or
    # written wrongly would show far above that.
    for (comp, fuse), got in runs.items():
        if comp:
            d = _rel(got, runs[0, fuse])
            _say("  compensated vs plain, fuse", fuse, d)
            assert d <= 1e-12


@pytest.mark.parametrize("nt", [3, 4, 5, 8, 9])
@pytest.mark.parametrize("prec", [0, 1])
def test_multi_step_every_step_count_3d(E, nt, prec):
    """Two-step 3-D launches with every remainder (N_T = 3, 4, 5, 8, 9; the
    half step, pairs, a last single step) against the oracle, FP64 and FP32,
    with free z faces and forcing."""
    n, bc = (47, 13, 21), (0, 0, 0, 0, 1, 1)
    rho, lam, mu = _media((22, 14, 48), 300 + nt)
    prob, op, wh = _oracle(3, n, None, bc, rho, lam, mu, 3.1, nt=nt)
    rng = np.random.default_rng(nt)
    u0 = rng.standard_normal(prob.field_shape) * prob.unknown_mask()
    f = rng.standard_normal(prob.field_shape) * prob.unknown_mask()
    ref = prob.scatter(wh.apply_filter(prob.gather(u0), prob.gather(f)))
    ctx = E.Context(3, n, rho, lam, mu, 3.1, bc, nt=nt, prec=prec, fuse=2)
    err = _rel(ctx.apply_filter(u0, f).cpu().numpy(), ref)
    _say("3-D two-step nt", nt, "prec", prec, "err", err)
    assert err <= (FP64_TOL if prec == 0 else fp32_bound(nt))


@pytest.mark.parametrize("nt", [3, 4, 5, 8, 9])
@pytest.mark.parametrize("prec", [0, 1])
def test_multi_step_every_step_count(E, nt, prec):
    """Half step + K-step launches (with a shorter launch or a single step
    for the remainder of N_T - 1) give the oracle's filter and A_h for every
    N_T and K = 2, 3, 4, with forcing, and agree with single-step launches.
    omega is chosen so that the time-step rule itself gives N_T (a smaller
    N_T than the rule's would be unstable)."""
    n, bc = (131, 23), (0, 0, 1, 1)
    rho, lam, mu = _media((24, 132), 300 + nt)
    prob = Problem(2, n, bc=bc)
    G = Operator(prob, rho, lam, mu).gershgorin()
    dt_star = 0.8 * 2.0 / math.sqrt(G)
    om = 2 * math.pi / (nt * dt_star) * 1.001
    prob, op, wh = _oracle(2, n, None, bc, rho, lam, mu, om)
    assert wh.nt == nt
    rng = np.random.default_rng(nt)
    u0 = rng.standard_normal(prob.field_shape) * prob.unknown_mask()
    f = rng.standard_normal(prob.field_shape) * prob.unknown_mask()
    ref = prob.scatter(wh.apply_filter(prob.gather(u0), prob.gather(f)))
    refA = prob.scatter(wh.apply_A(prob.gather(u0)))
    tol = FP64_TOL if prec == 0 else fp32_bound(nt)
    outs = {}
    for fuse in (2, 3, 4, 1):
        ctx = E.Context(2, n, rho, lam, mu, om, bc, prec=prec, fuse=fuse, autotune=0)
        assert ctx.info()["nt"] == nt
        got = ctx.apply_filter(u0, f).cpu().numpy()
        gotA = ctx.apply_A(u0).cpu().numpy()
        _say("pairs nt", nt, "prec", prec, "fuse", fuse, _rel(got, ref), _rel(gotA, refA))
        assert _rel(got, ref) <= tol
        assert _rel(gotA, refA) <= tol
        outs[fuse] = got
    for k in (2, 3, 4):
        assert _rel(outs[k], outs[1]) <= 2 * tol


def test_k_periods_and_standard_scheme(E):
    n, bc = (47, 29), (0, 0, 0, 1)
    rho, lam, mu = _media((30, 48), 41)
    rng = np.random.default_rng(10)
    for kw in ({"periods": 3}, {"scheme": 1}, {"nt": 40}, {"cfl": 0.3}):
        _say("variant", kw)
        okw = {k: (S.STANDARD if k == "scheme" else v) for k, v in kw.items()}
        prob, op, wh = _oracle(2, n, None, bc, rho, lam, mu, 5.5, **okw)
        u0 = rng.standard_normal(prob.field_shape) * prob.unknown_mask()
        ref = prob.scatter(wh.apply_filter(prob.gather(u0)))
        ctx = E.Context(2, n, rho, lam, mu, 5.5, bc, **kw)
        assert ctx.info()["nt"] == wh.nt
        assert _rel(ctx.apply_filter(u0).cpu().numpy(), ref) <= FP64_TOL


def test_dot_M(E):
    n, bc = (33, 20), (0, 0, 1, 1)
    rho, lam, mu = _media((21, 34), 51)
    prob = Problem(2, n, bc=bc)
    m = prob.mass_diag(rho)
    rng = np.random.default_rng(11)
    x = rng.standard_normal(prob.field_shape)
    y = rng.standard_normal(prob.field_shape)
    ctx = E.Context(2, n, rho, lam, mu, 3.0, bc)
    got = ctx.dot_M(x, y)
    ref = float(np.dot(m * prob.gather(x), prob.gather(y)))
    assert got == pytest.approx(ref, rel=1e-13)


def test_fixed_point_square64(E):
    """Sec. 1.1 / 4.3: Pi_h v* = v* with v* the direct Helmholtz solve."""
    c = inputs.constant_square64()
    prob, op, wh = _oracle(2, c.n, None, c.bc, c.rho, c.lam, c.mu, c.omega)
    v = prob.scatter(direct.solve(op, c.omega, prob.gather(c.f)))
    ctx = E.context_from_case(c)
    got = ctx.apply_filter(v, c.f).cpu().numpy()
    assert _rel(got, v) <= FP64_TOL


def test_solve_square64_matches_direct_and_oracle_cg(E):
    """64^2 constant medium: CG to 1e-10 matches the direct solve (<= 1e-10) and the
    oracle's CG iterate after the same number of iterations (<= 1e-12)."""
    c = inputs.constant_square64()
    prob, op, wh = _oracle(2, c.n, None, c.bc, c.rho, c.lam, c.mu, c.omega)
    fv = prob.gather(c.f)
    vstar = direct.solve(op, c.omega, fv)
    ctx = E.context_from_case(c)
    v, info = ctx.solve(c.f, tol=1e-10, maxit=200)
    _say("square64 solve", info)
    v = v.cpu().numpy()
    assert info["iters"] <= 20
    assert info["relres_fp64"] <= 1e-10
    assert _rel(prob.gather(v), vstar) <= 1e-10
    res = krylov.cg(wh.apply_A, wh.rhs(fv), op.m, tol=1e-10, maxit=200)
    # no residual replacement was needed here: the recurrence residual and
    # the true one agree, so the solve is the oracle's plain CG
    assert info["outer"] == 0
    assert res.iters == info["iters"]
    assert _rel(prob.gather(v), res.x) <= 1e-12
    assert info["cond_est"] == pytest.approx(res.lanczos_cond(), rel=1e-6)
    # tighter solve reaches the direct solution to 1e-12
    v2, info2 = ctx.solve(c.f, tol=1e-13, maxit=200)
    assert _rel(prob.gather(v2.cpu().numpy()), vstar) <= 1e-12


@pytest.mark.parametrize("prec", [0, 1])
def test_scaled_start_single_context(E, prec):
    """scale_x0 on elwh_solve: 3 v* as the start is rescaled to v* (no
    iteration needed); the unscaled 3 v* start needs several."""
    c = inputs.constant_square64()
    prob, op, wh = _oracle(2, c.n, None, c.bc, c.rho, c.lam, c.mu, c.omega)
    vstar = direct.solve(op, c.omega, prob.gather(c.f))
    x0 = 3.0 * prob.scatter(vstar)
    ctx = E.context_from_case(c, prec=prec, scale_x0=1)
    v, info = ctx.solve(c.f, x0=x0, tol=1e-8, maxit=200)
    plain = E.context_from_case(c, prec=prec)
    _, info_plain = plain.solve(c.f, x0=x0, tol=1e-8, maxit=200)
    _say("scaled start", info["iters"], "unscaled", info_plain["iters"])
    assert info["iters"] <= 1 < info_plain["iters"]
    assert _rel(prob.gather(v.cpu().numpy()), vstar) <= 1e-7


def test_stepwise_cg_and_warm_start(E):
    c = inputs.constant_square64()
    prob, op, wh = _oracle(2, c.n, None, c.bc, c.rho, c.lam, c.mu, c.omega)
    fv = prob.gather(c.f)
    ctx = E.context_from_case(c)
    ctx.cg_begin(c.f)
    r5 = ctx.cg_iterate(5)
    res5 = krylov.cg(wh.apply_A, wh.rhs(fv), op.m, tol=0.0, maxit=5)
    assert r5 == pytest.approx(res5.history[-1], rel=1e-9)
    v5, _ = ctx.cg_result()
    assert _rel(prob.gather(v5.cpu().numpy()), res5.x) <= 1e-12
    # resume by restart from the 5-iteration iterate
    v, info = ctx.solve(c.f, x0=v5, tol=1e-10, maxit=200)
    vstar = direct.solve(op, c.omega, fv)
    assert _rel(prob.gather(v.cpu().numpy()), vstar) <= 1e-9


@pytest.mark.parametrize("krylov_id", [1, 2])
def test_gmres_and_cr_match_direct(E, krylov_id):
    n, bc = (40, 30), (0, 0, 0, 1)
    rho, lam, mu = _media((31, 41), 61)
    om = 6.3
    prob, op, wh = _oracle(2, n, None, bc, rho, lam, mu, om)
    rng = np.random.default_rng(12)
    f = rng.standard_normal(prob.field_shape) * prob.unknown_mask()
    vstar = direct.solve(op, om, prob.gather(f))
    ctx = E.Context(2, n, rho, lam, mu, om, bc, krylov=krylov_id, gmres_m=20)
    v, info = ctx.solve(f, tol=1e-11, maxit=500)
    _say("krylov", krylov_id, info)
    assert info["relres_fp64"] <= 2e-11
    assert _rel(prob.gather(v.cpu().numpy()), vstar) <= 1e-9


@pytest.mark.parametrize("dim", [2, 3])
def test_gmres_iterations_match_oracle(E, dim):
    """GMRES(20) with the Gram-Schmidt coefficients on the device takes the
    oracle's GMRES(20) iteration count (CGS2 in the M inner product)."""
    n = (40, 30) if dim == 2 else (14, 12, 10)
    bc = (0, 0, 0, 1) if dim == 2 else (0, 0, 0, 0, 0, 1)
    rho, lam, mu = _media(tuple(k + 1 for k in reversed(n)), 62)
    om = 6.3 if dim == 2 else 4.1
    prob, op, wh = _oracle(dim, n, None, bc, rho, lam, mu, om)
    rng = np.random.default_rng(14)
    f = rng.standard_normal(prob.field_shape) * prob.unknown_mask()
    ctx = E.Context(dim, n, rho, lam, mu, om, bc, krylov=1, gmres_m=20)
    v, info = ctx.solve(f, tol=1e-10, maxit=500)
    res = krylov.gmres(wh.apply_A, wh.rhs(prob.gather(f)), op.m, tol=1e-10, maxit=500, restart=20)
    _say("gmres", dim, info["iters"], res.iters)
    assert res.converged and abs(info["iters"] - res.iters) <= 2, (info["iters"], res.iters)
    assert _rel(prob.gather(v.cpu().numpy()), res.x) <= 1e-8


def test_fp32_refinement_reaches_fp64_residual(E):
    """FP32 stepping + FP64 iterative refinement: the FP64-recomputed residual
    reaches 1e-8 and the solution matches the direct solve."""
    n, bc = (64, 64), (0, 0, 0, 1)
    rho, lam, mu = _media((65, 65), 71, 0.2)
    om = 12.0
    prob, op, wh = _oracle(2, n, None, bc, rho, lam, mu, om)
    rng = np.random.default_rng(13)
    f = inputs.gaussian_sources(2, n, (1.0, 1.0), [(0.4, 0.6)], [0.05], [(0.6, 0.8)])
    vstar = direct.solve(op, om, prob.gather(f))
    ctx = E.Context(2, n, rho, lam, mu, om, bc, prec=E.FP32_STEP)
    v, info = ctx.solve(f, tol=1e-10, maxit=2000)
    ctx64 = E.Context(2, n, rho, lam, mu, om, bc)
    v64, info64 = ctx64.solve(f, tol=1e-10, maxit=2000)
    err, err64 = _rel(prob.gather(v.cpu().numpy()), vstar), _rel(prob.gather(v64.cpu().numpy()), vstar)
    _say("fp32 reliable-update CG", info, "error", err, "| fp64 CG iterations", info64["iters"], "error", err64)
    assert info["relres_fp64"] <= 1e-10
    assert info["outer"] >= 2
    assert err <= 1e-6
    # FP32 stepping perturbs A_h by ~1e-7..1e-6 relative, which costs CG its
    # superlinear phase: about 2x the FP64 iterations at 1e-8 and 3x at
    # 1e-10 with the search direction kept across residual replacements
    assert info["iters"] <= 3.5 * info64["iters"] + 10


def test_rejects_bad_arguments(E):
    ok = np.ones((9, 9))
    bad = ok.copy()
    bad[2, 2] = np.inf
    with pytest.raises(E.ElwhError, match="ERR_ARG"):
        E.Context(2, (8, 8), bad, ok, ok, 3.0, (0, 0, 0, 0))
    with pytest.raises(E.ElwhError, match="ERR_ARG"):
        E.Context(2, (8, 8), ok, ok, ok, 3.0, (0, 1, 0, 0))
    with pytest.raises(E.ElwhError, match="ERR_ARG"):
        E.Context(2, (8, 8), ok, ok, ok, 0.0, (0, 0, 0, 0))


@pytest.mark.parametrize("prec", [0, 1])
def test_unstable_step_is_reported(E, prec):
    """A step count far below the stability limit (N_T = 6 where the rule
    gives 121) makes the solution grow by orders of magnitude per step; the
    first Rayleigh quotient (b, A_h b)_M / (b, b)_M then exceeds 4, which no
    stable step allows (|beta_h| <= 5/2), and the solver reports
    ELWH_ERR_UNSTABLE, alone and in a batch, instead of returning garbage."""
    c = inputs.constant_square64()
    ctx = E.Context(2, c.n, c.rho, c.lam, c.mu, c.omega, c.bc, nt=6, prec=prec)
    v, info = ctx.solve(c.f, tol=1e-10, maxit=50, raise_on_fail=False)
    assert info["status"] == "ERR_UNSTABLE"
    bt = E.Batch([c, inputs.constant_square64()], nt=6, prec=prec)
    _, infos, st = bt.solve([c.f, c.f], tol=1e-10, maxit=50)
    assert st == "ERR_UNSTABLE"


# ---------------------------------------------------------------- full size --

def test_square1024_full_size_fp64_and_fp32(E):
    """The 1024^2 random medium with a free top element by element against
    the oracle, in the launch configuration the benchmark times."""
    c = inputs.random_square()
    _say("1024^2 random medium, omega", c.omega)
    prob, op, wh = _oracle(2, c.n, None, c.bc, c.rho, c.lam, c.mu, c.omega)
    fv = prob.gather(c.f)
    u0 = inputs.gaussian_sources(2, c.n, (1.0, 1.0), [(0.3, 0.4), (0.7, 0.6)], [0.05, 0.03],
                                 [(1.0, 0.0), (0.0, 1.0)]) * prob.unknown_mask()
    ref = prob.scatter(wh.apply_filter(prob.gather(u0), fv))
    ctx = E.context_from_case(c)
    assert ctx.info()["nt"] == wh.nt
    got = ctx.apply_filter(u0, c.f).cpu().numpy()
    assert _rel(got, ref) <= FP64_TOL
    ctx32 = E.context_from_case(c, prec=E.FP32_STEP)
    err32 = _rel(ctx32.apply_filter(u0, c.f).cpu().numpy(), ref)
    _say("1024^2 fp32 rel err", err32, "bound", fp32_bound(wh.nt))
    assert err32 <= fp32_bound(wh.nt)


def test_cube256_full_size_fixed_point():
    """The 256^3 layered medium: the manufactured fixed point
    Pi_h v* = v* with f = omega^2 rho v* + Ltilde v* from the oracle's slice
    stencil, FP64 (<= 1e-12) and FP32 stepping (<= fp32_bound(N_T))."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_12344_amd import elwh as E
    from oracle.stencil import ltilde_dirichlet
    c = inputs.layered_cube()
    _say("256^3 layered medium, omega", c.omega)
    n = c.n[0]
    x = np.arange(n + 1) / n
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    bump = np.sin(np.pi * X) * np.sin(np.pi * Y) * np.sin(np.pi * Z)
    v = np.array([bump * np.sin(3 * np.pi * X), bump * np.cos(2 * np.pi * Y), bump * np.sin(5 * np.pi * Z)])
    del X, Y, Z
    f = c.omega ** 2 * c.rho[None] * v + ltilde_dirichlet(tuple(1.0 / m for m in c.n), c.lam, c.mu, v)
    ctx = E.context_from_case(c)
    got = ctx.apply_filter(v, f).cpu().numpy()
    err = _rel(got, v)
    _say("256^3 fp64 fixed point err", err)
    assert err <= FP64_TOL
    del ctx
    ctx32 = E.context_from_case(c, prec=E.FP32_STEP)
    err32 = _rel(ctx32.apply_filter(v, f).cpu().numpy(), v)
    nt = ctx32.info()["nt"]
    _say("256^3 fp32 fixed point err", err32, "bound", fp32_bound(nt))
    assert err32 <= fp32_bound(nt)


def test_large_sizes_fixed_point():
    """Sizes well beyond the benchmark's (4096^2 cells in 2-D, 16.8 M nodes;
    384^3 in 3-D, 57 M nodes): the manufactured fixed point Pi_h v* = v* of
    random and layered media with all faces Dirichlet, forcing from the
    oracle's slice stencil, in FP64 (<= 1e-11)."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_12344_amd import elwh as E
    from oracle.stencil import ltilde_dirichlet
    n = 4096
    h = 1.0 / n
    rho, lam, mu = inputs.media_random((n + 1, n + 1), (h, h), seed=21)
    om = 2 * math.pi * inputs.min_shear_speed(rho, mu) / (10 * h)
    x = np.arange(n + 1) / n
    Y, X = np.meshgrid(x, x, indexing="ij")
    bump = np.sin(np.pi * X) * np.sin(np.pi * Y)
    v = np.array([bump * np.sin(7 * np.pi * X + Y), bump * np.cos(5 * np.pi * Y)])
    del X, Y, bump
    f = om ** 2 * rho[None] * v + ltilde_dirichlet((h, h), lam, mu, v)
    _say("4096^2 fixed point, omega", om)
    ctx = E.Context(2, (n, n), rho, lam, mu, om, (0, 0, 0, 0))
    err = _rel(ctx.apply_filter(v, f).cpu().numpy(), v)
    _say("4096^2 fp64 fixed point err", err, "nt", ctx.info()["nt"])
    assert err <= 1e-11
    ctx.close()
    del ctx, v, f, rho, lam, mu
    c = inputs.layered_cube(n=384)
    m = c.n[0]
    x = np.arange(m + 1) / m
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    bump = np.sin(np.pi * X) * np.sin(np.pi * Y) * np.sin(np.pi * Z)
    v = np.array([bump * np.sin(3 * np.pi * X), bump * np.cos(2 * np.pi * Y), bump * np.sin(5 * np.pi * Z)])
    del X, Y, Z, bump
    f = c.omega ** 2 * c.rho[None] * v + ltilde_dirichlet(tuple(1.0 / k for k in c.n), c.lam, c.mu, v)
    _say("384^3 fixed point, omega", c.omega)
    ctx3 = E.context_from_case(c)
    err3 = _rel(ctx3.apply_filter(v, f).cpu().numpy(), v)
    _say("384^3 fp64 fixed point err", err3, "nt", ctx3.info()["nt"])
    assert err3 <= 1e-11


# ------------------------------------------------------------- tilings --------

def _tiles(dim, fp32, fuse=1):
    if dim == 2:
        vs = (1, 2, 4) if fp32 else (1, 2)
        return [(v, ty) for v in vs for ty in (4, 8, 16)] + [(1, 10), (1, 12)]
    if fuse >= 2:   # two-step 3-D launches: RB rows (plus two halo rows) x TZ planes;
        # RB 1 = single-step launches in a two-step context
        return [(rb, tz) for rb in (2, 4, 6) for tz in (8, 16, 32, 64)] + [(1, 16), (1, 32)]
    return [(rb, tz) for rb in (1, 2, 4, 8) for tz in (4, 8, 16, 32)]


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("prec", [0, 1])
def test_every_tiling_matches_oracle(E, dim, prec):
    """Every supported (nodes per lane, rows per wavefront) tiling of the
    fused step gives the oracle's result; grids ragged for every tiling."""
    if dim == 2:
        n, bc = (257, 45), (0, 0, 0, 1)
    else:
        n, bc = (67, 7, 41), (0, 0, 0, 0, 1, 1)
    shape = tuple(n[a] + 1 for a in reversed(range(dim)))
    rho, lam, mu = _media(shape, 90 + dim)
    om = 8.1
    prob, op, wh = _oracle(dim, n, None, bc, rho, lam, mu, om)
    rng = np.random.default_rng(14)
    u0 = rng.standard_normal(prob.field_shape) * prob.unknown_mask()
    f = rng.standard_normal(prob.field_shape) * prob.unknown_mask()
    ref = prob.scatter(wh.apply_filter(prob.gather(u0), prob.gather(f)))
    tol = FP64_TOL if prec == 0 else fp32_bound(wh.nt)
    outs = []
    for fuse in ((2, 1, 3, 4) if dim == 2 else (2, 1)):
        ctx = E.Context(dim, n, rho, lam, mu, om, bc, prec=prec, autotune=0, fuse=fuse)
        for v, rows in _tiles(dim, prec == 1, fuse):
            ctx.set_tile(prec, v, rows)
            got = ctx.apply_filter(u0, f).cpu().numpy()
            err = _rel(got, ref)
            _say("tile", dim, prec, "fuse", fuse, v, rows, err)
            assert err <= tol
            outs.append(got)
    # tilings differ only in how the compiler contracts multiply-adds
    for o in outs[1:]:
        assert _rel(o, outs[0]) <= (FP64_TOL if prec == 0 else 2 * fp32_bound(wh.nt))
    with pytest.raises(E.ElwhError, match="ERR_ARG"):
        ctx.set_tile(prec, 3, 8)


def test_autotune_choice_is_valid_and_cached(E):
    c = inputs.constant_square64()
    ctx = E.context_from_case(c, prec=E.FP32_STEP)
    v64, r64 = ctx.get_tile(0)
    v32, r32 = ctx.get_tile(1)
    assert (v64, r64) in _tiles(2, False) and (v32, r32) in _tiles(2, True)
    assert ctx.autotune(0) == -1.0          # cached per process


def test_autotune_cache_keeps_steps_per_launch_apart(E):
    """The tile cache is keyed by the steps per launch: a K = 3 context does
    not inherit the tile timed for single-step launches of the same grid."""
    c = inputs.random_problem_2d(200, 30.0, seed=41)
    E.context_from_case(c, fuse=1)                 # tunes and caches the K = 1 tile
    ctx3 = E.context_from_case(c, fuse=3, autotune=0)
    assert ctx3.autotune(0, reps=1) > 0.0           # not a cache hit: timed afresh
    assert ctx3.autotune(0) == -1.0


@pytest.mark.parametrize("K", [1, 2, 5])
def test_k_period_solve_matches_oracle(E, K):
    """K-period filter (eq. many_periods_filter) inside CG on the FD bar of
    the Table 3 analogue: the library's iteration count equals the oracle's
    (+-1) and the solutions agree."""
    n, length, bc = (128, 16), (8.0, 1.0), (0, 0, 1, 1)
    shape = (17, 129)
    rho, lam, mu = np.ones(shape), 2.0 * np.ones(shape), np.ones(shape)
    f = inputs.gaussian_sources(2, n, length, [(1.0, 0.5)], [0.25], [(1.0, 0.0)])
    prob, op, wh = _oracle(2, n, length, bc, rho, lam, mu, 5.123, periods=K)
    res = krylov.cg(wh.apply_A, wh.rhs(prob.gather(f)), op.m, tol=1e-10, maxit=2000)
    ctx = E.Context(2, n, rho, lam, mu, 5.123, bc, length=length, periods=K)
    v, info = ctx.solve(f, tol=1e-10, maxit=2000)
    _say("K periods", K, "iters", info["iters"], "oracle", res.iters)
    assert abs(info["iters"] - res.iters) <= 1
    assert _rel(prob.gather(v.cpu().numpy()), res.x) <= 1e-8


def test_cr_standard_scheme_point_source_matches_oracle(E):
    """The rectangle of the iterations-vs-omega experiment (5 x 1, standard
    scheme, discrete point source, conjugate residual to 1e-8) at
    omega = 8 + sqrt(2)/10: the library's CR takes the oracle's iteration
    count (+-1) and reaches its iterate."""
    w = 8 + math.sqrt(2) / 10
    n = (int(4 * 5 * w + 1), int(4 * w + 1))
    shape = (n[1] + 1, n[0] + 1)
    rho, lam, mu = np.ones(shape), 2.0 * np.ones(shape), np.ones(shape)
    prob, op, wh = _oracle(2, n, (5.0, 1.0), (0, 0, 0, 0), rho, lam, mu, w, scheme=S.STANDARD)
    f = np.zeros(prob.field_shape)
    f[0, n[1] // 2, n[0] // 10] = w * w / ((5.0 / n[0]) * (1.0 / n[1]))
    res = krylov.cr(wh.apply_A, wh.rhs(prob.gather(f)), op.m, tol=1e-8, maxit=3000)
    ctx = E.Context(2, n, rho, lam, mu, w, (0, 0, 0, 0), length=(5.0, 1.0), scheme=1, krylov=2)
    v, info = ctx.solve(f, tol=1e-8, maxit=3000)
    _say("CR point source: iters", info["iters"], "oracle", res.iters)
    assert abs(info["iters"] - res.iters) <= 1
    assert _rel(prob.gather(v.cpu().numpy()), res.x) <= 1e-7
