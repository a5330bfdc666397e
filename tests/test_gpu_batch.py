"""GPU tests of the ragged batch (one launch per step for many problems of
different size, omega and N_T; device-side CG per problem; hipGraph replay)."""

import sys

import numpy as np
import pytest

from oracle import direct, krylov
from oracle import stepping as S
from oracle.operator import Operator
from oracle.problem import Problem
from paper_2205_12344_amd import inputs

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-batch]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def E():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_12344_amd import elwh
    return elwh


def _cases():
    # (N_T - 1) mod 4 = 0, 1, 1, 1, 2, 0, 3: every remainder of a four-step tick
    spec = [(24, 6.0), (40, 9.5), (33, 4.2), (50, 12.0), (29, 7.7), (64, 15.0), (36, 7.9)]
    return [inputs.random_problem_2d(n, om, seed=200 + k) for k, (n, om) in enumerate(spec)]


def _direct(c):
    prob = Problem(2, c.n, bc=c.bc)
    op = Operator(prob, c.rho, c.lam, c.mu)
    return prob, op, direct.solve(op, c.omega, prob.gather(c.f))


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _fp32_bound(nt):
    """The FP32-stepping bound of one filter application (as in the parity
    tests): one rounding per step, a random walk over N_T steps amplified by
    N_T / (2 pi), twice, plus the rounding of the inputs."""
    u32 = 2.0 ** -24
    return 2.0 * u32 * np.sqrt(nt) * nt / (2 * np.pi) + 8.0 * u32


@pytest.mark.parametrize("fuse", [4, 2, 1])
def test_batch_fp64_matches_direct_and_oracle_cg(E, fuse):
    """Four-step ticks (the default), two-step ticks and single steps; the
    problems' N_T leave every remainder of the tick length."""
    cases = _cases()
    bt = E.Batch(cases, fuse=fuse)
    _say("tiles", fuse, bt.stats())
    vs, infos, status = bt.solve([c.f for c in cases], tol=1e-10, maxit=500)
    assert status == "OK"
    for c, v, info in zip(cases, vs, infos):
        prob, op, vstar = _direct(c)
        got = prob.gather(v.cpu().numpy())
        wh = S.WaveHoltz(op, c.omega)
        res = krylov.cg(wh.apply_A, wh.rhs(prob.gather(c.f)), op.m, tol=1e-10, maxit=500)
        _say(c.name, info["iters"], res.iters, info["relres_fp64"], _rel(got, vstar))
        assert info["nt"] == wh.nt
        assert abs(info["iters"] - res.iters) <= 1
        assert info["relres_fp64"] <= 1e-10
        assert _rel(got, vstar) <= 1e-8
        assert _rel(got, res.x) <= 1e-8


def test_batch_graph_replay_equals_eager(E):
    """The captured hipGraph of batched steps, replayed many times with host
    synchronisations in between, gives exactly the eager launches' result."""
    cases = _cases()[:4]
    bt = E.Batch(cases)
    f = [c.f for c in cases]
    v1, i1, s1 = bt.solve(f, tol=1e-9, maxit=300)
    v2, i2, s2 = bt.solve(f, tol=1e-9, maxit=300)
    bt.set_graph(False)
    v3, i3, s3 = bt.solve(f, tol=1e-9, maxit=300)
    assert s1 == s2 == s3 == "OK"
    for a, b, c in zip(v1, v2, v3):
        assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())
        assert np.array_equal(a.cpu().numpy(), c.cpu().numpy())
    assert [x["iters"] for x in i1] == [x["iters"] for x in i3]


def test_batch_warm_start_and_fixed_iterations(E):
    cases = _cases()[:3]
    bt = E.Batch(cases)
    f = [c.f for c in cases]
    v, info, st = bt.solve(f, tol=0.0, maxit=7)
    assert st == "OK" and all(x["iters"] == 7 for x in info)
    v2, info2, st2 = bt.solve(f, x0s=v, tol=1e-10, maxit=500)
    assert st2 == "OK"
    for c, x in zip(cases, v2):
        prob, op, vstar = _direct(c)
        assert _rel(prob.gather(x.cpu().numpy()), vstar) <= 1e-8


def test_batch_fp32_refinement(E):
    cases = _cases()
    bt = E.Batch(cases, prec=E.FP32_STEP)
    vs, infos, status = bt.solve([c.f for c in cases], tol=1e-8, maxit=2000)
    _say("fp32 batch", status, [(i["iters"], i["outer"], i["relres_fp64"]) for i in infos], bt.stats())
    assert status == "OK"
    for c, v, info in zip(cases, vs, infos):
        prob, op, vstar = _direct(c)
        assert info["relres_fp64"] <= 1e-8
        assert _rel(prob.gather(v.cpu().numpy()), vstar) <= 1e-6


@pytest.mark.parametrize("prec", [0, 1])
def test_scaled_warm_start(E, prec):
    """scale_x0: a start along the solution but 7x too large is rescaled to
    (almost) the solution, so CG stops at once; a start of pure noise is
    scaled towards zero and never costs more than one iteration over the
    zero start (the A_h-norm error of alpha x0 is at most that of 0)."""
    import torch
    cases = _cases()[:4]
    f = [c.f for c in cases]
    tol = 1e-8
    bt = E.Batch(cases, prec=prec, scale_x0=1)
    ref = E.Batch(cases, prec=prec)
    _, i0, s0 = ref.solve(f, tol=tol, maxit=2000)
    vstar = []
    for c in cases:
        prob, op, v = _direct(c)
        vstar.append(prob.scatter(v))
    x_big = [torch.from_numpy(7.0 * v).cuda() for v in vstar]
    v1, i1, s1 = bt.solve(f, x0s=x_big, tol=tol, maxit=2000)
    _say("scaled start along v*", [x["iters"] for x in i1], "zero start", [x["iters"] for x in i0])
    assert s0 == s1 == "OK"
    for x in i1:
        assert x["iters"] <= 2
    rng = np.random.default_rng(5)
    x_noise = [torch.from_numpy(rng.standard_normal(v.shape) * np.abs(v).max()).cuda() for v in vstar]
    v2, i2, s2 = bt.solve(f, x0s=x_noise, tol=tol, maxit=2000)
    _say("scaled noise start", [x["iters"] for x in i2])
    assert s2 == "OK"
    for a, z in zip(i2, i0):
        assert a["iters"] <= z["iters"] + (1 if prec == 0 else 0.2 * z["iters"] + 5)
    for c, x in zip(cases, v2):
        prob, op, vs = _direct(c)
        assert _rel(prob.gather(x.cpu().numpy()), vs) <= 1e-6


def test_ragged_batch48_full_size_matches_single_contexts(E):
    """The ragged batch at full size (48 problems, 256^2..1024^2 cells, omega in
    [10, 80], N_T up to ~3000) in one batch: two CG iterations of every
    problem equal those of the single-problem path (itself pinned to the
    oracle), which runs other kernels (K-step launches); and one iteration
    of two of its problems equals the oracle's, in FP64 and FP32."""
    cases = inputs.ragged_batch()
    bt = E.Batch(cases)
    _say("ragged batch tiles", bt.stats())
    vs, infos, st = bt.solve([c.f for c in cases], tol=0.0, maxit=2)
    assert st == "OK"
    worst = 0.0
    for c, v, info in zip(cases, vs, infos):
        ctx = E.context_from_case(c, autotune=0)
        assert ctx.info()["nt"] == info["nt"]
        ctx.cg_begin(c.f)
        ctx.cg_iterate(2)
        v1, _ = ctx.cg_result()
        worst = max(worst, _rel(v.cpu().numpy(), v1.cpu().numpy()))
        ctx.close()
    _say("ragged batch: worst rel diff batch vs single", worst)
    assert worst <= 1e-12
    # The oracle at full size, in the same batch launch (all 48 problems):
    # one CG iteration from zero is x1 = alpha0 b with b = Pi_h f and
    # alpha0 = (b, b)_M / (b, A_h b)_M.  Checked on the largest grid among
    # the problems with omega >= 50 (1002^2; the oracle's cost grows like
    # n^3 / omega) and on the longest period (N_T) among grids up to 400^2,
    # FP64 and FP32
    # stepping (FP32: alpha0 carries the FP32 error of one application of
    # A_h, relative to the Rayleigh quotient (b, A_h b)_M / (b, b)_M).
    nts = [i["nt"] for i in infos]
    sel = [max((p for p in range(len(cases)) if cases[p].omega >= 50.0), key=lambda p: cases[p].n[0]),
           max((p for p in range(len(cases)) if cases[p].n[0] <= 400), key=lambda p: nts[p])]
    refs = {}
    for p in sel:
        c = cases[p]
        prob = Problem(2, c.n, bc=c.bc)
        op = Operator(prob, c.rho, c.lam, c.mu)
        wh = S.WaveHoltz(op, c.omega)
        assert wh.nt == nts[p]
        b = wh.rhs(prob.gather(c.f))
        Ab = wh.apply_A(b)
        bb, bAb = float(np.dot(op.m * b, b)), float(np.dot(op.m * b, Ab))
        refs[p] = (prob, (bb / bAb) * b, bAb / bb)
    for prec in (E.FP64, E.FP32_STEP):
        bt1 = bt if prec == E.FP64 else E.Batch(cases, prec=prec)
        v1s, _, st1 = bt1.solve([c.f for c in cases], tol=0.0, maxit=1)
        assert st1 == "OK"
        for p in sel:
            prob, ref, rq = refs[p]
            err = _rel(prob.gather(v1s[p].cpu().numpy()), ref)
            tol = 1e-11 if prec == E.FP64 else 2.0 * _fp32_bound(nts[p]) / rq
            _say("ragged batch vs oracle", "fp64" if prec == E.FP64 else "fp32", "n", cases[p].n, "nt", nts[p],
                 "rayleigh", rq, "err", err, "tol", tol)
            assert err <= tol
        if bt1 is not bt:
            bt1.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_cr_fallback_after_cg_breakdown(E, prec):
    """A near-resonant warm-start problem (seed 4115, coarsened to
    64^2: omega = 59.0, N_T = 31) makes A_h slightly indefinite and CG break
    down (the oracle's CG does too); with cr_fallback the solve continues with
    conjugate residual in FP64 and reaches the residual target, alone and in
    a batch with other problems.  The system is nearly singular (a mode
    within ~1e-5 of resonance), so a residual of 1e-8 bounds the error only
    to ~1e-4 (the oracle's CR from zero happens to land at 2e-7); the check
    on the solution is accordingly |v - v*| / |v*| <= 1e-3."""
    c = inputs.warmstart_problem(4115, n=64)
    prob, op, vstar = _direct(c)
    with pytest.raises(E.ElwhError, match="BREAKDOWN"):
        E.context_from_case(c, prec=prec, cr_fallback=0).solve(c.f, tol=1e-8, maxit=3000)
    v, info = E.context_from_case(c, prec=prec).solve(c.f, tol=1e-8, maxit=3000)
    _say("single: cg iters", info["iters"], "cr iters", info["cr_iters"], "relres", info["relres_fp64"])
    assert info["cr_iters"] > 0 and info["relres_fp64"] <= 1e-8
    assert _rel(prob.gather(v.cpu().numpy()), vstar) <= 1e-3
    cases = [c] + [inputs.warmstart_problem(s, n=64) for s in (4099, 4096)]
    bt = E.Batch(cases, prec=prec)
    vs, infos, st = bt.solve([x.f for x in cases], tol=1e-8, maxit=3000)
    _say("batch:", st, [(i["iters"], i["cr_iters"], i["relres_fp64"]) for i in infos])
    assert st == "OK"
    assert infos[0]["cr_iters"] > 0
    for x, vv, info in zip(cases, vs, infos):
        prob, op, vs_ = _direct(x)
        assert info["relres_fp64"] <= 1e-8
        assert _rel(prob.gather(vv.cpu().numpy()), vs_) <= 1e-3


def test_fp32_stagnation_falls_back_to_fp64(E):
    """Warm-start problems (256^2, seeds 4096 and 4112) on which CG with FP32
    applications stalls: with the guard off the FP32 batch stops short of
    1e-8 at the iteration cap; with it (default) each problem switches to
    FP64 CG from its iterate and reaches 1e-8, alone and batched, and the
    solution equals the FP64 one."""
    cases = [inputs.warmstart_problem(s) for s in (4096, 4112)]
    fs = [c.f for c in cases]
    ref = E.Batch(cases)
    v64, i64, st64 = ref.solve(fs, tol=1e-8, maxit=3000)
    assert st64 == "OK"
    off = E.Batch(cases, prec=E.FP32_STEP, fp64_fallback=0)
    _, ioff, stoff = off.solve(fs, tol=1e-8, maxit=1500)
    _say("fp32 without fallback", stoff, [(i["iters"], i["relres_fp64"]) for i in ioff])
    assert stoff == "ERR_NOT_CONVERGED"
    on = E.Batch(cases, prec=E.FP32_STEP)
    v, infos, st = on.solve(fs, tol=1e-8, maxit=3000)
    _say("fp32 with fallback", st, [(i["iters"], i["fp64_iters"], i["relres_fp64"]) for i in infos])
    assert st == "OK"
    for a, b, info in zip(v, v64, infos):
        assert info["fp64_iters"] > 0 and info["relres_fp64"] <= 1e-8
        assert _rel(a.cpu().numpy(), b.cpu().numpy()) <= 1e-6
    c = cases[0]
    ctx = E.context_from_case(c, prec=E.FP32_STEP)
    vs, info = ctx.solve(c.f, tol=1e-8, maxit=3000)
    _say("single context fp32 with fallback", info)
    assert info["fp64_iters"] > 0 and info["relres_fp64"] <= 1e-8
    assert _rel(vs.cpu().numpy(), v64[0].cpu().numpy()) <= 1e-6


def test_fp64_first_then_fp32_reaches_the_fp64_solution(E):
    """opts.fp32_switch: FP64 CG down to a relative residual of 1e-3, then FP32
    segments continuing the same Krylov sequence (the relaxed-accuracy order:
    the FP32 perturbation of A_h is admitted only where the residual is small
    enough for it).  Batched and single-context solves of two warm-start
    problems reach the FP64 residual 1e-8, with iterations in both phases, and
    a solution within cond(A_h) x 2e-8 of the FP64 one (two solutions with
    residual 1e-8 can differ by that much; cond from the Lanczos estimate of
    FP64 CG).  (They take more iterations than FP64 CG: on these
    near-resonant problems the smallest eigenvalue of A_h is below the FP32
    perturbation of one application, so the admissible-perturbation bound,
    which scales with it, is not met even at small residuals.)"""
    cases = [inputs.warmstart_problem(s) for s in (4096, 4112)]
    fs = [c.f for c in cases]
    v64, i64, st64 = E.Batch(cases).solve(fs, tol=1e-8, maxit=3000)
    assert st64 == "OK"
    conds = []
    for c in cases:
        _, i1 = E.context_from_case(c).solve(c.f, tol=1e-8, maxit=3000)
        conds.append(i1["cond_est"])
    _say("cond_est", conds)
    for comp in (1, 0):
        bt = E.Batch(cases, prec=E.FP32_STEP, fp32_switch=1e-3, compensated=comp)
        v, infos, st = bt.solve(fs, tol=1e-8, maxit=4000)
        _say("fp64 then fp32, compensated", comp, st,
             [(i["iters"], i["fp64_iters"], i["outer"], i["relres_fp64"]) for i in infos], "fp64", [i["iters"] for i in i64])
        assert st == "OK"
        for a, b, info, cond in zip(v, v64, infos, conds):
            assert info["relres_fp64"] <= 1e-8
            assert 0 < info["fp64_iters"] < info["iters"]
            assert _rel(a.cpu().numpy(), b.cpu().numpy()) <= 2e-8 * cond
    c = cases[0]
    ctx = E.context_from_case(c, prec=E.FP32_STEP, fp32_switch=1e-3)
    vs, info = ctx.solve(c.f, tol=1e-8, maxit=4000)
    _say("single context fp64 then fp32", info)
    assert info["relres_fp64"] <= 1e-8 and 0 < info["fp64_iters"] < info["iters"]
    assert _rel(vs.cpu().numpy(), v64[0].cpu().numpy()) <= 2e-8 * conds[0]
