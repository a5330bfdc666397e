"""GPU parity on mapped (curvilinear) 2-D grids: the HIP path through the C ABI
(elwh_create_mapped) against the CPU FP64 oracle (oracle/curvilinear.py) on
the same seeded inputs -- quarter and half annular sectors (Sec. 5.5) and a
strongly non-orthogonal warped square.

Bars as in test_gpu_parity.py: FP64 rel-L2 <= 1e-12 per application, FP32
stepping <= fp32_bound(N_T); solves to their stated residuals."""

import math
import sys

import numpy as np
import pytest

from oracle import direct, krylov
from oracle import stepping as S
from oracle.curvilinear import MappedOperator, lh_stencil, metric
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


def _rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def _grid(kind, nq, nr, seed=0):
    if kind == "quarter":
        return inputs.sector_grid(nq, nr, 1)
    if kind == "half":
        return inputs.sector_grid(nq, nr, 2)
    return inputs.warped_grid(nq, nr, seed=seed)


def _interior(shape):
    m = np.zeros(shape)
    m[1:-1, 1:-1] = 1.0
    return m


# ragged in q (62 / 126 computed columns per wavefront) and in r (8 / 16 rows)
CASES = [("quarter", 70, 45), ("half", 130, 37), ("warped", 63, 17), ("warped", 2, 30), ("quarter", 40, 2)]


@pytest.mark.parametrize("kind,nq,nr", CASES)
@pytest.mark.parametrize("force", [False, True])
def test_mapped_filter_fp64(E, kind, nq, nr, force):
    _say("mapped filter fp64", kind, nq, nr, force)
    x, y = _grid(kind, nq, nr, seed=nq)
    rho, lam, mu = inputs.media_mapped(x, y, seed=nq + nr)
    om = 7.3
    op = MappedOperator(x, y, rho, lam, mu)
    wh = S.WaveHoltz(op, om)
    prob = op.prob
    rng = np.random.default_rng(3)
    mask = _interior(x.shape)
    u0 = rng.standard_normal(prob.field_shape) * mask
    f = rng.standard_normal(prob.field_shape) * mask if force else None
    ref = prob.scatter(wh.apply_filter(prob.gather(u0), prob.gather(f) if force else None))
    refA = prob.scatter(wh.apply_A(prob.gather(u0)))
    ctx = E.MappedContext(x, y, rho, lam, mu, om)
    assert ctx.info()["nt"] == wh.nt
    for V, TY in ((1, 8), (1, 16), (2, 8), (2, 16)):
        ctx.set_tile(0, V, TY)
        got = ctx.apply_filter(u0, f).cpu().numpy()
        assert _rel(got, ref) <= FP64_TOL, (V, TY)
        assert np.all(got[:, 0, :] == 0) and np.all(got[:, :, -1] == 0)
        gotA = ctx.apply_A(u0).cpu().numpy()
        assert _rel(gotA, refA) <= FP64_TOL, (V, TY)


def test_mapped_filter_fp32(E):
    x, y = _grid("quarter", 90, 200)
    rho, lam, mu = inputs.media_mapped(x, y, seed=4)
    om = 9.0
    op = MappedOperator(x, y, rho, lam, mu)
    wh = S.WaveHoltz(op, om)
    prob = op.prob
    rng = np.random.default_rng(5)
    mask = _interior(x.shape)
    u0 = rng.standard_normal(prob.field_shape) * mask
    f = rng.standard_normal(prob.field_shape) * mask
    ref = prob.scatter(wh.apply_filter(prob.gather(u0), prob.gather(f)))
    for comp in (1, 0):
        ctx = E.MappedContext(x, y, rho, lam, mu, om, prec=E.FP32_STEP, compensated=comp)
        for V, TY in ((1, 8), (2, 16)):
            ctx.set_tile(1, V, TY)
            err = _rel(ctx.apply_filter(u0, f).cpu().numpy(), ref)
            _say("mapped fp32 compensated", comp, (V, TY), "nt", wh.nt, "err", err, "bound", fp32_bound(wh.nt))
            assert err <= fp32_bound(wh.nt)


def test_mapped_dot_M_and_k_periods(E):
    x, y = _grid("half", 30, 60)
    rho, lam, mu = inputs.media_mapped(x, y, seed=6)
    op = MappedOperator(x, y, rho, lam, mu)
    prob = op.prob
    rng = np.random.default_rng(7)
    mask = _interior(x.shape)
    a = rng.standard_normal(prob.field_shape) * mask
    b = rng.standard_normal(prob.field_shape) * mask
    ctx = E.MappedContext(x, y, rho, lam, mu, 5.0, periods=3, scheme=1)
    ref = float(np.dot(op.m * prob.gather(a), prob.gather(b)))
    assert ctx.dot_M(a, b) == pytest.approx(ref, rel=1e-13)
    wh = S.WaveHoltz(op, 5.0, periods=3, scheme=S.STANDARD)
    got = ctx.apply_filter(a, b).cpu().numpy()
    assert _rel(got, prob.scatter(wh.apply_filter(prob.gather(a), prob.gather(b)))) <= FP64_TOL


def test_mapped_solve_matches_direct_and_oracle_cg(E):
    x, y = _grid("quarter", 24, 110)
    rho, lam, mu = inputs.media_mapped(x, y, seed=8)
    om = 4.1
    op = MappedOperator(x, y, rho, lam, mu)
    wh = S.WaveHoltz(op, om)
    prob = op.prob
    f = np.zeros(prob.field_shape)
    f[0, 50, 12] = 1.0 / (op.J[50, 12] / (24 * 110))
    f[1, 70, 8] = 0.5 / (op.J[70, 8] / (24 * 110))
    fv = prob.gather(f)
    vstar = direct.solve(op, om, fv)
    res = krylov.cg(wh.apply_A, wh.rhs(fv), op.m, tol=1e-10, maxit=3000)
    ctx = E.MappedContext(x, y, rho, lam, mu, om)
    v, info = ctx.solve(f, tol=1e-10, maxit=3000)
    _say("mapped solve", info, "oracle iters", res.iters, res.converged)
    assert info["relres_fp64"] <= 1e-10
    assert abs(info["iters"] - res.iters) <= 1
    assert _rel(prob.gather(v.cpu().numpy()), vstar) <= 1e-8


@pytest.mark.parametrize("geometry", ["quarter", "half"])
def test_mapped_cr_point_source_matches_oracle(E, geometry):
    """The annular sectors of the iterations-vs-omega experiment at
    omega = 6 + sqrt(2)/10 (standard scheme, point source, CR to 1e-8): the
    library takes the oracle's count (+-1) and reaches its iterate."""
    w = 6 + math.sqrt(2) / 10
    nq, nr = int(4 * w + 1), int(4 * 5 * w + 1)
    x, y = _grid(geometry, nq, nr)
    one = np.ones(x.shape)
    op = MappedOperator(x, y, one, 2 * one, one)
    wh = S.WaveHoltz(op, w, scheme=S.STANDARD)
    prob = op.prob
    f = np.zeros(prob.field_shape)
    i = (nq + 1) // 2
    f[0, i, i] = w * w / (op.J[i, i] / (nq * nr))
    res = krylov.cr(wh.apply_A, wh.rhs(prob.gather(f)), op.m, tol=1e-8, maxit=3000)
    ctx = E.MappedContext(x, y, one, 2 * one, one, w, scheme=1, krylov=2)
    v, info = ctx.solve(f, tol=1e-8, maxit=3000)
    _say("mapped CR", geometry, "iters", info["iters"], "oracle", res.iters)
    assert abs(info["iters"] - res.iters) <= 1
    assert _rel(prob.gather(v.cpu().numpy()), res.x) <= 1e-7


def test_mapped_full_size_fixed_point(E):
    """The benchmark's mapped workload (quarter annulus of Sec. 5.5 at
    omega = 200 + sqrt(2)/10: 801 x 4003 cells, random media) in the launch
    configuration it times: with the forcing of a discrete manufactured v*
    (f = omega^2 rho v* + J^-1 L_h v*, from the oracle's stencil form) the
    filter returns v* (a property of the exact operator at any size), in FP64
    and in FP32 stepping."""
    x, y, rho, lam, mu, om, _ = inputs.sector_case(200, 1, seed=14)
    nr, nq = x.shape[0] - 1, x.shape[1] - 1
    J, _, _ = metric(x, y, 1.0 / nq, 1.0 / nr)
    rng = np.random.default_rng(13)
    Q, R = np.meshgrid(np.arange(nq + 1) / nq, np.arange(nr + 1) / nr)
    bump = np.sin(np.pi * Q) * np.sin(np.pi * R)          # zero on the boundary
    vsm = np.stack([np.sin(3 * x) * np.cos(2 * y), np.cos(x + y)]) * bump
    vs = vsm.copy()
    vs[:, 1:-1, 1:-1] += 0.1 * rng.standard_normal((2, nr - 1, nq - 1))
    f = (om ** 2 * rho * vs + lh_stencil(x, y, lam, mu, vs) / J) * _interior(x.shape)
    ctx = E.MappedContext(x, y, rho, lam, mu, om)
    nt = ctx.info()["nt"]
    _say("mapped full size: cells", (nq, nr), "nt", nt, "omega", om)
    got = ctx.apply_filter(vs, f).cpu().numpy()
    err = _rel(got, vs)
    _say("  fp64 fixed-point error", err)
    assert err <= 1e-11
    # FP32 stepping on a smooth v* (white noise would add rounding of the
    # stencil sums that the per-step bound does not model)
    fsm = (om ** 2 * rho * vsm + lh_stencil(x, y, lam, mu, vsm) / J) * _interior(x.shape)
    got32 = E.MappedContext(x, y, rho, lam, mu, om, prec=E.FP32_STEP).apply_filter(vsm, fsm).cpu().numpy()
    err32 = _rel(got32, vsm)
    _say("  fp32 fixed-point error", err32, "bound", fp32_bound(nt))
    assert err32 <= fp32_bound(nt)


def test_mapped_rejects_bad_arguments(E):
    x, y = _grid("quarter", 10, 20)
    one = np.ones(x.shape)
    with pytest.raises(E.ElwhError, match="J > 0"):
        E.MappedContext(x[:, ::-1].copy(), y[:, ::-1].copy(), one, one, one, 3.0)
    with pytest.raises(ValueError):
        E.MappedContext(x, y[:-1], one, one, one, 3.0)
    ctx = E.MappedContext(x, y, one, one, one, 3.0)
    with pytest.raises(E.ElwhError, match="ERR_ARG"):
        ctx.set_tile(0, 4, 8)


# ---- traction-free r sides ------------------------------------------------------

FREE_CASES = [("ring", 70, 21, (0, 0, 1, 1)), ("ring", 130, 16, (0, 0, 0, 1)), ("warped", 63, 17, (0, 0, 1, 0)),
              ("quarter", 40, 33, (0, 0, 1, 1)), ("ring", 5, 2, (0, 0, 1, 1))]


def _grid_bc(kind, nq, nr, seed=0):
    if kind == "ring":
        return inputs.ring_grid(nq, nr)
    return _grid(kind, nq, nr, seed)


@pytest.mark.parametrize("kind,nq,nr,bc", FREE_CASES)
@pytest.mark.parametrize("force", [False, True])
def test_mapped_free_sides_filter_fp64(E, kind, nq, nr, bc, force):
    _say("mapped free filter fp64", kind, nq, nr, bc, force)
    x, y = _grid_bc(kind, nq, nr, seed=nq)
    rho, lam, mu = inputs.media_mapped(x, y, seed=nq + 2 * nr)
    om = 6.3
    op = MappedOperator(x, y, rho, lam, mu, bc=bc)
    wh = S.WaveHoltz(op, om)
    prob = op.prob
    rng = np.random.default_rng(17)
    mask = prob.unknown_mask()
    u0 = rng.standard_normal(prob.field_shape) * mask
    f = rng.standard_normal(prob.field_shape) * mask if force else None
    ref = prob.scatter(wh.apply_filter(prob.gather(u0), prob.gather(f) if force else None))
    refA = prob.scatter(wh.apply_A(prob.gather(u0)))
    ctx = E.MappedContext(x, y, rho, lam, mu, om, bc=bc)
    assert ctx.info()["nt"] == wh.nt
    for V, TY in ((1, 8), (1, 16), (2, 8), (2, 16)):
        ctx.set_tile(0, V, TY)
        got = ctx.apply_filter(u0, f).cpu().numpy()
        assert _rel(got, ref) <= FP64_TOL, (V, TY)
        assert _rel(ctx.apply_A(u0).cpu().numpy(), refA) <= FP64_TOL, (V, TY)
    a = rng.standard_normal(prob.field_shape) * mask
    assert ctx.dot_M(a, u0) == pytest.approx(float(np.dot(op.m * prob.gather(a), prob.gather(u0))), rel=1e-13)


def test_mapped_free_sides_fp32(E):
    x, y = inputs.ring_grid(150, 50)
    rho, lam, mu = inputs.media_mapped(x, y, seed=31)
    bc = (0, 0, 1, 1)
    om = 8.0
    op = MappedOperator(x, y, rho, lam, mu, bc=bc)
    wh = S.WaveHoltz(op, om)
    prob = op.prob
    rng = np.random.default_rng(32)
    u0 = rng.standard_normal(prob.field_shape) * prob.unknown_mask()
    f = rng.standard_normal(prob.field_shape) * prob.unknown_mask()
    ref = prob.scatter(wh.apply_filter(prob.gather(u0), prob.gather(f)))
    for comp in (1, 0):
        ctx = E.MappedContext(x, y, rho, lam, mu, om, bc=bc, prec=E.FP32_STEP, compensated=comp)
        err = _rel(ctx.apply_filter(u0, f).cpu().numpy(), ref)
        _say("mapped free fp32 compensated", comp, "nt", wh.nt, "err", err, "bound", fp32_bound(wh.nt))
        assert err <= fp32_bound(wh.nt)


def test_ring_sector_with_free_arcs_cr_matches_oracle(E):
    """A 2-D analogue of the toroidal shell of Sec. 5.11: the ring sector
    1 <= radius <= 2, 0 <= angle <= pi with traction-free inner and outer arcs
    and Dirichlet cuts, the paper's forcing form (sqrt(sigma^3)/20) (1, 1)
    exp(-zeta^2), sigma = 100 omega, at omega = 5.1234, conjugate residual to
    1e-5 as in that experiment: the library's count equals the oracle's (+-1)
    and its iterate matches."""
    w = 5.1234
    x, y = inputs.ring_grid(120, 40)
    one = np.ones(x.shape)
    rho, lam, mu = one, 2 * one, one
    bc = (0, 0, 1, 1)
    op = MappedOperator(x, y, rho, lam, mu, bc=bc)
    wh = S.WaveHoltz(op, w)
    prob = op.prob
    sigma = 100 * w
    zeta2 = 0.5 * sigma * ((x + 0.4) ** 2 + (y - 1.3) ** 2)
    amp = math.sqrt(sigma ** 3) / 20 * np.exp(-zeta2)
    f = np.stack([amp, amp]) * prob.unknown_mask()
    res = krylov.cr(wh.apply_A, wh.rhs(prob.gather(f)), op.m, tol=1e-5, maxit=5000)
    ctx = E.MappedContext(x, y, rho, lam, mu, w, bc=bc, krylov=2)
    v, info = ctx.solve(f, tol=1e-5, maxit=5000)
    _say("ring with free arcs, CR: iters", info["iters"], "oracle", res.iters, "nt", wh.nt)
    assert res.converged and abs(info["iters"] - res.iters) <= 1
    assert _rel(prob.gather(v.cpu().numpy()), res.x) <= 1e-4
    # CG to 1e-10 reaches the direct solution
    ctx_cg = E.MappedContext(x, y, rho, lam, mu, w, bc=bc)
    v2, info2 = ctx_cg.solve(f, tol=1e-10, maxit=5000)
    vstar = direct.solve(op, w, prob.gather(f))
    _say("ring with free arcs, CG: iters", info2["iters"], "cr", info2.get("cr_iters"))
    assert _rel(prob.gather(v2.cpu().numpy()), vstar) <= 1e-7


def test_mapped_fp32_solve_reaches_fp64_residual(E):
    """FP32 stepping on a mapped grid: CG with FP32 applications and FP64
    residual replacement reaches an FP64-recomputed residual of 1e-10 and the
    direct solution."""
    x, y = inputs.ring_grid(90, 30)
    rho, lam, mu = inputs.media_mapped(x, y, seed=51)
    bc = (0, 0, 1, 1)
    om = 4.3
    op = MappedOperator(x, y, rho, lam, mu, bc=bc)
    prob = op.prob
    f = np.zeros(prob.field_shape)
    f[0, 15, 40] = 1.0 / (op.J[15, 40] / (90 * 30))
    vstar = direct.solve(op, om, prob.gather(f))
    ctx64 = E.MappedContext(x, y, rho, lam, mu, om, bc=bc)
    _, i64 = ctx64.solve(f, tol=1e-10, maxit=4000)
    ctx = E.MappedContext(x, y, rho, lam, mu, om, bc=bc, prec=E.FP32_STEP)
    v, info = ctx.solve(f, tol=1e-10, maxit=4000)
    _say("mapped fp32 solve", info, "fp64 iters", i64["iters"])
    assert info["relres_fp64"] <= 1e-10
    assert _rel(prob.gather(v.cpu().numpy()), vstar) <= 1e-7
    assert info["iters"] <= 3.5 * i64["iters"] + 10


@pytest.mark.parametrize("K", [1, 3])
def test_mapped_k_period_cg_matches_oracle(E, K):
    x, y = _grid("half", 20, 60)
    rho, lam, mu = inputs.media_mapped(x, y, seed=52)
    om = 3.7
    op = MappedOperator(x, y, rho, lam, mu)
    wh = S.WaveHoltz(op, om, periods=K)
    prob = op.prob
    f = np.zeros(prob.field_shape)
    f[1, 30, 10] = 1.0 / (op.J[30, 10] / (20 * 60))
    res = krylov.cg(wh.apply_A, wh.rhs(prob.gather(f)), op.m, tol=1e-10, maxit=3000)
    ctx = E.MappedContext(x, y, rho, lam, mu, om, periods=K)
    v, info = ctx.solve(f, tol=1e-10, maxit=3000)
    _say("mapped K-period CG", K, "iters", info["iters"], "oracle", res.iters)
    assert abs(info["iters"] - res.iters) <= 1
    assert _rel(prob.gather(v.cpu().numpy()), res.x) <= 1e-8
