"""Pins of the mapped-grid oracle (curvilinear finite differences, Sec. 4.1;
the annular sectors of Sec. 5.5).

Each pin ties oracle/curvilinear.py to something other than itself:
* the Cartesian operator (independently pinned) for a scaled identity map;
* exact rotation equivariance of the continuous operator, kept by the
  discrete one;
* symmetry, definiteness and the energy identity;
* the stencil form against the energy Hessian;
* second-order truncation error and second-order convergence of the
  Helmholtz solution against a continuous manufactured solution, whose
  stress divergence comes from exact jets (themselves checked against
  finite differences);
* the paper's observation that iteration counts on the quarter and half
  annulus are very close to the rectangle's (Sec. 5.5).
"""

import math

import numpy as np
import pytest

import jets
from jets import Jet
from oracle import direct, krylov
from oracle.curvilinear import MappedOperator, lh_stencil, metric
from oracle.operator import Operator
from oracle.problem import Problem
from oracle.stepping import STANDARD, WaveHoltz
from paper_2205_12344_amd.inputs import media_mapped, rectangle_grid, ring_grid, sector_grid, warped_grid


def rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


# ---- the manufactured-solution helper ----------------------------------------

def _fields(X, Y):
    x, y = Jet.var_x(X), Jet.var_y(Y)
    u = jets.sin(0.7 * x + 0.3 * y) * (x * y + 1.0)
    v = jets.cos(0.4 * x - 0.9 * y) * jets.exp(0.1 * x)
    lam = 2.0 + 0.5 * jets.sin(x + 2.0 * y)
    mu = 1.0 + 0.3 * jets.cos(2.0 * x - y)
    return u, v, lam, mu


def test_jets_and_stress_divergence_match_finite_differences():
    rng = np.random.default_rng(0)
    X, Y = rng.uniform(-1, 2, 50), rng.uniform(-1, 2, 50)
    u, v, lam, mu = _fields(X, Y)
    d = 1e-4
    for comp in (u, v):
        def val(dx, dy, comp=comp):
            w = _fields(X + dx, Y + dy)
            return (w[0] if comp is u else w[1]).v
        assert np.allclose(comp.gx, (val(d, 0) - val(-d, 0)) / (2 * d), atol=1e-7)
        assert np.allclose(comp.gy, (val(0, d) - val(0, -d)) / (2 * d), atol=1e-7)
        assert np.allclose(comp.hxx, (val(d, 0) - 2 * comp.v + val(-d, 0)) / d ** 2, atol=1e-5)
        assert np.allclose(comp.hyy, (val(0, d) - 2 * comp.v + val(0, -d)) / d ** 2, atol=1e-5)
        assert np.allclose(comp.hxy, (val(d, d) - val(d, -d) - val(-d, d) + val(-d, -d)) / (4 * d * d), atol=1e-5)

    # stress from its definition at shifted points, divergence by differences
    def stress(dx, dy):
        uu, vv, ll, mm = _fields(X + dx, Y + dy)
        div = uu.gx + vv.gy
        sxx = ll.v * div + 2 * mm.v * uu.gx
        syy = ll.v * div + 2 * mm.v * vv.gy
        sxy = mm.v * (uu.gy + vv.gx)
        return sxx, sxy, syy

    fx, fy = jets.stress_divergence(u, v, lam, mu)
    xp, xm, yp, ym = stress(d, 0), stress(-d, 0), stress(0, d), stress(0, -d)
    assert np.allclose(fx, (xp[0] - xm[0]) / (2 * d) + (yp[1] - ym[1]) / (2 * d), atol=1e-6)
    assert np.allclose(fy, (xp[1] - xm[1]) / (2 * d) + (yp[2] - ym[2]) / (2 * d), atol=1e-6)


# ---- structure -----------------------------------------------------------------

def test_scaled_identity_map_is_the_cartesian_operator():
    nq, nr, lq, lr = 9, 13, 1.3, 2.1
    x, y = rectangle_grid(nq, nr, lq, lr)
    rho, lam, mu = media_mapped(x, y, seed=5)
    m = MappedOperator(x, y, rho, lam, mu)
    c = Operator(Problem(2, (nq, nr), length=(lq, lr)), rho, lam, mu)
    d = (m.Lt - c.Lt).toarray()
    assert np.max(np.abs(d)) <= 1e-12 * np.max(np.abs(c.Lt.toarray()))
    assert np.allclose(m.m, c.m * lq * lr, rtol=1e-14)
    assert abs(m.gershgorin() - c.gershgorin()) <= 1e-12 * c.gershgorin()


def test_rotation_equivariance():
    x, y = sector_grid(7, 20, 1)
    rho, lam, mu = media_mapped(x, y, seed=1)
    phi = 0.7
    cs, sn = math.cos(phi), math.sin(phi)
    a = MappedOperator(x, y, rho, lam, mu)
    b = MappedOperator(cs * x - sn * y, sn * x + cs * y, rho, lam, mu)
    prob = a.prob
    U = np.random.default_rng(2).standard_normal(prob.field_shape)
    RU = np.stack([cs * U[0] - sn * U[1], sn * U[0] + cs * U[1]])
    LU = prob.scatter(a.Lh @ prob.gather(U))
    LRU = prob.scatter(b.Lh @ prob.gather(RU))
    expect = np.stack([cs * LU[0] - sn * LU[1], sn * LU[0] + cs * LU[1]])
    assert rel(LRU, expect) <= 1e-12


def test_symmetric_definite_and_energy():
    x, y = warped_grid(6, 8, seed=3)
    rho, lam, mu = media_mapped(x, y, seed=3)
    op = MappedOperator(x, y, rho, lam, mu)
    L = op.Lh.toarray()
    assert np.max(np.abs(L - L.T)) <= 1e-14 * np.max(np.abs(L))
    ev = np.linalg.eigvalsh(-L)
    assert ev[0] > 0
    U = np.random.default_rng(4).standard_normal(op.prob.field_shape)
    U[:, 0, :] = U[:, -1, :] = U[:, :, 0] = U[:, :, -1] = 0.0
    xv = op.prob.gather(U)
    assert abs(op.energy(U) - 0.5 * xv @ (-op.Lh @ xv)) <= 1e-12 * abs(op.energy(U))
    # the full Hessian (boundary nodes included) is semi-definite with the
    # rigid translations in its kernel
    K = op.stiffness()
    T = np.concatenate([np.ones(x.size), np.zeros(x.size)])
    assert np.max(np.abs(K @ T)) <= 1e-12 * np.max(np.abs(K.diagonal()))


def test_stencil_form_equals_energy_hessian():
    for x, y in (warped_grid(11, 9, seed=7), sector_grid(6, 25, 2)):
        rho, lam, mu = media_mapped(x, y, seed=8)
        op = MappedOperator(x, y, rho, lam, mu)
        U = np.random.default_rng(9).standard_normal(op.prob.field_shape)
        U[:, 0, :] = U[:, -1, :] = U[:, :, 0] = U[:, :, -1] = 0.0
        got = op.prob.gather(lh_stencil(x, y, lam, mu, U))
        assert rel(got, op.Lh @ op.prob.gather(U)) <= 1e-13


def test_metric_of_the_sector():
    # J = (r_out - r_in) * (n_an pi / 2) * radius for the polar map, to O(h^2)
    errs = []
    for nq in (8, 16, 32):
        x, y = sector_grid(nq, 5 * nq, 2)
        J, Gq, Gr = metric(x, y, 1.0 / nq, 1.0 / (5 * nq))
        rad = np.hypot(x, y)
        errs.append(np.max(np.abs(J - math.pi * rad)) / np.max(J))
    assert errs[0] < 1e-2 and errs[1] / errs[2] > 3.5 and errs[0] / errs[1] > 3.5


# ---- accuracy against a continuous manufactured solution -------------------------

def test_truncation_error_is_second_order_on_the_quarter_annulus():
    inner, near = [], []
    for nq in (8, 16, 32):
        x, y = sector_grid(nq, 5 * nq, 1)
        u, v, lam, mu = _fields(x, y)
        U = np.stack([u.v, v.v])
        J, _, _ = metric(x, y, 1.0 / nq, 1.0 / (5 * nq))
        LU = lh_stencil(x, y, lam.v, mu.v, U)
        fx, fy = jets.stress_divergence(u, v, lam, mu)
        e = np.abs(np.stack([LU[0] / J - fx, LU[1] / J - fy]))
        inner.append(np.max(e[:, 2:-2, 2:-2]))
        near.append(np.max(e[:, 1:-1, 1:-1]))
    r_inner = np.log2(inner[1] / inner[2])
    assert r_inner > 1.85, inner
    # next to the boundary the one-sided metric costs one order (a layer one
    # node wide: the solution stays second order, next test)
    assert np.log2(near[1] / near[2]) > 0.9, near


def test_helmholtz_solution_converges_at_second_order():
    errs = []
    r_out = 10.0 / math.pi
    r_in = r_out - 1.0
    omega = 1.3
    for nq in (8, 16, 32):
        x, y = sector_grid(nq, 5 * nq, 1)
        X, Y = Jet.var_x(x), Jet.var_y(y)
        R2 = X * X + Y * Y
        g = X * Y * (R2 - r_in ** 2) * (r_out ** 2 - R2) * 0.05
        u = g * jets.sin(0.7 * X + 0.3 * Y)
        v = g * jets.cos(0.4 * X - 0.9 * Y)
        lam = 2.0 + 0.5 * jets.sin(X + 2.0 * Y)
        mu = 1.0 + 0.3 * jets.cos(2.0 * X - Y)
        rho = 1.0 + 0.2 * np.sin(x - y)
        op = MappedOperator(x, y, rho, lam.v, mu.v)
        fx, fy = jets.stress_divergence(u, v, lam, mu)
        f = np.stack([omega ** 2 * rho * u.v + fx, omega ** 2 * rho * v.v + fy])
        sol = op.prob.scatter(direct.solve(op, omega, op.prob.gather(f)))
        exact = np.stack([u.v, v.v])
        errs.append(np.max(np.abs(sol - exact)) / np.max(np.abs(exact)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert errs[-1] < 3e-3 and np.all(rates > 1.9), (errs, rates)


def test_filter_fixed_point_on_a_mapped_grid():
    x, y = sector_grid(10, 30, 2)
    rho, lam, mu = media_mapped(x, y, seed=11)
    op = MappedOperator(x, y, rho, lam, mu)
    omega = 6.0
    wh = WaveHoltz(op, omega)
    vs = np.random.default_rng(12).standard_normal(op.ndof)
    f = direct.manufactured_forcing(op, omega, vs)
    assert rel(wh.apply_filter(vs, f), vs) <= 1e-12
    assert rel(direct.solve(op, omega, f), vs) <= 1e-10


# ---- Sec. 5.5: the geometry hardly changes the iteration count ---------------------

def sector_cr_iterations(k, geometry):
    """CR iterations to 1e-8 (standard scheme, lambda = 2, mu = rho = 1,
    n_r = 4 L omega + 1, n_q = 4 omega + 1, point source of amplitude
    omega^2 at i = j = (n_q + 1) / 2) on the rectangle or an annular sector."""
    w = k + math.sqrt(2) / 10
    nq, nr = int(4 * w + 1), int(4 * 5 * w + 1)
    if geometry == "rectangle":
        x, y = rectangle_grid(nq, nr, 1.0, 5.0)
    else:
        x, y = sector_grid(nq, nr, 1 if geometry == "quarter" else 2)
    one = np.ones(x.shape)
    op = MappedOperator(x, y, one, 2.0 * one, one)
    f = np.zeros(op.prob.field_shape)
    i = (nq + 1) // 2
    f[0, i, i] = w * w / (op.J[i, i] / (nq * nr))
    wh = WaveHoltz(op, w, scheme=STANDARD)
    r = krylov.cr(wh.apply_A, wh.rhs(op.prob.gather(f)), op.m, tol=1e-8, maxit=5000)
    assert r.converged
    return r.iters


@pytest.mark.slow
def test_sector_iterations_match_the_rectangle():
    """The paper's figure prints no values; its statement that the three
    geometries need very similar counts is read as: within 40 % of the
    rectangle at every frequency, with the same omega^2 growth.  The oracle
    gives 16/54/71/180 (rectangle), 16/42/65/151 (quarter) and 13/39/55/127
    (half annulus) for k = 4, 6, 8, 12."""
    ks = (4, 6, 8, 12)
    its = {g: [sector_cr_iterations(k, g) for k in ks] for g in ("rectangle", "quarter", "half")}
    ws = np.log([k + math.sqrt(2) / 10 for k in ks])
    for g, n in its.items():
        slope = np.polyfit(ws, np.log(n), 1)[0]
        assert 1.6 <= slope <= 2.6, (g, n, slope)
    for g in ("quarter", "half"):
        ratio = np.array(its[g]) / np.array(its["rectangle"])
        assert np.all(ratio > 0.6) and np.all(ratio < 1.4), (its, ratio)


# ---- traction-free r sides (the free curved surfaces of Sec. 5.11, in 2-D) ----------

@pytest.mark.parametrize("bc", [(0, 0, 1, 1), (0, 0, 0, 1), (0, 0, 1, 0)])
def test_free_sides_of_a_scaled_identity_map_are_the_cartesian_closure(bc):
    nq, nr, lq, lr = 8, 11, 0.9, 1.7
    x, y = rectangle_grid(nq, nr, lq, lr)
    rho, lam, mu = media_mapped(x, y, seed=21)
    m = MappedOperator(x, y, rho, lam, mu, bc=bc)
    c = Operator(Problem(2, (nq, nr), length=(lq, lr), bc=bc), rho, lam, mu)
    assert m.ndof == c.ndof
    d = (m.Lt - c.Lt).toarray()
    assert np.max(np.abs(d)) <= 1e-12 * np.max(np.abs(c.Lt.toarray()))
    assert np.allclose(m.m, c.m * lq * lr, rtol=1e-14)


def test_free_sides_structure_on_a_ring_sector():
    x, y = ring_grid(18, 7)
    rho, lam, mu = media_mapped(x, y, seed=22)
    bc = (0, 0, 1, 1)
    op = MappedOperator(x, y, rho, lam, mu, bc=bc)
    L = op.Lh.toarray()
    assert np.max(np.abs(L - L.T)) <= 1e-14 * np.max(np.abs(L))
    assert np.linalg.eigvalsh(-L)[0] > 0
    prob = op.prob
    U = np.random.default_rng(23).standard_normal(prob.field_shape) * prob.unknown_mask()
    xv = prob.gather(U)
    assert abs(op.energy(U) - 0.5 * xv @ (-op.Lh @ xv)) <= 1e-12 * abs(op.energy(U))
    K = op.stiffness()
    for c in range(2):
        T = np.zeros(2 * x.size)
        T[c * x.size:(c + 1) * x.size] = 1.0
        assert np.max(np.abs(K @ T)) <= 1e-12 * np.max(np.abs(K.diagonal()))
    # rotation equivariance with free sides
    phi = -1.1
    cs, sn = math.cos(phi), math.sin(phi)
    b = MappedOperator(cs * x - sn * y, sn * x + cs * y, rho, lam, mu, bc=bc)
    RU = np.stack([cs * U[0] - sn * U[1], sn * U[0] + cs * U[1]])
    LU = prob.scatter(op.Lh @ xv)
    expect = np.stack([cs * LU[0] - sn * LU[1], sn * LU[0] + cs * LU[1]])
    assert rel(prob.scatter(b.Lh @ prob.gather(RU)), expect) <= 1e-12


def test_free_sides_converge_at_second_order():
    """Self-convergence of the Helmholtz solution on the ring sector with
    traction-free inner and outer arcs (no closed-form solution satisfies the
    free condition on the curved sides with variable media): differences
    between successive refinements, at the coarse nodes, fall like h^2."""
    sols = []
    omega = 1.7
    for k in (1, 2, 4):
        nq, nr = 24 * k, 8 * k
        x, y = ring_grid(nq, nr)
        rho = 1.0 + 0.2 * np.sin(x + 0.5 * y)
        mu = 1.0 + 0.3 * np.cos(0.7 * x - y)
        lam = 2.0 + 0.5 * np.sin(x * y)
        op = MappedOperator(x, y, rho, lam, mu, bc=(0, 0, 1, 1))
        f = np.stack([np.exp(-((x + 0.8) ** 2 + (y - 1.1) ** 2) / 0.18),
                      0.5 * np.exp(-((x - 1.0) ** 2 + (y - 1.2) ** 2) / 0.2)])
        sol = op.prob.scatter(direct.solve(op, omega, op.prob.gather(f)))
        sols.append(sol[:, ::k, ::k])
    scale = np.max(np.abs(sols[-1]))
    d1 = np.max(np.abs(sols[0] - sols[1])) / scale
    d2 = np.max(np.abs(sols[1] - sols[2])) / scale
    assert np.log2(d1 / d2) > 1.8, (d1, d2)
