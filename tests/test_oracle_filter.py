"""Pins of the oracle's stepper, filter and Krylov solvers against what the
paper prints and what the mathematics fixes (CPU only)."""

import json
import math
import os

import numpy as np
import pytest

from oracle import direct, krylov, spectral
from oracle import stepping as S
from oracle.operator import Operator
from oracle.problem import DIRICHLET, FREE, Problem
from paper_2205_12344_amd import inputs


def _media(prob, seed, s=0.3):
    rng = np.random.default_rng(seed)
    sh = prob.node_shape
    rho = np.exp(s * rng.standard_normal(sh))
    mu = np.exp(s * rng.standard_normal(sh))
    return rho, 2.0 * mu * np.exp(s * rng.standard_normal(sh)), mu


# ---------------------------------------------------------------- weights ----

@pytest.mark.parametrize("nt", [3, 4, 5, 7, 64, 121])
def test_weights_reproduce_fixed_point(nt):
    """Sec. 3: a field v cos(w t) is a fixed point of the filter; the trapezoid
    rule with a whole number of steps keeps this exactly (sum cos^2 = N/2 for
    N >= 3), and the transfer at lambda = 0 is -1/2."""
    w, cosn = S.filter_weights(nt)
    assert np.dot(w, cosn) == pytest.approx(1.0, abs=1e-14)
    assert w.sum() == pytest.approx(-0.5, abs=1e-14)


def test_weights_k_periods():
    """eq. (many_periods_filter): K periods, prefactor 2/(K T)."""
    for K in (1, 2, 3, 5):
        w, cosn = S.filter_weights(9, K)
        assert len(w) == 9 * K + 1
        assert np.dot(w, cosn) == pytest.approx(1.0, abs=1e-14)


def test_continuous_transfer_limits():
    """beta_bar closed form vs the trapezoid sum at many steps; beta(0) = -1/2,
    beta(1) = 1 (Sec. 3 and App. B)."""
    r = np.array([0.0, 0.3, 0.77, 0.999, 1.0, 1.4, 2.5])
    np.testing.assert_allclose(spectral.beta_bar_h(r, 4000), spectral.beta_bar(r), atol=2e-6)
    assert spectral.beta_bar([1.0])[0] == 1.0


def test_appendix_b_gap_bound(golden_dir):
    """App. B: the leftmost r* < 1 where the trapezoid transfer reaches 1
    obeys 1 - r* <= 0.022 dt^2, k = 5..100."""
    g = json.load(open(os.path.join(golden_dir, "appendix_b_gap.json")))
    worst = 0.0
    for k in range(g["k_min"], g["k_max"] + 1):
        dt = 2 * math.pi / k
        gap = 1.0 - spectral.resonance_gap(k)
        assert 0 < gap <= g["constant"] * dt * dt
        worst = max(worst, gap / (dt * dt))
    assert worst > 0.02          # the bound is nearly tight, as the figure shows


# ---------------------------------------------------- fixed point, exactness --

def _case_free_top(seed=11):
    prob = Problem(2, (20, 16), bc=(DIRICHLET, DIRICHLET, DIRICHLET, FREE))
    op = Operator(prob, *_media(prob, seed))
    return prob, op


def test_fixed_point_square64():
    """Sec. 1.1 / 4.3: with the corrected scheme the discrete WaveHoltz fixed
    point is the direct discretisation of the Helmholtz equation:
    Pi_h v* = v*, v* = (w^2 M + L_h)^-1 W f."""
    c = inputs.constant_square64()
    prob = Problem(2, c.n, bc=c.bc)
    op = Operator(prob, c.rho, c.lam, c.mu)
    wh = S.WaveHoltz(op, c.omega)
    assert wh.nt == 121
    f = prob.gather(c.f)
    v = direct.solve(op, c.omega, f)
    assert np.abs(wh.apply_filter(v, f) - v).max() <= 1e-12 * np.abs(v).max()


@pytest.mark.parametrize("periods", [1, 3])
def test_fixed_point_free_surface(periods):
    prob, op = _case_free_top()
    wh = S.WaveHoltz(op, 6.3, periods=periods)
    f = np.random.default_rng(1).standard_normal(op.ndof)
    v = direct.solve(op, 6.3, f)
    assert np.abs(wh.apply_filter(v, f) - v).max() <= 1e-12 * np.abs(v).max()


def test_fixed_point_3d():
    prob = Problem(3, (6, 5, 7), bc=(DIRICHLET,) * 4 + (FREE, FREE))
    op = Operator(prob, *_media(prob, 12))
    wh = S.WaveHoltz(op, 3.7)
    f = np.random.default_rng(2).standard_normal(op.ndof)
    v = direct.solve(op, 3.7, f)
    assert np.abs(wh.apply_filter(v, f) - v).max() <= 1e-12 * np.abs(v).max()


def test_standard_scheme_converges_to_modified_frequency():
    """Sec. 4.3: the uncorrected scheme's fixed point solves the Helmholtz
    system at wt = 2 sin(w dt/2)/dt, not at w."""
    prob, op = _case_free_top(13)
    om = 5.1
    wh = S.WaveHoltz(op, om, scheme=S.STANDARD)
    wt = 2 * math.sin(om * wh.dt / 2) / wh.dt
    f = np.random.default_rng(3).standard_normal(op.ndof)
    vt = direct.solve(op, wt, f)
    v = direct.solve(op, om, f)
    assert np.abs(wh.apply_filter(vt, f) - vt).max() <= 1e-12 * np.abs(vt).max()
    assert np.abs(wh.apply_filter(v, f) - v).max() > 1e-6 * np.abs(v).max()


class _LiteralStart(S.WaveHoltz):
    """A planted mistake: the initial data exactly as printed in Sec. 4.3,
    u^{-1} = u0 - c dt^2/2 L(u0 + f)."""

    def trajectory(self, u0, f=None):
        L = self.op.apply_Ltilde
        fz = np.zeros_like(u0) if f is None else f
        u_prev = u0 - 0.5 * self.a * L(u0 + fz)
        u_cur = np.asarray(u0, np.float64).copy()
        yield u_cur
        for n in range(0, self.periods * self.nt):
            g = L(u_cur) - fz * self.cosn[n]
            u_next = 2.0 * u_cur - u_prev + self.a * g
            u_prev, u_cur = u_cur, u_next
            yield u_cur


class _NoShift(S.WaveHoltz):
    """A planted mistake: the -1/4 shift of the filter kernel dropped."""

    def __init__(self, *a, **k):
        super().__init__(*a, **k)
        nt = self.nt * self.periods
        eta = np.ones(nt + 1)
        eta[0] = eta[-1] = 0.5
        self.weights = (2.0 / nt) * eta * self.cosn


def test_planted_mistakes_are_caught():
    """The pins are sharp: the literal printed start moves the fixed point off
    v*; a dropped -1/4 shift keeps v* fixed (sum w cos = 1 either way) but
    changes the zero-frequency transfer beta(0) = -1/2 that makes the fixed
    point unique (Sec. 3), and with it the spectrum of A_h."""
    prob, op = _case_free_top(14)
    f = np.random.default_rng(4).standard_normal(op.ndof)
    v = direct.solve(op, 6.3, f)
    good = S.WaveHoltz(op, 6.3)
    assert np.abs(good.apply_filter(v, f) - v).max() <= 1e-12 * np.abs(v).max()
    bad = _LiteralStart(op, 6.3)
    assert np.abs(bad.apply_filter(v, f) - v).max() > 1e-3 * np.abs(v).max()
    ns = _NoShift(op, 6.3)
    assert abs(ns.weights.sum() + 0.5) > 0.4
    assert abs(good.weights.sum() + 0.5) < 1e-14


# --------------------------------------------------------------- invariants --

def test_energy_conserved_and_forced_balance():
    """Sec. 4.1 eq. (8), corrected form: E^{n+1/2} constant for f = 0 over three
    periods; with forcing, E^{n+1/2} - E^{n-1/2} = -cos_n (W f).(u^{n+1} - u^{n-1})."""
    prob, op = _case_free_top(15)
    wh = S.WaveHoltz(op, 4.4, periods=3)
    u0 = np.random.default_rng(5).standard_normal(op.ndof)
    E = wh.energies(u0)
    assert E.min() > 0
    assert (E.max() - E.min()) <= 1e-12 * E.max()
    f = np.random.default_rng(6).standard_normal(op.ndof)
    traj = list(wh.trajectory(u0, f))
    E = wh.energies(u0, f)
    for n in range(1, len(E)):
        lhs = E[n] - E[n - 1]
        rhs = -wh.cosn[n] * float((op.w * f) @ (traj[n + 1] - traj[n - 1]))
        assert lhs == pytest.approx(rhs, rel=1e-8, abs=1e-10 * E.max())


def test_brute_force_operator_properties():
    """Tiny grid, A_h assembled column by column: M A_h symmetric (Sec. 4.5),
    eigenvalues in (0, 3/2) (Sec. 3), and A_h^-1 b = v* (dense solve)."""
    prob = Problem(2, (6, 5), bc=(DIRICHLET, DIRICHLET, DIRICHLET, FREE))
    op = Operator(prob, *_media(prob, 16))
    wh = S.WaveHoltz(op, 2.9)
    A = direct.dense_operator(wh.apply_A, op.ndof)
    MA = op.m[:, None] * A
    assert np.abs(MA - MA.T).max() <= 1e-13 * np.abs(MA).max()
    ev = np.linalg.eigvals(A)
    assert np.abs(ev.imag).max() < 1e-10
    assert ev.real.min() > 0 and ev.real.max() < 1.5
    f = np.random.default_rng(7).standard_normal(op.ndof)
    b = wh.rhs(f)
    x = np.linalg.solve(A, b)
    v = direct.solve_dense(op, 2.9, f)
    assert np.abs(x - v).max() <= 1e-11 * np.abs(v).max()


def test_spectral_closed_form():
    """eig(A_h) = 1 - beta_h(theta_j), theta_j = 2 arcsin(sin(w dt/2) lam_j / w)
    for the eigenpairs -L_h phi = lam^2 M phi."""
    import scipy.linalg as sl
    prob = Problem(2, (7, 6), bc=(DIRICHLET, DIRICHLET, DIRICHLET, FREE))
    op = Operator(prob, *_media(prob, 17, 0.2))
    om = 4.2
    wh = S.WaveHoltz(op, om)
    lam2 = sl.eigh(-op.Lh.toarray(), np.diag(op.m), eigvals_only=True)
    theta = spectral.mode_angle(np.sqrt(lam2), om, wh.dt)
    pred = np.sort(1.0 - spectral.beta_h(theta, wh.weights))
    A = direct.dense_operator(wh.apply_A, op.ndof)
    got = np.sort(np.linalg.eigvals(A).real)
    np.testing.assert_allclose(got, pred, atol=1e-12)


# ------------------------------------------------------------- Table 1 ------

def _quartic_case(n, om=1.0, lam=1.0, mu=1.0):
    prob = Problem(2, (n, n))
    X, Y = prob.mesh()
    p = lambda s: s ** 2 * (s - 1) ** 2
    d1 = lambda s: 2 * s * (s - 1) ** 2 + 2 * s ** 2 * (s - 1)
    d2 = lambda s: 2 * (s - 1) ** 2 + 8 * s * (s - 1) + 2 * s ** 2
    U = 256 * p(X) * p(Y)
    uxx, uyy, uxy = 256 * d2(X) * p(Y), 256 * p(X) * d2(Y), 256 * d1(X) * d1(Y)
    A = lam + 2 * mu
    f = np.array([om ** 2 * U + A * uxx + mu * uyy + (lam + mu) * uxy,
                  om ** 2 * U + mu * uxx + A * uyy + (lam + mu) * uxy])
    return prob, np.array([U, U]), f


def test_table1_fd_accuracy(golden_dir):
    """Table 1 (Sec. 5.1): standard leapfrog with k = 0.4 h / sqrt(3 mu + lam),
    omega = 1; the converged WaveHoltz solution is the fixed point, i.e. the
    Helmholtz solve at the modified frequency (Sec. 4.3), checked here by
    one filter application.  Rates match the printed ones to two decimals
    (+-0.011), errors within 2.5 percent."""
    g = json.load(open(os.path.join(golden_dir, "table1_fd_accuracy.json")))
    errs = []
    for n in g["n"]:
        prob, U, f = _quartic_case(n)
        op = Operator(prob, 1.0, 1.0, 1.0)
        k = 0.4 * prob.h[0] / math.sqrt(3.0 + 1.0)
        nt = int(math.ceil(2 * math.pi / k))
        wh = S.WaveHoltz(op, 1.0, nt=nt, scheme=S.STANDARD)
        wt = 2 * math.sin(wh.dt / 2) / wh.dt
        fv = prob.gather(f)
        v = direct.solve(op, wt, fv)
        if n <= 40:
            assert np.abs(wh.apply_filter(v, fv) - v).max() <= 1e-11 * np.abs(v).max()
        errs.append(float(np.mean(np.abs(v - prob.gather(U)))))
    for e, ep in zip(errs, g["error"]):
        assert e == pytest.approx(ep, rel=0.025)
    rates = [math.log2(errs[i - 1] / errs[i]) for i in range(1, len(errs))]
    for r, rp in zip(rates, g["rate"][1:]):
        assert abs(r - rp) <= 0.011


def _manufactured_variable_2d(n, om):
    """u = sin(pi x) sin(pi y) (1 + x y), v = sin(2 pi x) sin(pi y) with
    lam = 2 + x y, mu = 1 + x^2 / 2, rho = 1 + y / 2; f = w^2 rho u + div T(u)
    by hand-written derivatives."""
    prob = Problem(2, (n, n))
    X, Y = prob.mesh()
    pi = math.pi
    s, c = np.sin, np.cos
    lam, lx, ly = 2 + X * Y, Y, X
    mu, mx, my = 1 + X ** 2 / 2, X, 0 * X
    rho = 1 + Y / 2
    A, Ax, Ay = lam + 2 * mu, lx + 2 * mx, ly + 2 * my
    g = 1 + X * Y
    u = s(pi * X) * s(pi * Y) * g
    ux = pi * c(pi * X) * s(pi * Y) * g + s(pi * X) * s(pi * Y) * Y
    uy = pi * s(pi * X) * c(pi * Y) * g + s(pi * X) * s(pi * Y) * X
    uxx = -pi ** 2 * u + 2 * pi * c(pi * X) * s(pi * Y) * Y
    uyy = -pi ** 2 * u + 2 * pi * s(pi * X) * c(pi * Y) * X
    uxy = (pi ** 2 * c(pi * X) * c(pi * Y) * g + pi * c(pi * X) * s(pi * Y) * X
           + pi * s(pi * X) * c(pi * Y) * Y + s(pi * X) * s(pi * Y))
    v = s(2 * pi * X) * s(pi * Y)
    vx = 2 * pi * c(2 * pi * X) * s(pi * Y)
    vy = pi * s(2 * pi * X) * c(pi * Y)
    vxx = -4 * pi ** 2 * v
    vyy = -pi ** 2 * v
    vxy = 2 * pi ** 2 * c(2 * pi * X) * c(pi * Y)
    # div T: d/dx[A ux + lam vy] + d/dy[mu (uy + vx)];  d/dx[mu (vx + uy)] + d/dy[lam ux + A vy]
    f1 = Ax * ux + A * uxx + lx * vy + lam * vxy + my * (uy + vx) + mu * (uyy + vxy)
    f2 = mx * (vx + uy) + mu * (vxx + uxy) + ly * ux + lam * uxy + Ay * vy + A * vyy
    f = np.array([om ** 2 * rho * u + f1, om ** 2 * rho * v + f2])
    return prob, rho, lam, mu, np.array([u, v]), f


def test_manufactured_variable_medium_second_order():
    """Second-order convergence to a closed-form solution in a smooth
    variable medium: catches a wrong coefficient average or a dropped
    derivative of the coefficients (both give O(1) or O(h) error)."""
    errs = []
    om = 3.0
    for n in (16, 32, 64):
        prob, rho, lam, mu, U, f = _manufactured_variable_2d(n, om)
        op = Operator(prob, rho, lam, mu)
        v = direct.solve(op, om, prob.gather(f))
        errs.append(np.abs(v - prob.gather(U)).max())
    rates = [math.log2(errs[i - 1] / errs[i]) for i in range(1, 3)]
    assert min(rates) > 1.9 and errs[-1] < 5e-3


def _manufactured_free_top(n, om, lam=2.0, mu=1.0):
    """Traction-free top y = 1, Dirichlet elsewhere, constant medium:
    u = 2 pi y (1 - y) sin(2 pi x),  v = (1 - cos 2 pi x) sin(pi y / 2).
    At y = 1: sigma_xy = mu (u_y + v_x) = 0 and sigma_yy = lam u_x + A v_y = 0,
    while v does not vanish there."""
    prob = Problem(2, (n, n), bc=(DIRICHLET, DIRICHLET, DIRICHLET, FREE))
    X, Y = prob.mesh()
    pi = math.pi
    A = lam + 2 * mu
    a, a1, a2 = 2 * pi * Y * (1 - Y), 2 * pi * (1 - 2 * Y), -4 * pi + 0 * Y
    b, b1, b2 = np.sin(pi * Y / 2), (pi / 2) * np.cos(pi * Y / 2), -(pi / 2) ** 2 * np.sin(pi * Y / 2)
    sx, sx1, sx2 = np.sin(2 * pi * X), 2 * pi * np.cos(2 * pi * X), -4 * pi ** 2 * np.sin(2 * pi * X)
    tx, tx1, tx2 = 1 - np.cos(2 * pi * X), 2 * pi * np.sin(2 * pi * X), 4 * pi ** 2 * np.cos(2 * pi * X)
    u, v = sx * a, tx * b
    uxx, uyy, uxy = sx2 * a, sx * a2, sx1 * a1
    vxx, vyy, vxy = tx2 * b, tx * b2, tx1 * b1
    f1 = A * uxx + mu * uyy + (lam + mu) * vxy
    f2 = mu * vxx + A * vyy + (lam + mu) * uxy
    f = np.array([om ** 2 * u + f1, om ** 2 * v + f2])
    return prob, lam, mu, np.array([u, v]), f


def test_manufactured_free_surface_converges():
    """Second-order convergence with the free-surface closure (its absolute
    values are otherwise parity unpinned)."""
    errs = []
    om = 2.5
    for n in (16, 32, 64, 128):
        prob, lam, mu, U, f = _manufactured_free_top(n, om)
        op = Operator(prob, 1.0, lam, mu)
        v = direct.solve(op, om, prob.gather(f))
        errs.append(np.abs(v - prob.gather(U)).max())
    rates = [math.log2(errs[i - 1] / errs[i]) for i in range(1, len(errs))]
    assert rates[-1] > 1.8 and errs[-1] < 2e-3


# --------------------------------------------------------------- Krylov -----

def test_cg_square64_matches_direct():
    """64^2 constant medium: CG in the M inner product to 1e-10 reproduces the direct
    solve (14 iterations, error about 3e-12)."""
    c = inputs.constant_square64()
    prob = Problem(2, c.n, bc=c.bc)
    op = Operator(prob, c.rho, c.lam, c.mu)
    wh = S.WaveHoltz(op, c.omega)
    f = prob.gather(c.f)
    v = direct.solve(op, c.omega, f)
    res = krylov.cg(wh.apply_A, wh.rhs(f), op.m, tol=1e-10, maxit=100)
    assert res.converged and res.iters <= 20
    assert np.linalg.norm(res.x - v) <= 1e-10 * np.linalg.norm(v)
    assert 1 < res.lanczos_cond() < 1e5


@pytest.mark.parametrize("method", ["cg", "cr", "gmres"])
def test_krylov_variable_medium_matches_direct(method):
    prob, op = _case_free_top(18)
    wh = S.WaveHoltz(op, 5.3)
    f = np.random.default_rng(8).standard_normal(op.ndof)
    v = direct.solve(op, 5.3, f)
    solver = getattr(krylov, method)
    kw = {"restart": 12} if method == "gmres" else {}
    res = solver(wh.apply_A, wh.rhs(f), op.m, tol=1e-12, maxit=400, **kw)
    assert res.converged
    assert np.linalg.norm(res.x - v) <= 1e-10 * np.linalg.norm(v)
    # warm start from a perturbed solution converges too
    x0 = v + 1e-3 * np.random.default_rng(9).standard_normal(op.ndof)
    res = solver(wh.apply_A, wh.rhs(f), op.m, x0=x0, tol=1e-12, maxit=400, **kw)
    assert res.converged and np.linalg.norm(res.x - v) <= 1e-10 * np.linalg.norm(v)
