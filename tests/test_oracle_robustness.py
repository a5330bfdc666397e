"""Pins of the oracle's robustness tools near resonance (CPU only):

* MINRES in the M inner product (the remedy the remark in Sec. 4.4
  recommends when A_h is slightly indefinite), pinned by its defining
  property: its residual after k steps is the smallest M-norm residual over
  x0 + K_k(A, r0), computed here independently by a dense least-squares
  solve over an explicit Krylov basis.
* The Lanczos condition estimate from the CG coefficients (Sec. 4.5), pinned
  against the extreme eigenvalues of the dense A_h when CG has run through
  the whole space.
* The modified trapezoid weights (the remark closing Sec. 4.4): under the
  standard stepper the fixed point equals the direct Helmholtz solution.
"""

import math

import numpy as np
import pytest

from oracle import direct, krylov
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


def _indefinite_system(n=40, seed=0):
    """A random M-self-adjoint indefinite matrix A = M^-1 S (S symmetric with
    eigenvalues on both sides of zero) and positive weights m."""
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    ev = np.concatenate([rng.uniform(-1.0, -0.05, n // 4), rng.uniform(0.02, 2.0, n - n // 4)])
    m = rng.uniform(0.5, 2.0, n)
    # A = M^-1/2 Q diag(ev) Q^T M^1/2 is self-adjoint in (x, y)_M
    sq = np.sqrt(m)
    A = (Q * ev) @ Q.T
    A = A * sq[None, :] / sq[:, None]
    return A, m, rng.standard_normal(n)


def _min_residual_over_krylov(A, m, b, x0, k):
    """min ||b - A x||_M over x0 + span{r0, A r0, ..., A^{k-1} r0}: an
    M-orthonormal basis of the Krylov space by modified Gram-Schmidt, then a
    dense least-squares solve in coordinates where the M norm is Euclidean."""
    sq = np.sqrt(m)
    r0 = b - A @ x0
    basis = []
    v = r0.copy()
    for _ in range(k):
        for u in basis:
            v = v - np.dot(m * u, v) * u
        for u in basis:                       # twice is enough
            v = v - np.dot(m * u, v) * u
        nv = math.sqrt(np.dot(m * v, v))
        basis.append(v / nv)
        v = A @ basis[-1]
    K = np.array(basis).T
    AK = sq[:, None] * (A @ K)
    y, *_ = np.linalg.lstsq(AK, sq * r0, rcond=None)
    res = sq * r0 - AK @ y
    return float(np.linalg.norm(res))


def test_minres_residuals_are_the_krylov_minimum():
    A, m, b = _indefinite_system()
    bn = math.sqrt(np.dot(m * b, b))
    res = krylov.minres(lambda x: A @ x, b, m, tol=0.0, maxit=25)
    for k in (1, 2, 3, 5, 8, 13, 21, 25):
        want = _min_residual_over_krylov(A, m, b, np.zeros_like(b), k) / bn
        assert res.history[k] == pytest.approx(want, rel=1e-9, abs=1e-13)
    # warm start: the same minimum over x0 + K_k
    x0 = np.random.default_rng(5).standard_normal(b.size)
    res = krylov.minres(lambda x: A @ x, b, m, x0=x0, tol=0.0, maxit=12)
    for k in (1, 4, 12):
        want = _min_residual_over_krylov(A, m, b, x0, k) / bn
        assert res.history[k] == pytest.approx(want, rel=1e-9, abs=1e-13)


def test_minres_history_is_the_true_residual_and_converges():
    A, m, b = _indefinite_system(seed=3)
    res = krylov.minres(lambda x: A @ x, b, m, tol=1e-12, maxit=200)
    assert res.converged
    x = np.linalg.solve(A, b)
    assert np.linalg.norm(res.x - x) <= 1e-9 * np.linalg.norm(x)
    r = b - A @ res.x
    assert math.sqrt(np.dot(m * r, r) / np.dot(m * b, b)) <= 2e-12
    # the residual never grows (a minimum over nested spaces)
    h = np.array(res.history)
    assert np.all(np.diff(h) <= 1e-15)


class _PlantedMinres:
    """MINRES with one plausible slip each; the Krylov-minimum pin must catch
    every one of them."""

    @staticmethod
    def run(A, m, b, slip, maxit):
        x = np.zeros_like(b)
        beta = math.sqrt(np.dot(m * b, b))
        v_prev, v = np.zeros_like(b), b / beta
        dp2, dp = np.zeros_like(b), np.zeros_like(b)
        c2 = c1 = 1.0
        s2 = s1 = 0.0
        g = beta
        hist = [1.0]
        for k in range(1, maxit + 1):
            q = A @ v
            alpha = np.dot(m * v, q)
            q = q - alpha * v - beta * v_prev
            bn = math.sqrt(np.dot(m * q, q))
            bj = beta if k > 1 else 0.0
            eps = 0.0 if slip == "drop_eps" else s2 * bj
            t = c2 * bj
            delta = c1 * t + (-s1 if slip == "sign" else s1) * alpha
            gbar = -s1 * t + c1 * alpha
            gam = math.hypot(gbar, bn)
            c, s = gbar / gam, bn / gam
            tau = c * g
            g = -s * g
            d = (v - delta * dp - eps * dp2) / gam
            x = x + tau * d
            r = b - A @ x
            hist.append(math.sqrt(np.dot(m * r, r)) / math.sqrt(np.dot(m * b, b)))
            dp2, dp = dp, d
            c2, s2, c1, s1 = c1, s1, c, s
            v_prev, v = v, q / bn
            beta = bn
        return hist


@pytest.mark.parametrize("slip", ["drop_eps", "sign"])
def test_minres_pin_catches_planted_mistakes(slip):
    A, m, b = _indefinite_system()
    bn = math.sqrt(np.dot(m * b, b))
    hist = _PlantedMinres.run(A, m, b, slip, 12)
    bad = [abs(hist[k] - _min_residual_over_krylov(A, m, b, np.zeros_like(b), k) / bn) for k in (4, 8, 12)]
    assert max(bad) > 1e-6


def test_minres_on_the_near_resonant_warmstart_problem():
    """The config-5 problem with seed 4115, coarsened to 64^2 cells, has a
    medium eigenvalue inside the band where the trapezoid transfer exceeds
    one: A_h is indefinite and CG breaks down; MINRES converges to the
    direct solution, in no more iterations than conjugate residual (both
    minimise ||r||_M over the same Krylov space)."""
    c = inputs.warmstart_problem(4115, n=64)
    prob = Problem(2, c.n, bc=c.bc)
    op = Operator(prob, c.rho, c.lam, c.mu)
    wh = S.WaveHoltz(op, c.omega)
    fv = prob.gather(c.f)
    b = wh.rhs(fv)
    xs = direct.solve(op, c.omega, fv)
    with pytest.raises(ArithmeticError, match="breakdown"):
        krylov.cg(wh.apply_A, b, op.m, tol=1e-8, maxit=3000)
    mr = krylov.minres(wh.apply_A, b, op.m, tol=1e-8, maxit=3000)
    assert mr.converged
    assert np.linalg.norm(mr.x - xs) / np.linalg.norm(xs) <= 1e-6
    cr = krylov.cr(wh.apply_A, b, op.m, tol=1e-8, maxit=3000)
    assert mr.iters <= cr.iters + 2
    r = b - wh.apply_A(mr.x)
    assert math.sqrt(wh.m_dot(r, r) / wh.m_dot(b, b)) <= 1.5e-8


# ------------------------------------------------------ Lanczos estimate ----

def _tiny_case(seed=7):
    prob = Problem(2, (5, 4), bc=(DIRICHLET, DIRICHLET, DIRICHLET, FREE))
    op = Operator(prob, *_media(prob, seed))
    wh = S.WaveHoltz(op, 8.0)             # condition number about 56
    return prob, op, wh


def test_lanczos_condition_equals_dense_spectrum():
    """After n CG steps on an n-dof system the Lanczos tridiagonal is similar
    to A_h, so its extreme eigenvalues are those of A_h; the estimate from
    the CG coefficients must equal lambda_max / lambda_min of the dense
    operator."""
    prob, op, wh = _tiny_case()
    n = op.ndof
    Ad = direct.dense_operator(wh.apply_A, n)
    ev = np.sort(np.linalg.eigvals(Ad).real)
    assert ev[0] > 0
    b = np.random.default_rng(3).standard_normal(n)
    res = krylov.cg(wh.apply_A, b, op.m, tol=1e-300, maxit=n)
    assert len(res.alphas) == n
    assert res.lanczos_cond() == pytest.approx(ev[-1] / ev[0], rel=1e-8)


def test_lanczos_pin_catches_an_index_shift():
    """The same tridiagonal with the beta of the previous step (an off-by-one
    in the diagonal term) misses the dense condition number."""
    prob, op, wh = _tiny_case()
    n = op.ndof
    ev = np.sort(np.linalg.eigvals(direct.dense_operator(wh.apply_A, n)).real)
    b = np.random.default_rng(3).standard_normal(n)
    res = krylov.cg(wh.apply_A, b, op.m, tol=1e-300, maxit=n)
    a, bt = res.alphas, res.betas
    T = np.zeros((n, n))
    for i in range(n):
        T[i, i] = 1.0 / a[i] + (bt[i - 2] / a[i - 1] if i > 1 else 0.0)
        if i + 1 < n:
            T[i, i + 1] = T[i + 1, i] = math.sqrt(bt[i]) / a[i]
    e = np.linalg.eigvalsh(T)
    assert abs(e[-1] / e[0] - ev[-1] / ev[0]) > 1e-2 * ev[-1] / ev[0]


# --------------------------------------------- modified trapezoid weights ----

@pytest.mark.parametrize("nt", [4, 5, 9, 40, 121])
def test_modified_weights_reproduce_the_harmonic_at_wbar(nt):
    """sum_n w_n cos(wbar t_n) = 1: the filter keeps v cos(wbar t) fixed."""
    omega = 3.0
    w, cbar = S.modified_filter_weights(nt, omega)
    assert np.dot(w, cbar) == pytest.approx(1.0, abs=1e-13)
    dt = 2 * math.pi / (omega * nt)
    wbar = S.modified_forcing_frequency(omega, dt)
    # the standard leapfrog's dispersion relation maps wbar back to omega
    assert 2.0 * math.sin(0.5 * wbar * dt) / dt == pytest.approx(omega, rel=1e-14)


def test_modified_weights_need_four_steps():
    with pytest.raises(ValueError):
        S.modified_filter_weights(3, 1.0)         # omega dt / 2 = pi / 3 > 1
    S.modified_filter_weights(4, 1.0)


@pytest.mark.parametrize("periods", [1, 2])
def test_modified_weights_fixed_point_standard_stepper(periods):
    """The remark closing Sec. 4.4: with the modified weights the standard
    (uncorrected) scheme has no time error in its fixed point either."""
    prob = Problem(2, (20, 16), bc=(DIRICHLET, DIRICHLET, DIRICHLET, FREE))
    op = Operator(prob, *_media(prob, 11))
    wh = S.WaveHoltz(op, 6.3, periods=periods, scheme=S.MODIFIED)
    assert wh.c == 1.0
    f = np.random.default_rng(1).standard_normal(op.ndof)
    v = direct.solve(op, 6.3, f)
    assert np.abs(wh.apply_filter(v, f) - v).max() <= 1e-11 * np.abs(v).max()
    # CG on the modified operator reaches the same direct solution
    res = krylov.cg(wh.apply_A, wh.rhs(f), op.m, tol=1e-11, maxit=600)
    assert res.converged and np.linalg.norm(res.x - v) <= 1e-9 * np.linalg.norm(v)


def test_modified_weights_3d_fixed_point():
    prob = Problem(3, (6, 5, 7), bc=(DIRICHLET,) * 4 + (FREE, FREE))
    op = Operator(prob, *_media(prob, 12))
    wh = S.WaveHoltz(op, 3.7, scheme=S.MODIFIED)
    f = np.random.default_rng(2).standard_normal(op.ndof)
    v = direct.solve(op, 3.7, f)
    assert np.abs(wh.apply_filter(v, f) - v).max() <= 1e-11 * np.abs(v).max()


def test_literal_modified_frequency_misses_the_fixed_point():
    """The other reading of the printed ratio (forcing at omega, denominator
    cos(wt t_n) with wt = 2 sin(omega dt / 2) / dt) does not remove the time
    error: the standard stepper's solution oscillates at omega, not at wt."""
    prob = Problem(2, (20, 16), bc=(DIRICHLET, DIRICHLET, DIRICHLET, FREE))
    op = Operator(prob, *_media(prob, 11))
    wh = S.WaveHoltz(op, 6.3, scheme=S.STANDARD)
    wt = 2.0 * math.sin(0.5 * 6.3 * wh.dt) / wh.dt
    t = wh.dt * np.arange(wh.nt + 1)
    wh.weights = wh.weights * np.cos(6.3 * t) / np.cos(wt * t)
    f = np.random.default_rng(1).standard_normal(op.ndof)
    v = direct.solve(op, 6.3, f)
    assert np.abs(wh.apply_filter(v, f) - v).max() > 1e-6 * np.abs(v).max()
