"""Pins of the oracle's spatial operator against facts fixed by the paper or
by the mathematics (CPU only)."""

import math

import numpy as np
import pytest

from oracle import operator as O
from oracle.problem import DIRICHLET, FREE, Problem
from paper_2205_12344_amd import inputs


def _random_media(prob, seed):
    rng = np.random.default_rng(seed)
    s = prob.node_shape
    rho = np.exp(0.3 * rng.standard_normal(s))
    mu = np.exp(0.3 * rng.standard_normal(s))
    lam = mu * np.exp(0.3 * rng.standard_normal(s)) * 2
    return rho, lam, mu


CASES = [
    Problem(2, (9, 7)),
    Problem(2, (10, 8), bc=(DIRICHLET, DIRICHLET, DIRICHLET, FREE)),
    Problem(2, (8, 9), bc=(DIRICHLET, DIRICHLET, FREE, FREE)),
    Problem(3, (5, 4, 6)),
    Problem(3, (5, 5, 4), bc=(DIRICHLET,) * 4 + (FREE, FREE)),
]


@pytest.mark.parametrize("prob", CASES, ids=lambda p: f"d{p.dim}_{p.bc}")
def test_symmetric_negative_definite(prob):
    """Sec. 4.1: L_h symmetric; energy-conserving BCs make -L_h >= 0 (here
    definite since every component has a Dirichlet face)."""
    op = O.Operator(prob, *_random_media(prob, 1))
    L = op.Lh.toarray()
    assert np.abs(L - L.T).max() <= 1e-14 * np.abs(L).max()
    ev = np.linalg.eigvalsh(L)
    assert ev.max() < 0


@pytest.mark.parametrize("prob", CASES, ids=lambda p: f"d{p.dim}_{p.bc}")
def test_quadratic_form_is_energy(prob):
    """1/2 u^T K u equals the energy summed term by term."""
    rho, lam, mu = _random_media(prob, 2)
    K = O.stiffness(prob, lam, mu)
    u = np.random.default_rng(3).standard_normal(prob.field_shape) * prob.unknown_mask()
    uv = u.ravel()
    assert 0.5 * uv @ (K @ uv) == pytest.approx(O.energy(prob, lam, mu, u), rel=1e-12)


def _c2_stencil_2d(u, v, lam, mu, h):
    """The interior second-order stencil written out directly:
    D+x(Abar D-x u) + D+y(mubar D-y u) + D0x(lam D0y v) + D0y(mu D0x v), and
    the v-row with the roles of the coefficients exchanged."""
    hx, hy = h
    A = lam + 2 * mu
    c = (slice(1, -1), slice(1, -1))

    def sh(a, dj, di):
        ny, nx = a.shape
        return a[1 + dj:ny - 1 + dj, 1 + di:nx - 1 + di]

    def compact(w, cx, cy):
        fxp = 0.5 * (sh(cx, 0, 1) + cx[c]) * (sh(w, 0, 1) - w[c])
        fxm = 0.5 * (sh(cx, 0, -1) + cx[c]) * (w[c] - sh(w, 0, -1))
        fyp = 0.5 * (sh(cy, 1, 0) + cy[c]) * (sh(w, 1, 0) - w[c])
        fym = 0.5 * (sh(cy, -1, 0) + cy[c]) * (w[c] - sh(w, -1, 0))
        return (fxp - fxm) / hx ** 2 + (fyp - fym) / hy ** 2

    def mixed(w, cxy, cyx):
        # D0x(cxy D0y w) + D0y(cyx D0x w)
        t1 = (sh(cxy, 0, 1) * (sh(w, 1, 1) - sh(w, -1, 1))
              - sh(cxy, 0, -1) * (sh(w, 1, -1) - sh(w, -1, -1))) / (4 * hx * hy)
        t2 = (sh(cyx, 1, 0) * (sh(w, 1, 1) - sh(w, 1, -1))
              - sh(cyx, -1, 0) * (sh(w, -1, 1) - sh(w, -1, -1))) / (4 * hx * hy)
        return t1 + t2

    Lu = compact(u, A, mu) + mixed(v, lam, mu)
    Lv = compact(v, mu, A) + mixed(u, mu, lam)
    return Lu, Lv


def test_interior_matches_conservative_stencil():
    """The energy Hessian reproduces the standard conservative stencil of the
    Cartesian specialisation of the equations in Sec. 4.1 on variable media."""
    prob = Problem(2, (12, 10), length=(1.0, 0.8))
    rho, lam, mu = _random_media(prob, 4)
    op = O.Operator(prob, rho, lam, mu)
    u = np.random.default_rng(5).standard_normal(prob.field_shape) * prob.unknown_mask()
    Lt = prob.scatter(op.apply_Ltilde(prob.gather(u)))
    Lu, Lv = _c2_stencil_2d(u[0], u[1], lam, mu, prob.h)
    np.testing.assert_allclose(Lt[0][1:-1, 1:-1], Lu, rtol=0, atol=1e-11 * np.abs(Lu).max())
    np.testing.assert_allclose(Lt[1][1:-1, 1:-1], Lv, rtol=0, atol=1e-11 * np.abs(Lv).max())


def _div_stress_const(grad2, lam, mu, d):
    """div T(u) for constant lam, mu from second derivatives grad2[c][a][b]."""
    out = []
    for c in range(d):
        s = 0.0
        for a in range(d):
            s = s + mu * grad2[c][a][a] + (lam + mu) * grad2[a][a][c]
        out.append(s)
    return out


@pytest.mark.parametrize("dim", [2, 3])
def test_exact_on_quadratics(dim):
    """Second-order central stencils are exact on quadratic fields: with
    constant coefficients, (Ltilde u)_c = mu Lap u_c + (lam + mu) d_c div u
    exactly at nodes two or more cells from the boundary."""
    n = (8, 7, 6)[:dim]
    prob = Problem(dim, n, length=(1.0, 1.3, 0.9)[:dim])
    lam, mu = 1.7, 0.6
    X = prob.mesh()
    rng = np.random.default_rng(6)
    Q = rng.standard_normal((dim, dim, dim))
    Q = 0.5 * (Q + Q.transpose(0, 2, 1))          # u_c = x^T Q_c x + g_c . x
    g = rng.standard_normal((dim, dim))
    u = np.array([sum(Q[c, a, b] * X[a] * X[b] for a in range(dim) for b in range(dim))
                  + sum(g[c, a] * X[a] for a in range(dim)) for c in range(dim)])
    K = O.stiffness(prob, lam, mu)
    Lu = -(K @ u.ravel()).reshape(u.shape)         # all-dof rows, h^d dropped
    grad2 = [[[2 * Q[c, a, b] for b in range(dim)] for a in range(dim)] for c in range(dim)]
    exact = _div_stress_const(grad2, lam, mu, dim)
    core = (slice(None),) + (slice(2, -2),) * dim
    np.testing.assert_allclose(Lu[core], np.broadcast_to(np.array(exact).reshape((dim,) + (1,) * dim),
                                                         Lu[core].shape), rtol=1e-10, atol=1e-9)


@pytest.mark.parametrize("dim", [2, 3])
def test_free_surface_traction_of_linear_fields(dim):
    """For a linear displacement with constant coefficients the stress sigma is
    constant; interior rows vanish and a free-face row equals the boundary
    flux -sigma.n / (w_node h), i.e. -(2/h) sigma n on a face: the discrete
    form of the natural (traction) boundary term of the energy."""
    n = (6, 7, 5)[:dim]
    bc = [DIRICHLET] * (2 * dim)
    bc[2 * (dim - 1) + 1] = FREE                     # free top face of the last axis
    prob = Problem(dim, n, bc=tuple(bc))
    lam, mu = 2.3, 0.7
    X = prob.mesh()
    G = np.random.default_rng(7).standard_normal((dim, dim))      # u_c = G[c] . x
    u = np.array([sum(G[c, a] * X[a] for a in range(dim)) for c in range(dim)])
    eps = 0.5 * (G + G.T)
    sigma = lam * np.trace(G) * np.eye(dim) + 2 * mu * eps
    K = O.stiffness(prob, lam, mu)
    wn = prob.node_weight()
    Lu = -(K @ u.ravel()).reshape(u.shape) / wn     # Ltilde on all nodes
    top = dim - 1
    k = prob.npaxis(top)
    # rows two or more cells from every Dirichlet face (their stencils see no
    # Dirichlet node, where the field is not zero)
    interior = [slice(None)] + [slice(2, -2)] * dim
    interior[1 + k] = slice(2, -1)
    np.testing.assert_allclose(Lu[tuple(interior)], 0.0, atol=1e-9)
    face = [slice(None)] + [slice(2, -2)] * dim
    face[1 + k] = slice(-1, None)
    nrm = np.zeros(dim)
    nrm[top] = 1.0
    traction = sigma @ nrm
    expect = -(2.0 / prob.h[top]) * traction
    got = Lu[tuple(face)]
    for c in range(dim):
        np.testing.assert_allclose(got[c], expect[c], rtol=1e-10, atol=1e-9)


@pytest.mark.parametrize("prob", [CASES[1], CASES[2], CASES[4]], ids=["free_top", "free_tb", "free3d"])
def test_rigid_motions_in_null_space(prob):
    """Rows not adjacent to a Dirichlet face annihilate translations (any
    medium) and, for constant coefficients, the rotation (-y, x)."""
    lam, mu = 1.9, 0.8
    rho, vlam, vmu = _random_media(prob, 8)
    X = prob.mesh()
    d = prob.dim
    # rows whose stencil touches no Dirichlet node
    far = np.ones(prob.node_shape, bool)
    for a in range(d):
        k = prob.npaxis(a)
        for s in (0, 1):
            if prob.face_bc(a, s) == DIRICHLET:
                idx = [slice(None)] * d
                idx[k] = slice(0, 2) if s == 0 else slice(-2, None)
                far[tuple(idx)] = False
    assert far.any()
    for coefs, fields in [((vlam, vmu), [np.eye(d)[c] for c in range(d)]),
                          ((lam, mu), ["rot"])]:
        K = O.stiffness(prob, *coefs)
        for fdir in fields:
            if isinstance(fdir, str):
                u = np.zeros(prob.field_shape)
                u[0], u[1] = -X[1], X[0]
            else:
                u = np.array([np.full(prob.node_shape, fdir[c]) for c in range(d)])
            Lu = -(K @ u.ravel()).reshape(u.shape)
            assert np.abs(Lu[:, far]).max() <= 1e-9 * max(1.0, np.abs(K).max())


@pytest.mark.parametrize("dim,closed", [(2, lambda l, m: 4 * (l + 3 * m)), (3, lambda l, m: 4 * (l + 4 * m))])
def test_spectral_radius_constant_medium(dim, closed):
    """Constant medium, Dirichlet box: the largest eigenvalue of M^-1(-L_h)
    is bounded by the symbol maximum 4(lam+3mu)/(rho h^2) in 2-D
    (4(lam+4mu) in 3-D) and approaches it; the 2-D value gives the leapfrog
    limit dt = h / sqrt(lam + 3 mu), the CFL of the FD runs of Sec. 5.1."""
    import scipy.sparse.linalg as spl
    n = 40 if dim == 2 else 14
    prob = Problem(dim, (n,) * dim)
    lam, mu, rho = 2.0, 1.0, 1.3
    op = O.Operator(prob, rho, lam, mu)
    ev = spl.eigsh(-op.Lh, k=1, M=None, which="LA", tol=1e-10)[0][0] / (rho * 1.0)
    bound = closed(lam, mu) / (rho * prob.h[0] ** 2)
    assert ev <= bound * (1 + 1e-12)
    assert ev >= bound * (0.985 if dim == 2 else 0.93)


@pytest.mark.parametrize("dim,closed", [(2, lambda l, m: 5 * l + 13 * m), (3, lambda l, m: 6 * l + 18 * m)])
def test_gershgorin_constant_medium(dim, closed):
    """Gershgorin row sum of rho^-1 Ltilde for a constant medium, in closed
    form: every stencil entry of an interior row counted once."""
    n = 8 if dim == 2 else 5
    prob = Problem(dim, (n,) * dim)
    lam, mu, rho = 2.0, 1.0, 1.5
    op = O.Operator(prob, rho, lam, mu)
    assert op.gershgorin() == pytest.approx(closed(lam, mu) / (rho * prob.h[0] ** 2), rel=1e-13)


def test_inputs_are_sane():
    c1 = inputs.constant_square64()
    assert c1.f.shape == (2, 65, 65) and c1.f[1].max() == 0
    c2 = inputs.random_square(n=64)
    assert c2.rho.shape == (65, 65) and np.all(c2.lam >= c2.mu * 0.999999) and np.all(c2.lam <= 3 * c2.mu * 1.000001)
    assert c2.omega > 0


@pytest.mark.parametrize("dim,n", [(2, (11, 9)), (3, (6, 7, 5))])
def test_slice_stencil_matches_energy_assembly(dim, n):
    """The slice form used for the largest grids equals the assembled operator
    on all-Dirichlet boxes with variable media."""
    from oracle.stencil import ltilde_dirichlet
    prob = Problem(dim, n, length=(1.0, 0.8, 1.2)[:dim])
    rho, lam, mu = _random_media(prob, 21)
    op = O.Operator(prob, rho, lam, mu)
    u = np.random.default_rng(22).standard_normal(prob.field_shape) * prob.unknown_mask()
    ref = prob.scatter(op.apply_Ltilde(prob.gather(u)))
    got = ltilde_dirichlet(prob.h, lam, mu, u)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-11 * np.abs(ref).max())
