"""Discrete stress divergence L_h from a discrete elastic energy (oracle).

Test infrastructure only.  What the paper fixes, and the reading taken here:

* Sec. 4.1 writes the semi-discrete system as M u'' = L_h u with M diagonal
  and L_h symmetric after a diagonal scaling Lambda (x2 on free sides, x4
  where free sides meet), and states that the scheme conserves a discrete
  energy.  The exact stencils are deferred to another publication.
* Reading: on the Cartesian grid L_h is minus the Hessian of a discrete
  strain energy E_h(u) = 1/2 u^T K u, built with the trapezoid rule:

    edge terms   1/2 w_e [ Abar (D+_a u_a)^2 + mubar (D+_a u_c)^2 (c != a) ]
    node terms   w_p [ lam (Dh_a u_a)(Dh_b u_b) + mu (Dh_b u_a)(Dh_a u_b) ]
                 for every axis pair a < b, at unknown nodes only

  with A = lam + 2 mu, bars the arithmetic mean over the edge's two nodes,
  D+ the forward difference over an edge, Dh the central difference in the
  interior and the one-sided difference into the domain on a free face, and
  w_e, w_p the trapezoid weights (1/2 per free face an edge or node lies
  on).  This is the continuous energy density
  1/2 A (sum u_a,a^2) + lam sum_{a<b} u_a,a u_b,b + 1/2 mu sum_{a != b} u_a,b^2
  + mu sum_{a<b} u_a,b u_b,a, discretised term by term.
* In the interior the Hessian reproduces the standard conservative
  second-order stencil  D+x(Abar D-x u) + D+y(mubar D-y u) + D0x(lam D0y v)
  + D0y(mu D0x v) (and its cyclic 3-D analogue); traction-free is the
  natural boundary condition of the energy, and K is symmetric positive
  semi-definite by construction.

Parity: the interior operator is pinned by the manufactured-solution
convergence rates of Table 1 and by exactness on quadratic fields; the
free-surface closure is pinned only by invariants (symmetry, translation and
rotation null space, the traction of linear fields, manufactured convergence)
-- its absolute values are otherwise "parity unpinned".
"""

import numpy as np
import scipy.sparse as sp

from .problem import FREE, Problem


def _node_index(prob: Problem):
    return np.arange(int(np.prod(prob.node_shape))).reshape(prob.node_shape)


def _slab(arr, k, sl):
    idx = [slice(None)] * arr.ndim
    idx[k] = sl
    return arr[tuple(idx)]


def _edges(prob: Problem, a):
    """Endpoint node indices (lo, hi) of every grid edge along axis a, and the
    edge trapezoid weight (1/2 per free face of another axis it lies on)."""
    k = prob.npaxis(a)
    ni = _node_index(prob)
    lo = _slab(ni, k, slice(0, -1)).ravel()
    hi = _slab(ni, k, slice(1, None)).ravel()
    w = np.ones(prob.node_shape)
    for b in range(prob.dim):
        if b == a:
            continue
        for s in (0, 1):
            if prob.face_bc(b, s) == FREE:
                w = np.where(prob.on_face(b, s), 0.5 * w, w)
    return lo, hi, w.ravel()[lo]


def forward_difference(prob: Problem, a):
    """D+_a : node values -> edge values along axis a."""
    lo, hi, _ = _edges(prob, a)
    ne, nn = lo.size, int(np.prod(prob.node_shape))
    h = prob.h[a]
    rows = np.concatenate([np.arange(ne), np.arange(ne)])
    cols = np.concatenate([lo, hi])
    vals = np.concatenate([-np.ones(ne) / h, np.ones(ne) / h])
    return sp.csr_matrix((vals, (rows, cols)), shape=(ne, nn))


def node_difference(prob: Problem, a):
    """Dh_a : node values -> node values.  Central difference in the interior
    of axis a; one-sided into the domain on a free face of axis a; zero on a
    Dirichlet face (such nodes are not unknowns)."""
    k = prob.npaxis(a)
    ni = _node_index(prob)
    n = prob.n[a]
    h = prob.h[a]
    rows, cols, vals = [], [], []
    mid = _slab(ni, k, slice(1, n)).ravel()
    rows += [mid, mid]
    cols += [_slab(ni, k, slice(2, n + 1)).ravel(), _slab(ni, k, slice(0, n - 1)).ravel()]
    vals += [np.full(mid.size, 0.5 / h), np.full(mid.size, -0.5 / h)]
    if prob.face_bc(a, 0) == FREE:
        p = _slab(ni, k, slice(0, 1)).ravel()
        q = _slab(ni, k, slice(1, 2)).ravel()
        rows += [p, p]
        cols += [q, p]
        vals += [np.full(p.size, 1 / h), np.full(p.size, -1 / h)]
    if prob.face_bc(a, 1) == FREE:
        p = _slab(ni, k, slice(n, n + 1)).ravel()
        q = _slab(ni, k, slice(n - 1, n)).ravel()
        rows += [p, p]
        cols += [p, q]
        vals += [np.full(p.size, 1 / h), np.full(p.size, -1 / h)]
    nn = int(np.prod(prob.node_shape))
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(nn, nn))


def stiffness(prob: Problem, lam, mu):
    """K with E_h(u) = 1/2 u^T K u over ALL node dofs (component-major,
    nodes in C order), including Dirichlet nodes; the factor h^d of the
    quadrature is omitted (it cancels against the mass matrix)."""
    d = prob.dim
    nn = int(np.prod(prob.node_shape))
    lam = np.broadcast_to(np.asarray(lam, np.float64), prob.node_shape).ravel()
    mu = np.broadcast_to(np.asarray(mu, np.float64), prob.node_shape).ravel()
    A = lam + 2.0 * mu
    blocks = [[None] * d for _ in range(d)]

    def add(i, j, m):
        blocks[i][j] = m if blocks[i][j] is None else blocks[i][j] + m

    # edge (compact) terms
    for a in range(d):
        lo, hi, we = _edges(prob, a)
        Dp = forward_difference(prob, a)
        for c in range(d):
            coef = 0.5 * (A[lo] + A[hi]) if c == a else 0.5 * (mu[lo] + mu[hi])
            add(c, c, (Dp.T @ sp.diags(we * coef) @ Dp).tocsr())
    # node (cross) terms at unknown nodes
    wn = (prob.node_weight() * prob.unknown_mask()).ravel()
    Dh = [node_difference(prob, a) for a in range(d)]
    Cl = sp.diags(wn * lam)
    Cm = sp.diags(wn * mu)
    for a in range(d):
        for b in range(a + 1, d):
            # lam (Dh_a u_a)(Dh_b u_b)
            add(a, b, (Dh[a].T @ Cl @ Dh[b]).tocsr())
            add(b, a, (Dh[b].T @ Cl @ Dh[a]).tocsr())
            # mu (Dh_b u_a)(Dh_a u_b)
            add(a, b, (Dh[b].T @ Cm @ Dh[a]).tocsr())
            add(b, a, (Dh[a].T @ Cm @ Dh[b]).tocsr())
    for i in range(d):
        for j in range(d):
            if blocks[i][j] is None:
                blocks[i][j] = sp.csr_matrix((nn, nn))
    return sp.bmat(blocks, format="csr")


def energy(prob: Problem, lam, mu, full):
    """E_h(u) evaluated term by term from the node field (no matrix)."""
    d = prob.dim
    u = [np.asarray(full[c], np.float64).ravel() for c in range(d)]
    lam = np.broadcast_to(np.asarray(lam, np.float64), prob.node_shape).ravel()
    mu = np.broadcast_to(np.asarray(mu, np.float64), prob.node_shape).ravel()
    A = lam + 2.0 * mu
    E = 0.0
    for a in range(d):
        lo, hi, we = _edges(prob, a)
        for c in range(d):
            coef = 0.5 * (A[lo] + A[hi]) if c == a else 0.5 * (mu[lo] + mu[hi])
            g = (u[c][hi] - u[c][lo]) / prob.h[a]
            E += 0.5 * np.sum(we * coef * g * g)
    wn = (prob.node_weight() * prob.unknown_mask()).ravel()
    Dh = [node_difference(prob, a) for a in range(d)]
    for a in range(d):
        for b in range(a + 1, d):
            E += np.sum(wn * lam * (Dh[a] @ u[a]) * (Dh[b] @ u[b]))
            E += np.sum(wn * mu * (Dh[b] @ u[a]) * (Dh[a] @ u[b]))
    return E


class Operator:
    """L_h, M and Ltilde = (W)^-1 L_h restricted to the unknown dofs.

    Semi-discrete system (Sec. 4.1, eq. (symmetric FD), with forcing as in
    eq. (elastic-time)):   M u'' = L_h u - W f cos(omega t),
    i.e. pointwise   rho u'' = Ltilde u - f cos(omega t),
    with M = diag(w rho), W = diag(w) (w = trapezoid node weight; the common
    factor h^d is dropped from M, L_h and W f alike).
    """

    def __init__(self, prob: Problem, rho, lam, mu):
        self.prob = prob
        shape = prob.node_shape
        self.rho = np.broadcast_to(np.asarray(rho, np.float64), shape).copy()
        self.lam = np.broadcast_to(np.asarray(lam, np.float64), shape).copy()
        self.mu = np.broadcast_to(np.asarray(mu, np.float64), shape).copy()
        if not (np.all(self.rho > 0) and np.all(self.lam > 0) and np.all(self.mu > 0)):
            raise ValueError("rho, lambda, mu must be positive")
        keep = prob.dof_mask().ravel()
        K = stiffness(prob, self.lam, self.mu)
        self.Lh = (-K[keep][:, keep]).tocsr()
        self.w = prob.gather(np.broadcast_to(prob.node_weight(), prob.field_shape))
        self.m = prob.mass_diag(self.rho)                       # w * rho per dof
        self.rho_dof = prob.gather(np.broadcast_to(self.rho, prob.field_shape))
        self.Lt = (sp.diags(1.0 / self.w) @ self.Lh).tocsr()    # Ltilde
        self.ndof = int(keep.sum())

    def apply_Ltilde(self, x):
        return self.Lt @ x

    def gershgorin(self):
        """max over unknown rows of sum_j |(rho^-1 Ltilde)_ij| -- a bound on the
        spectral radius of M^-1 (-L_h), used by the time-step rule."""
        rows = np.asarray(abs(self.Lt).sum(axis=1)).ravel() / self.rho_dof
        return float(rows.max())
