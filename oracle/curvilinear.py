"""Finite differences on a mapped 2-D grid (oracle; test infrastructure only).

What the paper fixes (Sec. 4.1): for a smooth one-to-one map (q, r) in
[0, 1]^2 -> (x, y) with Jacobian J = x_q y_r - x_r y_q, the elastic wave
equation is written in conservation form on the unit square,
    J rho u_tt = d_q[J (q_x s_xx + q_y s_xy)] + d_r[J (r_x s_xx + r_y s_xy)]
    J rho v_tt = d_q[J (q_x s_yx + q_y s_yy)] + d_r[J (r_x s_yx + r_y s_yy)],
s the stress of the isotropic medium, and discretised on a uniform (q, r)
grid by an energy-conserving scheme  rho J u_h'' = L_h u_h  whose stencils
the paper leaves to another publication.

Reading taken here (the Cartesian reading of operator.py carried over):

* With U = (u, v) and g_q = grad q, g_r = grad r, J times the stress
  divergence is  sum_{a, b in {q, r}} d_a (K^{ab} d_b U)  with the 2x2 blocks
      K^{ab} = J [lam g_a g_b^T + mu (g_a . g_b) I + mu g_b g_a^T],
  so K^{ba} = (K^{ab})^T and the 4x4 matrix [[K^qq, K^qr], [K^rq, K^rr]] is
  the (positive semi-definite) elasticity tensor seen in (q, r).
* Discrete energy
      E_h = 1/2 sum_{q-edges} (D+q U)^T Kbar^qq (D+q U)
          + 1/2 sum_{r-edges} (D+r U)^T Kbar^rr (D+r U)
          + sum_{unknown nodes} (D0q U)^T K^qr (D0r U),
  Kbar the two-point mean over the edge, and L_h = -grad E_h; inside it is
      D+q(Kbar^qq D-q U) + D+r(Kbar^rr D-r U) + D0q(K^qr D0r U) + D0r(K^rq D0q U).
  E_h >= 0 because the mean of the two one-sided quadratic forms at a node
  bounds the central one (convexity), so the scheme conserves a non-negative
  discrete energy, as the paper requires.
* Metric terms: x_q, x_r, y_q, y_r by second-order differences of the node
  coordinates (central inside, one-sided over three nodes on the edges of
  the square); J g_q = (y_r, -x_r), J g_r = (-y_q, x_q).
* Mass rho J, forcing J f:  rho J u'' = L_h u - J f cos(omega t).  In the
  Operator convention of operator.py (rho u'' = Ltilde u - f cos) this is
  Ltilde = W^-1 L_h with node weight W = J w_p and M = W rho.
* Boundary: homogeneous Dirichlet on the q sides; Dirichlet (default; the
  annular-sector experiments of Sec. 5.5 state no boundary condition and
  the rectangle beside them is Dirichlet) or traction-free on each r side
  (the free curved surfaces of the toroidal shell of Sec. 5.11, in 2-D).  A
  free side is closed from the same energy as on Cartesian grids (reading of
  operator.py): trapezoid weight w_p = 1/2 for its nodes and for the q-edges
  lying in it, and the one-sided r difference into the domain in place of
  D0r in its cross terms; traction-free is the natural boundary condition.

Parity: pinned by the reduction to the Cartesian operator for a scaled
identity map, exact rotation equivariance, symmetry and semi-definiteness,
the agreement of the energy Hessian with the stencil form, second-order
convergence of the truncation error and of the Helmholtz solution against a
continuous manufactured solution on the quarter annulus, and the paper's
observation that the iteration count on the annular sectors matches the
rectangle's (Sec. 5.5).  The paper's own closure differs and prints no
numbers for these grids, so absolute values are otherwise "parity unpinned".
"""

import numpy as np
import scipy.sparse as sp

from .operator import _edges, forward_difference, node_difference
from .problem import DIRICHLET, FREE, Problem  # noqa: F401


def _diff(f, h, axis):
    """Second-order derivative of node values along a NumPy axis: central
    inside, one-sided three-point at both ends."""
    f = np.moveaxis(np.asarray(f, np.float64), axis, 0)
    g = np.empty_like(f)
    g[1:-1] = (f[2:] - f[:-2]) / (2.0 * h)
    g[0] = (-3.0 * f[0] + 4.0 * f[1] - f[2]) / (2.0 * h)
    g[-1] = (3.0 * f[-1] - 4.0 * f[-2] + f[-3]) / (2.0 * h)
    return np.moveaxis(g, 0, axis)


def metric(x, y, hq, hr):
    """J and the scaled contravariant vectors Gq = J grad q, Gr = J grad r at
    every node.  x, y: node coordinates of shape (n_r + 1, n_q + 1), q along
    the last NumPy axis."""
    xq, yq = _diff(x, hq, 1), _diff(y, hq, 1)
    xr, yr = _diff(x, hr, 0), _diff(y, hr, 0)
    J = xq * yr - xr * yq
    if not np.all(J > 0):
        raise ValueError("the map must be one-to-one and orientation preserving (J > 0)")
    Gq = np.stack([yr, -xr])
    Gr = np.stack([-yq, xq])
    return J, Gq, Gr


def blocks(J, Gq, Gr, lam, mu):
    """K^qq, K^qr, K^rr as arrays of shape (2, 2, *node_shape):
    K^ab = (1/J) [lam Ga Gb^T + mu (Ga . Gb) I + mu Gb Ga^T]."""
    def K(Ga, Gb):
        dot = Ga[0] * Gb[0] + Ga[1] * Gb[1]
        out = np.empty((2, 2) + J.shape)
        for i in range(2):
            for k in range(2):
                out[i, k] = lam * Ga[i] * Gb[k] + mu * Gb[i] * Ga[k] + (mu * dot if i == k else 0.0)
        return out / J
    return K(Gq, Gq), K(Gq, Gr), K(Gr, Gr)


class MappedOperator:
    """L_h, M and Ltilde = J^-1 L_h on a mapped grid, restricted to the
    unknown (interior) dofs; the same interface as operator.Operator, so the
    filter, the Krylov solvers and the direct solve apply unchanged.

    x, y, rho, lam, mu: node arrays of shape (n_r + 1, n_q + 1); bc: the
    sides (-q, +q, -r, +r), q sides Dirichlet, r sides DIRICHLET or FREE."""

    def __init__(self, x, y, rho, lam, mu, bc=(DIRICHLET,) * 4):
        x = np.asarray(x, np.float64)
        shape = x.shape
        nr, nq = shape[0] - 1, shape[1] - 1
        if bc[0] != DIRICHLET or bc[1] != DIRICHLET:
            raise ValueError("the q sides must be Dirichlet")
        self.prob = Problem(2, (nq, nr), length=(1.0, 1.0), bc=tuple(bc))
        self.hq, self.hr = 1.0 / nq, 1.0 / nr
        self.rho = np.broadcast_to(np.asarray(rho, np.float64), shape).copy()
        self.lam = np.broadcast_to(np.asarray(lam, np.float64), shape).copy()
        self.mu = np.broadcast_to(np.asarray(mu, np.float64), shape).copy()
        if not (np.all(self.rho > 0) and np.all(self.lam > 0) and np.all(self.mu > 0)):
            raise ValueError("rho, lambda, mu must be positive")
        self.J, self.Gq, self.Gr = metric(x, np.asarray(y, np.float64), self.hq, self.hr)
        self.Kqq, self.Kqr, self.Krr = blocks(self.J, self.Gq, self.Gr, self.lam, self.mu)
        prob = self.prob
        keep = prob.dof_mask().ravel()
        Kfull = self.stiffness()
        self.Lh = (-Kfull[keep][:, keep]).tocsr()
        self.w = prob.gather(np.broadcast_to(self.J * prob.node_weight(), prob.field_shape))
        self.rho_dof = prob.gather(np.broadcast_to(self.rho, prob.field_shape))
        self.m = self.w * self.rho_dof
        self.Lt = (sp.diags(1.0 / self.w) @ self.Lh).tocsr()
        self.ndof = int(keep.sum())

    # ---- assembly from the energy -------------------------------------------
    def stiffness(self):
        """Hessian of E_h over all node dofs (component-major), Dirichlet
        nodes included."""
        prob = self.prob
        n = self.J.size
        B = [[sp.csr_matrix((n, n)) for _ in range(2)] for _ in range(2)]
        for axis, Kn in ((0, self.Kqq), (1, self.Krr)):
            lo, hi, we = _edges(prob, axis)
            D = forward_difference(prob, axis)
            for c in range(2):
                for e in range(2):
                    k = Kn[c, e].ravel()
                    B[c][e] = B[c][e] + D.T @ sp.diags(we * 0.5 * (k[lo] + k[hi])) @ D
        wn = (prob.node_weight() * prob.unknown_mask()).ravel()
        Dq, Dr = node_difference(prob, 0), node_difference(prob, 1)     # D0q, Dhat_r
        for c in range(2):
            for e in range(2):
                C = Dq.T @ sp.diags(wn * self.Kqr[c, e].ravel()) @ Dr     # w (D0q u_c) K_ce (Dhat_r u_e)
                B[c][e] = B[c][e] + C
                B[e][c] = B[e][c] + C.T
        return sp.bmat(B, format="csr")

    def energy(self, full):
        """E_h of a full node field (2, n_r + 1, n_q + 1), term by term."""
        prob = self.prob
        U = [np.asarray(full[c], np.float64).ravel() for c in range(2)]
        E = 0.0
        for axis, Kn in ((0, self.Kqq), (1, self.Krr)):
            lo, hi, we = _edges(prob, axis)
            h = prob.h[axis]
            g = [(U[c][hi] - U[c][lo]) / h for c in range(2)]
            for c in range(2):
                for e in range(2):
                    k = Kn[c, e].ravel()
                    E += 0.5 * float(np.sum(we * 0.5 * (k[lo] + k[hi]) * g[c] * g[e]))
        wn = (prob.node_weight() * prob.unknown_mask()).ravel()
        Dq, Dr = node_difference(prob, 0), node_difference(prob, 1)
        dq = [Dq @ U[c] for c in range(2)]
        dr = [Dr @ U[c] for c in range(2)]
        for c in range(2):
            for e in range(2):
                E += float(np.sum(wn * self.Kqr[c, e].ravel() * dq[c] * dr[e]))
        return E

    # ---- interface shared with operator.Operator ------------------------------
    def apply_Ltilde(self, x):
        return self.Lt @ x

    def gershgorin(self):
        """max over unknown rows of sum_j |(rho^-1 Ltilde)_ij|."""
        rows = np.asarray(abs(self.Lt).sum(axis=1)).ravel() / self.rho_dof
        return float(rows.max())


def lh_stencil(x, y, lam, mu, U):
    """L_h U at the interior nodes written out as the stencil (zeros on the
    boundary), with U = (u, v) of shape (2, n_r + 1, n_q + 1) and zero
    boundary values (all sides Dirichlet): a second statement of the operator
    that needs no matrix (it reaches the largest grids)."""
    x = np.asarray(x, np.float64)
    nr, nq = x.shape[0] - 1, x.shape[1] - 1
    hq, hr = 1.0 / nq, 1.0 / nr
    J, Gq, Gr = metric(x, np.asarray(y, np.float64), hq, hr)
    Kqq, Kqr, Krr = blocks(J, Gq, Gr, np.broadcast_to(lam, J.shape), np.broadcast_to(mu, J.shape))
    U = np.asarray(U, np.float64)
    I = (slice(1, -1), slice(1, -1))

    def at(a, dj, di):
        return a[..., 1 + dj:a.shape[-2] - 1 + dj, 1 + di:a.shape[-1] - 1 + di]

    def mv(K, V):
        return np.einsum("ik...,k...->i...", K, V)

    C = U[(slice(None),) + I]
    out = np.zeros_like(U)
    Kp, Km = 0.5 * (at(Kqq, 0, 1) + Kqq[..., 1:-1, 1:-1]), 0.5 * (Kqq[..., 1:-1, 1:-1] + at(Kqq, 0, -1))
    acc = (mv(Kp, at(U, 0, 1) - C) - mv(Km, C - at(U, 0, -1))) / hq ** 2
    Kp, Km = 0.5 * (at(Krr, 1, 0) + Krr[..., 1:-1, 1:-1]), 0.5 * (Krr[..., 1:-1, 1:-1] + at(Krr, -1, 0))
    acc += (mv(Kp, at(U, 1, 0) - C) - mv(Km, C - at(U, -1, 0))) / hr ** 2
    # D0q(K^qr D0r U): K^qr at (j, i +- 1) times the r-difference there
    acc += (mv(at(Kqr, 0, 1), at(U, 1, 1) - at(U, -1, 1))
            - mv(at(Kqr, 0, -1), at(U, 1, -1) - at(U, -1, -1))) / (4 * hq * hr)
    # D0r(K^rq D0q U), K^rq = (K^qr)^T, at (j +- 1, i)
    KrqN = np.swapaxes(at(Kqr, 1, 0), 0, 1)
    KrqS = np.swapaxes(at(Kqr, -1, 0), 0, 1)
    acc += (mv(KrqN, at(U, 1, 1) - at(U, 1, -1)) - mv(KrqS, at(U, -1, 1) - at(U, -1, -1))) / (4 * hq * hr)
    out[(slice(None),) + I] = acc
    return out
