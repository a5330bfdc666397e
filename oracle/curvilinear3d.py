"""Finite differences on a mapped 3-D grid (oracle; test infrastructure only).

What the paper fixes (Sec. 4.1): for a smooth one-to-one map of the unit
cube (q, r, s) -> (x, y, z) with Jacobian J, the elastic wave equation is
written in conservation form on the cube,
    J rho u_tt = sum_a d_a [ J sum_k (grad a)_k sigma_{k .} ],
and discretised on a uniform (q, r, s) grid by an energy-conserving scheme
rho J u_h'' = L_h u_h whose stencils the paper leaves to another
publication.  Its 3-D curvilinear experiment is the partial toroidal shell
of Sec. 5.11: free surfaces on the two radial faces, Dirichlet elsewhere.

Reading taken here -- the 2-D reading of curvilinear.py carried to three
axes:

* With U = (u, v, w), G_a = J grad a (a in {q, r, s}; G_q = x_r x x_s,
  G_r = x_s x x_q, G_s = x_q x x_r with x_a the column dx/da), J times the
  stress divergence is sum_{a, b} d_a (K^{ab} d_b U) with the 3x3 blocks
      K^{ab} = (1/J) [lam G_a G_b^T + mu (G_a . G_b) I + mu G_b G_a^T],
  K^{ba} = (K^{ab})^T; the 9x9 matrix of the nine blocks is the
  elasticity tensor seen in (q, r, s) (positive semi-definite).
* Discrete energy
      E_h = 1/2 sum_a sum_{a-edges} w_e (D+a U)^T Kbar^aa (D+a U)
          + sum_{a < b} sum_{unknown nodes} w_n (Dh_a U)^T K^{ab} (Dh_b U),
  Kbar the two-point mean over the edge, Dh the central difference (the
  one-sided difference into the domain on a free face), w the trapezoid
  weights (1/2 per free face a node or an edge lies on); L_h = -grad E_h.
  Inside, L_h is sum_a D+a(Kbar^aa D-a U) + sum_{a != b} D0a(K^ab D0b U).
* Metric terms by second-order differences of the node coordinates
  (central inside, one-sided over three nodes on the faces of the cube).
* Mass rho J, forcing J f: with node weight W = J w and M = W rho the
  semi-discrete system is M u'' = L_h u - W f cos(omega t), the Operator
  convention of operator.py.
* Faces: the q and r faces are Dirichlet; each s face is Dirichlet or
  traction-free (the free radial surfaces of the toroidal shell).

Parity: pinned by the reduction to the Cartesian 3-D operator for a scaled
identity map, exact rotation equivariance, symmetry and semi-definiteness,
translations in the kernel of the full Hessian, second-order convergence of
the interior truncation error against the continuous stress divergence on a
section of the torus (node coordinates from inputs.torus_section), and the
exact WaveHoltz fixed point (Sec. 4.3).  The
paper's own closure is another publication's and prints no values for these
grids (only CR iteration counts, Sec. 5.11), so absolute values are
otherwise "parity unpinned".
"""

import numpy as np
import scipy.sparse as sp

from .curvilinear import _diff
from .operator import _edges, forward_difference, node_difference
from .problem import DIRICHLET, FREE, Problem  # noqa: F401


def metric3(x, y, z, hq, hr, hs):
    """J and G = (G_q, G_r, G_s), each (3, *node_shape), from node
    coordinates of shape (n_s + 1, n_r + 1, n_q + 1) (q along the last NumPy
    axis, s along the first)."""
    X = [np.asarray(c, np.float64) for c in (x, y, z)]
    xq = np.stack([_diff(c, hq, 2) for c in X])
    xr = np.stack([_diff(c, hr, 1) for c in X])
    xs = np.stack([_diff(c, hs, 0) for c in X])
    Gq = np.cross(xr, xs, axis=0)
    Gr = np.cross(xs, xq, axis=0)
    Gs = np.cross(xq, xr, axis=0)
    J = np.sum(xq * Gq, axis=0)
    if not np.all(J > 0):
        raise ValueError("the map must be one-to-one and orientation preserving (J > 0)")
    return J, (Gq, Gr, Gs)


def block(J, Ga, Gb, lam, mu):
    """K^{ab} as an array (3, 3, *node_shape)."""
    dot = np.sum(Ga * Gb, axis=0)
    out = lam * Ga[:, None] * Gb[None, :] + mu * Gb[:, None] * Ga[None, :]
    for i in range(3):
        out[i, i] = out[i, i] + mu * dot
    return out / J


class MappedOperator3D:
    """L_h, M and Ltilde = W^-1 L_h on a mapped 3-D grid restricted to the
    unknown dofs; the interface of operator.Operator, so the filter, the
    Krylov solvers and the direct solve apply unchanged.

    x, y, z, rho, lam, mu: node arrays of shape (n_s + 1, n_r + 1, n_q + 1);
    bc: the faces (-q, +q, -r, +r, -s, +s), q and r faces DIRICHLET, s faces
    DIRICHLET or FREE."""

    def __init__(self, x, y, z, rho, lam, mu, bc=(DIRICHLET,) * 6):
        x = np.asarray(x, np.float64)
        shape = x.shape
        ns, nr, nq = (k - 1 for k in shape)
        if any(bc[f] != DIRICHLET for f in range(4)):
            raise ValueError("the q and r faces must be Dirichlet")
        self.prob = Problem(3, (nq, nr, ns), length=(1.0, 1.0, 1.0), bc=tuple(bc))
        self.h = (1.0 / nq, 1.0 / nr, 1.0 / ns)
        self.rho = np.broadcast_to(np.asarray(rho, np.float64), shape).copy()
        self.lam = np.broadcast_to(np.asarray(lam, np.float64), shape).copy()
        self.mu = np.broadcast_to(np.asarray(mu, np.float64), shape).copy()
        if not (np.all(self.rho > 0) and np.all(self.lam > 0) and np.all(self.mu > 0)):
            raise ValueError("rho, lambda, mu must be positive")
        self.J, self.G = metric3(x, y, z, *self.h)
        self.K = [[block(self.J, self.G[a], self.G[b], self.lam, self.mu) for b in range(3)] for a in range(3)]
        prob = self.prob
        keep = prob.dof_mask().ravel()
        self.Kfull = self.stiffness()
        self.Lh = (-self.Kfull[keep][:, keep]).tocsr()
        self.w = prob.gather(np.broadcast_to(self.J * prob.node_weight(), prob.field_shape))
        self.rho_dof = prob.gather(np.broadcast_to(self.rho, prob.field_shape))
        self.m = self.w * self.rho_dof
        self.Lt = (sp.diags(1.0 / self.w) @ self.Lh).tocsr()
        self.ndof = int(keep.sum())

    def stiffness(self):
        """Hessian of E_h over all node dofs (component-major), Dirichlet
        nodes included."""
        prob = self.prob
        n = self.J.size
        B = [[sp.csr_matrix((n, n)) for _ in range(3)] for _ in range(3)]
        for a in range(3):
            lo, hi, we = _edges(prob, a)
            D = forward_difference(prob, a)
            Kaa = self.K[a][a]
            for c in range(3):
                for e in range(3):
                    k = Kaa[c, e].ravel()
                    B[c][e] = B[c][e] + D.T @ sp.diags(we * 0.5 * (k[lo] + k[hi])) @ D
        wn = (prob.node_weight() * prob.unknown_mask()).ravel()
        Dh = [node_difference(prob, a) for a in range(3)]
        for a in range(3):
            for b in range(a + 1, 3):
                Kab = self.K[a][b]
                for c in range(3):
                    for e in range(3):
                        C = Dh[a].T @ sp.diags(wn * Kab[c, e].ravel()) @ Dh[b]   # w (Dh_a u_c) K_ce (Dh_b u_e)
                        B[c][e] = B[c][e] + C
                        B[e][c] = B[e][c] + C.T
        return sp.bmat(B, format="csr")

    def apply_Ltilde(self, x):
        return self.Lt @ x

    def gershgorin(self):
        """max over unknown rows of sum_j |(rho^-1 Ltilde)_ij|."""
        rows = np.asarray(abs(self.Lt).sum(axis=1)).ravel() / self.rho_dof
        return float(rows.max())
