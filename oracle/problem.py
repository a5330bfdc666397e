"""Grid, boundary faces and trapezoid weights (oracle; test infrastructure only).

The paper discretises the mapped unit square/cube on a uniform grid
q_i = i h_q, i = 0..n_q (Sec. 4.1 and the grid description of Sec. 5.5).
Here the mapping is the identity scaled by the box lengths, so the grid is
Cartesian with h_a = len_a / n_a and n_a + 1 nodes per axis a.

Arrays of node values use the layout [component][z][y][x] (2-D: [c][y][x]):
NumPy axis (d - 1 - a) is coordinate axis a (a = 0 is x).

Faces are ordered -x, +x, -y, +y, -z, +z; each is DIRICHLET (homogeneous
displacement) or FREE (traction-free), the two energy-conserving conditions of
Sec. 2.1.  A node is an unknown iff it lies on no Dirichlet face; Dirichlet
nodes hold zero.  Nodes on a free face carry trapezoid weight 1/2 per free
face they lie on; this is the diagonal scaling Lambda of Sec. 4.1 (x2 on free
sides, x4 where free sides meet) seen from the quadrature side.
"""

from dataclasses import dataclass, field
from typing import Tuple

import numpy as np

DIRICHLET = 0
FREE = 1


@dataclass(frozen=True)
class Problem:
    dim: int
    n: Tuple[int, ...]                 # cells per axis (x, y[, z])
    length: Tuple[float, ...] = field(default=None)
    bc: Tuple[int, ...] = field(default=None)   # 2*dim faces: -x,+x,-y,+y[,-z,+z]

    def __post_init__(self):
        if self.dim not in (2, 3):
            raise ValueError("dim must be 2 or 3")
        if len(self.n) != self.dim or min(self.n) < 2:
            raise ValueError("need dim cell counts, each >= 2")
        if self.length is None:
            object.__setattr__(self, "length", (1.0,) * self.dim)
        if self.bc is None:
            object.__setattr__(self, "bc", (DIRICHLET,) * (2 * self.dim))
        if len(self.bc) != 2 * self.dim:
            raise ValueError("bc needs 2*dim faces")

    # ---- geometry -------------------------------------------------------
    @property
    def h(self):
        return tuple(self.length[a] / self.n[a] for a in range(self.dim))

    @property
    def vol(self):
        return float(np.prod(self.h))

    @property
    def node_shape(self):
        """NumPy shape of one component: (nz+1, ny+1, nx+1) or (ny+1, nx+1)."""
        return tuple(self.n[a] + 1 for a in reversed(range(self.dim)))

    @property
    def field_shape(self):
        return (self.dim,) + self.node_shape

    def npaxis(self, a):
        return self.dim - 1 - a

    def coords(self, a):
        """1-D node coordinates along axis a."""
        return np.arange(self.n[a] + 1) * self.h[a]

    def mesh(self):
        """Coordinate arrays X, Y[, Z] of node_shape (x varies fastest)."""
        axes = [self.coords(a) for a in reversed(range(self.dim))]
        grids = np.meshgrid(*axes, indexing="ij")
        return tuple(reversed(grids))      # (X, Y[, Z])

    # ---- face membership ------------------------------------------------
    def on_face(self, a, side):
        """Boolean node array: node lies on face (axis a, side 0=low/1=high)."""
        idx = np.arange(self.n[a] + 1)
        line = idx == (0 if side == 0 else self.n[a])
        shape = [1] * self.dim
        shape[self.npaxis(a)] = self.n[a] + 1
        return np.broadcast_to(line.reshape(shape), self.node_shape)

    def face_bc(self, a, side):
        return self.bc[2 * a + side]

    def unknown_mask(self):
        """Nodes on no Dirichlet face."""
        m = np.ones(self.node_shape, bool)
        for a in range(self.dim):
            for s in (0, 1):
                if self.face_bc(a, s) == DIRICHLET:
                    m &= ~self.on_face(a, s)
        return m

    def node_weight(self):
        """Trapezoid weight: product of 1/2 over the free faces a node is on."""
        w = np.ones(self.node_shape)
        for a in range(self.dim):
            for s in (0, 1):
                if self.face_bc(a, s) == FREE:
                    w = np.where(self.on_face(a, s), 0.5 * w, w)
        return w

    # ---- vectors of unknowns --------------------------------------------
    def dof_mask(self):
        return np.broadcast_to(self.unknown_mask(), self.field_shape)

    def gather(self, full):
        """Full node field (dim, *node_shape) -> vector of unknown dofs."""
        return np.asarray(full, dtype=np.float64)[self.dof_mask()].copy()

    def scatter(self, vec):
        """Vector of unknown dofs -> full node field with zero Dirichlet nodes."""
        out = np.zeros(self.field_shape)
        out[self.dof_mask()] = vec
        return out

    def mass_diag(self, rho):
        """Per-dof weights m = w_node * rho of the M inner product (Sec. 4.1:
        M = diag(Lambda rho J); the factor h^d is dropped, it cancels in
        every ratio the method forms)."""
        per_node = self.node_weight() * np.asarray(rho, dtype=np.float64)
        return self.gather(np.broadcast_to(per_node, self.field_shape))
