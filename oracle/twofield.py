"""Two-field El-WaveHoltz for impedance (absorbing) faces (oracle; test
infrastructure only).

Passages followed:

* Sec. 3, the remark after eq. (many_periods_filter): with boundary
  conditions that are not energy conserving the initial velocity u_1 is no
  longer zero, and the filter acts on the pair of initial displacement and
  velocity,  Pi [u0; u1] = (2/T) int_0^T (cos(w t) - 1/4) [u; u_t] dt,  whose
  fixed point is sought simultaneously in both fields; the resulting system
  is positive definite but not symmetric and is solved with GMRES (Sec. 5,
  the remark on impedance / non-reflecting conditions before Table 3).
* Sec. 2.1: the energy identity dE/dt = boundary integral of u_t . T(u) n;
  an impedance face T(u) n = -Z u_t makes that integral -u_t . Z u_t <= 0.

The paper leaves the discretisation to future work.  Readings taken here:

* Impedance matrix (the classical Lysmer-Kuhlemeyer choice): Z = rho c_p on
  the normal component and rho c_s on the tangential ones, c_p =
  sqrt((lam + 2 mu) / rho), c_s = sqrt(mu / rho), at each face node.
* Space: an impedance face is a traction-type face of the discrete energy of
  Sec. 4.1 (same stiffness and trapezoid weights as a traction-free face),
  plus the boundary integral of u_t . Z u_t by the trapezoid rule along the
  face.  Divided by the node mass w rho (w = 1/2 across the face) this is
  the per-dof damping  B = 2 c / h_a  (c = c_p normal, c_s tangential,
  h_a the spacing normal to the face; contributions of two faces add), so
        rho u'' = Ltilde u - rho B u' - f cos(w t).
* Time: the corrected leapfrog of Sec. 4.3 with the damping term centred,
        u^{n+1} - 2u^n + u^{n-1} = c dt^2 [rho^-1 (Ltilde u^n - f cos(w t_n))
                                           - Bt (u^{n+1} - u^{n-1}) / (2 dt)],
  Bt = B (w dt) / sin(w dt) for the corrected scheme (Bt = B for the
  standard one).  Applied to e^{i w t} the centred difference gives
  i sin(w dt) / dt, so Bt sin(w dt) / dt = w B, and together with the
  correction factor c of the second difference a time-harmonic discrete
  solution solves the damped Helmholtz system below with no time error, the
  property Sec. 4.3 establishes for the undamped scheme.  Per dof, with
  g = c dt Bt / 2:  (1 + g) u^{n+1} = 2u^n - (1 - g) u^{n-1} + a (Ltilde u^n
  - f cos(w t_n)),  a = c dt^2 / rho.
* Velocity: the centred difference v^n = (u^{n+1} - u^{n-1}) / (2 dt) at
  every level n = 0..K N_T (one step beyond the filter window for the last
  level), and the second field is the velocity at t = 0 in the same sense,
  u_1 = (u^1 - u^{-1}) / (2 dt).  Eliminating u^{-1} from the scheme at n = 0:
        u^1 = u^0 + dt (1 - g) u_1 + (a / 2) (Ltilde u^0 - f).
* Filter: the trapezoid weights w_n of the one-field filter on both fields,
  Pi_h [u0; u1] = [sum w_n u^n; sum w_n v^n].
* Fixed point.  For u^n = a cos(w t_n) + b sin(w t_n) the filter returns a
  and (sin(w dt) / dt) b, and u_1 = (sin(w dt) / dt) b, so with the
  corrected scheme the fixed point is  u0 = Re v,  u1 = -(sin(w dt) / dt) Im v
  for v the solution of
        (w^2 M + L_h - i w D) v = W f,   D = diag(m B)  (m = w rho),
  the direct discretisation of w^2 rho v + div T(v) - i w rho B v = f.
* Krylov: GMRES on A_h = I - S_h of the stacked unknown [u0; u1 / w] in the
  M inner product of each half (the 1/w scaling gives both halves the units
  of a displacement), from the zero guess, with b = Pi_h [0; 0].

Parity: the fixed point is pinned to the complex direct solve (a plain
definition, sparse LU); the damped stepping by the discrete energy decay it
implies, and the whole operator by its reduction to the one-field operator
when no face is an impedance face.
"""

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spl

from . import krylov
from .operator import Operator
from .problem import FREE
from .stepping import CORRECTED, WaveHoltz


def damping(op: Operator, faces):
    """Per-dof damping B of the impedance faces (a list of (axis, side);
    each must be a traction-type face of op.prob)."""
    prob = op.prob
    d = prob.dim
    B = np.zeros(prob.field_shape)
    cp = np.sqrt((op.lam + 2.0 * op.mu) / op.rho)
    cs = np.sqrt(op.mu / op.rho)
    for a, side in faces:
        if prob.face_bc(a, side) != FREE:
            raise ValueError("an impedance face must be a traction-type face")
        on = prob.on_face(a, side)
        for comp in range(d):
            speed = cp if comp == a else cs
            B[comp] += np.where(on, 2.0 * speed / prob.h[a], 0.0)
    return prob.gather(B)


class TwoField:
    """Pi_h, S_h, A_h and b of the two-field operator on the CPU, in float64."""

    def __init__(self, op: Operator, omega, faces, cfl=0.8, nt=None, periods=1, scheme=CORRECTED):
        self.wh = WaveHoltz(op, omega, cfl=cfl, nt=nt, periods=periods, scheme=scheme)
        self.op = op
        self.omega = self.wh.omega
        self.dt = self.wh.dt
        self.nt = self.wh.nt
        self.periods = self.wh.periods
        self.B = damping(op, faces)
        wdt = self.omega * self.dt
        self.Bt = self.B * (wdt / math.sin(wdt) if scheme == CORRECTED else 1.0)
        self.g = 0.5 * self.wh.c * self.dt * self.Bt
        self.weights = self.wh.weights
        self.cosn = self.wh.cosn

    # ---- the damped time stepping ------------------------------------------
    def trajectory(self, u0, u1, f=None, nsteps=None):
        """Yield u^0, u^1, ..., u^{nsteps} (default K N_T + 1)."""
        L = self.op.apply_Ltilde
        a, g, dt = self.wh.a, self.g, self.dt
        total = self.periods * self.nt + 1 if nsteps is None else nsteps
        cosn = lambda n: math.cos(2.0 * math.pi * n / self.nt)
        u_prev = np.asarray(u0, np.float64).copy()
        r = L(u_prev)
        if f is not None:
            r = r - f * cosn(0)
        u_cur = u_prev + dt * (1.0 - g) * np.asarray(u1, np.float64) + 0.5 * a * r
        yield u_prev
        yield u_cur
        for n in range(1, total):
            r = L(u_cur)
            if f is not None:
                r = r - f * cosn(n)
            u_next = (2.0 * u_cur - (1.0 - g) * u_prev + a * r) / (1.0 + g)
            u_prev, u_cur = u_cur, u_next
            yield u_cur

    def apply_filter(self, u0, u1, f=None):
        """Pi_h [u0; u1] = [sum_n w_n u^n; sum_n w_n v^n], v^n the centred
        velocity (S_h when f is None)."""
        N = self.periods * self.nt
        traj = list(self.trajectory(u0, u1, f))          # u^0 .. u^{N+1}
        acc0 = np.zeros(self.op.ndof)
        acc1 = np.zeros(self.op.ndof)
        for n in range(N + 1):
            acc0 += self.weights[n] * traj[n]
            vel = np.asarray(u1, np.float64) if n == 0 else (traj[n + 1] - traj[n - 1]) / (2.0 * self.dt)
            acc1 += self.weights[n] * vel
        return acc0, acc1

    def energies(self, u0, u1, nsteps):
        """Discrete energies E^{n+1/2} = (u^{n+1} - u^n)^T M (u^{n+1} - u^n) / (c dt^2)
        - (u^{n+1})^T L_h u^n of the unforced damped scheme, n = 0..nsteps-1."""
        Lh, m = self.op.Lh, self.op.m
        cdt2 = self.wh.c * self.dt ** 2
        out, prev = [], None
        for u in self.trajectory(u0, u1, None, nsteps):
            if prev is not None:
                d = u - prev
                out.append(float(d @ (m * d)) / cdt2 - float(u @ (Lh @ prev)))
            prev = u
        return np.array(out)

    # ---- the stacked linear system ------------------------------------------
    def split(self, z):
        n = self.op.ndof
        return z[:n], self.omega * z[n:]

    def join(self, x0, x1):
        return np.concatenate([x0, np.asarray(x1) / self.omega])

    def apply_A(self, z):
        """A_h z = z - S_h z on the stacked unknown z = [u0; u1 / w]."""
        s0, s1 = self.apply_filter(*self.split(z))
        return z - self.join(s0, s1)

    def rhs(self, f):
        zero = np.zeros(self.op.ndof)
        return self.join(*self.apply_filter(zero, zero, f))

    def mass(self):
        return np.concatenate([self.op.m, self.op.m])

    def solve(self, f, tol=1e-10, maxit=2000, restart=30):
        """GMRES on the stacked system; returns (u0, u1, KrylovResult)."""
        res = krylov.gmres(self.apply_A, self.rhs(f), self.mass(), tol=tol, maxit=maxit, restart=restart)
        u0, u1 = self.split(res.x)
        return u0, u1, res

    # ---- the time-harmonic problem it solves ---------------------------------
    def helmholtz_direct(self, f):
        """v with (w^2 M + L_h - i w D) v = W f, D = diag(m B), by sparse LU
        (f real or complex)."""
        op, w = self.op, self.omega
        H = (sp.diags(w * w * op.m - 1j * w * op.m * self.B) + op.Lh).tocsc()
        return spl.splu(H).solve(op.w * np.asarray(f).astype(complex))

    def fixed_point_of(self, v):
        """[u0; u1] that the corrected scheme's fixed point takes for the
        complex amplitude v: (Re v, -(sin(w dt) / dt) Im v)."""
        return v.real.copy(), -(math.sin(self.omega * self.dt) / self.dt) * v.imag
