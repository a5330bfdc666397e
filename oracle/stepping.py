"""Time stepping, the WaveHoltz filter and the affine split (oracle).

Test infrastructure only.  Passages followed:

* Filter (Sec. 3, eq. (el_WHI_OP)):  Pi u0 = (2/T) int_0^T (cos(w t) - 1/4) u dt,
  u the solution with u(0) = u0, u_t(0) = 0.  Over K periods (eq.
  (many_periods_filter)) the prefactor is 2/(K T) and the range [0, K T].
* Quadrature: the trapezoidal rule (Sec. 4; App. B writes it with weights
  eta_n = 1/2 at both ends, 1 inside).  With N_T steps per period and
  t_n = n T / N_T the weights are
      w_n = (2 / (K N_T)) eta_n (cos(2 pi n / N_T) - 1/4),  n = 0..K N_T.
* Corrected explicit scheme (Sec. 4.3, eq. (elastic-time-explicit-corrected)):
      u^{n+1} - 2u^n + u^{n-1} = (wt^2 / w^2) dt^2 [Ltilde u^n - f cos(w t_n)] / rho,
  wt = 2 sin(w dt / 2) / dt;  the standard scheme (eq. (elastic-time-explicit))
  is the same with the factor 1.
* Initial data.  The printed u^{-1} (Sec. 4.3) is garbled (sign on L_h, and
  "L_h(u0 + f)").  Reading: the even-in-time Taylor start that encodes
  u_t(0) = 0,  u^{-1} = u^0 + (c dt^2 / 2) rho^-1 (Ltilde u^0 - f),  so that
  the first step gives u^1 = u^{-1}.  Pinned by the fixed-point identity
  Pi_h v* = v* (exact for this reading, O(1) wrong for the literal one).
* Time step.  For explicit FD the paper fixes no rule beyond a CFL number
  (Sec. 5.1); the implicit scheme uses dt = T/k for an integer k (Sec. 4.4).
  Reading: dt* = cfl * 2 / sqrt(G), G the Gershgorin bound of the spectrum of
  rho^-1 Ltilde;  N_T = max(3, ceil(T / dt*)),  dt = T / N_T exactly (a whole
  number of steps per period is what makes the trapezoid rule reproduce the
  fixed point exactly; N_T >= 3 makes sum cos^2 = N_T / 2).
* Modified trapezoid weights (the remark closing Sec. 4.4, after Peng et al.):
  the standard scheme keeps its time error out of the fixed point when the
  weights are multiplied by cos(w t_n) / cos(wbar t_n).  The printed formula
  names the ratio but not the frequency the discrete solution oscillates at.
  Reading: the standard leapfrog is forced at wbar = (2 / dt) asin(w dt / 2),
  the frequency whose discrete dispersion relation gives w, so its
  time-harmonic solution is v cos(wbar t_n) with (w^2 M + L_h) v = W f exactly
  (2 sin(wbar dt / 2) / dt = w), and the weights
      w_n = (2 / (K N_T)) eta_n (cos(w t_n) - 1/4) cos(w t_n) / cos(wbar t_n)
  give sum_n w_n cos(wbar t_n) = sum_n (2/(K N_T)) eta_n (cos - 1/4) cos = 1,
  so Pi_h v = v.  Needs w dt / 2 < 1, i.e. N_T >= 4; the denominator can come
  close to zero, the risk the remark names.
* Affine split (Sec. 4.5, eq. (amat_non_sym)):  A_h = I - S_h with S_h = Pi_h
  at f = 0, and b = Pi_h 0.
* Discrete energy (Sec. 4.1, eq. (8), in the corrected form):
      E^{n+1/2} = (u^{n+1} - u^n)^T M (u^{n+1} - u^n) / (c dt^2) - (u^{n+1})^T L_h u^n
  is constant when f = 0.
"""

import math

import numpy as np

from .operator import Operator

CORRECTED = "corrected"
STANDARD = "standard"
MODIFIED = "modified"          # standard stepping, modified trapezoid weights


def steps_per_period(gershgorin_bound, omega, cfl=0.8):
    """N_T = max(3, ceil(T / dt*)), dt* = cfl * 2 / sqrt(G)."""
    T = 2.0 * math.pi / omega
    dt_star = cfl * 2.0 / math.sqrt(gershgorin_bound)
    return max(3, int(math.ceil(T / dt_star)))


def correction_factor(omega, dt):
    """c = (wt / w)^2 = (sin(w dt / 2) / (w dt / 2))^2  (Sec. 4.3)."""
    x = 0.5 * omega * dt
    return (math.sin(x) / x) ** 2


def modified_forcing_frequency(omega, dt):
    """wbar = (2 / dt) asin(w dt / 2): the standard leapfrog forced at wbar has
    the time-harmonic solution of the Helmholtz problem at w."""
    x = 0.5 * omega * dt
    if not x < 1.0:
        raise ValueError("modified weights need omega dt / 2 < 1 (N_T >= 4)")
    return 2.0 * math.asin(x) / dt


def modified_filter_weights(nt, omega, periods=1):
    """Weights and forcing factors of the modified trapezoid rule (reading in
    the module docstring): w_n cos(w t_n) / cos(wbar t_n) and cos(wbar t_n)."""
    w, cosn = filter_weights(nt, periods)
    dt = 2.0 * math.pi / (omega * nt)
    wbar = modified_forcing_frequency(omega, dt)
    t = dt * np.arange(periods * nt + 1)
    cbar = np.cos(wbar * t)
    return w * cosn / cbar, cbar


def filter_weights(nt, periods=1):
    """Trapezoid weights w_n, n = 0..periods*nt, of the (K-period) filter."""
    ntot = periods * nt
    n = np.arange(ntot + 1)
    eta = np.ones(ntot + 1)
    eta[0] = eta[-1] = 0.5
    cosn = np.array([math.cos(2.0 * math.pi * k / nt) for k in range(ntot + 1)])
    return (2.0 / ntot) * eta * (cosn - 0.25), cosn


class WaveHoltz:
    """Pi_h, S_h, A_h and b for one problem on the CPU, in float64."""

    def __init__(self, op: Operator, omega, cfl=0.8, nt=None, periods=1, scheme=CORRECTED):
        if omega <= 0:
            raise ValueError("omega must be positive")
        self.op = op
        self.omega = float(omega)
        self.periods = int(periods)
        self.nt = int(nt) if nt is not None else steps_per_period(op.gershgorin(), omega, cfl)
        if self.nt < 3:
            raise ValueError("need at least 3 steps per period")
        self.T = 2.0 * math.pi / self.omega
        self.dt = self.T / self.nt
        self.scheme = scheme
        self.c = correction_factor(self.omega, self.dt) if scheme == CORRECTED else 1.0
        if scheme == MODIFIED:
            self.weights, self.cosn = modified_filter_weights(self.nt, self.omega, self.periods)
        else:
            self.weights, self.cosn = filter_weights(self.nt, self.periods)
        self.a = self.c * self.dt ** 2 / op.rho_dof          # per dof

    # ---- the time-stepping filter -----------------------------------------
    def trajectory(self, u0, f=None):
        """Yield u^0, u^1, ..., u^{K N_T} of the corrected scheme."""
        L = self.op.apply_Ltilde
        u_prev = np.asarray(u0, np.float64).copy()
        g = L(u_prev)
        if f is not None:
            g = g - f * self.cosn[0]
        u_cur = u_prev + 0.5 * self.a * g          # u^1 = u^{-1}
        yield u_prev
        yield u_cur
        for n in range(1, self.periods * self.nt):
            g = L(u_cur)
            if f is not None:
                g = g - f * self.cosn[n]
            u_next = 2.0 * u_cur - u_prev + self.a * g
            u_prev, u_cur = u_cur, u_next
            yield u_cur

    def apply_filter(self, u0, f=None):
        """Pi_h u0 = sum_n w_n u^n  (S_h u0 when f is None)."""
        acc = np.zeros(self.op.ndof)
        for n, u in enumerate(self.trajectory(u0, f)):
            acc += self.weights[n] * u
        return acc

    def apply_A(self, x):
        """A_h x = x - S_h x."""
        return np.asarray(x, np.float64) - self.apply_filter(x, None)

    def rhs(self, f):
        """b = Pi_h 0 with forcing f."""
        return self.apply_filter(np.zeros(self.op.ndof), f)

    # ---- diagnostics --------------------------------------------------------
    def energies(self, u0, f=None, nsteps=None):
        """Discrete energies E^{n+1/2}, n = 0..nsteps-1 (defaults to K N_T)."""
        Lh, m = self.op.Lh, self.op.m
        out = []
        prev = None
        cdt2 = self.c * self.dt ** 2
        for n, u in enumerate(self.trajectory(u0, f)):
            if prev is not None:
                d = u - prev
                out.append(float(d @ (m * d)) / cdt2 - float(u @ (Lh @ prev)))
            prev = u
            if nsteps is not None and len(out) >= nsteps:
                break
        return np.array(out)

    def m_dot(self, x, y):
        return float(np.dot(self.op.m * x, y))
