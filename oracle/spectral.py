"""Filter transfer functions (oracle; test infrastructure only).

Sec. 3: for a mode cos(lambda t) the filter multiplies by
    beta(lambda) = (2/T) int_0^T (cos(omega t) - 1/4) cos(lambda t) dt;
App. B rescales r = lambda / omega,  beta_bar(r) = (1/pi) int_0^{2 pi}
(cos t - 1/4) cos(r t) dt, and defines the trapezoid analogue
    beta_bar_h(r) = (dt/pi) sum_n eta_n cos(r t_n) (cos t_n - 1/4),  t_n = 2 pi n / N.

For the corrected scheme a mode of M^-1(-L_h) with eigenvalue lambda_j^2
evolves as cos(n theta_j) with sin(theta_j / 2) = sin(omega dt / 2) lambda_j / omega
(the Taylor start makes u^{-1} = u^1), so the discrete S_h has eigenvalues
beta_h(theta_j) = sum_n w_n cos(n theta_j) and A_h has 1 - beta_h(theta_j).
"""

import math

import numpy as np


def beta_bar(r):
    """Closed form of the continuous rescaled transfer function:
    beta_bar(r) = (sin(2 pi r) / pi) (-r / (1 - r^2) - 1 / (4 r)), with the
    removable singularities at r = 0 (-1/2) and r = 1 (1)."""
    r = np.asarray(r, np.float64)
    out = np.empty_like(r)
    for i, x in np.ndenumerate(r):
        if abs(x) < 1e-12:
            out[i] = -0.5
        elif abs(x - 1.0) < 1e-12:
            out[i] = 1.0
        else:
            out[i] = math.sin(2 * math.pi * x) / math.pi * (-x / (1 - x * x) - 0.25 / x)
    return out


def beta_bar_h(r, nsteps):
    """Trapezoid transfer function of App. B with nsteps steps per period."""
    t = 2 * math.pi * np.arange(nsteps + 1) / nsteps
    eta = np.ones(nsteps + 1)
    eta[0] = eta[-1] = 0.5
    dt = 2 * math.pi / nsteps
    r = np.atleast_1d(np.asarray(r, np.float64))
    return (dt / math.pi) * (eta * (np.cos(t) - 0.25) * np.cos(np.outer(r, t))).sum(axis=1)


def beta_h(theta, weights):
    """sum_n w_n cos(n theta) for a weight table w_n."""
    n = np.arange(len(weights))
    theta = np.atleast_1d(np.asarray(theta, np.float64))
    return (np.asarray(weights) * np.cos(np.outer(theta, n))).sum(axis=1)


def mode_angle(lam_j, omega, dt):
    """theta_j = 2 arcsin(sin(omega dt / 2) lambda_j / omega) (corrected scheme)."""
    s = math.sin(0.5 * omega * dt) * np.asarray(lam_j, np.float64) / omega
    return 2.0 * np.arcsin(s)


def resonance_gap(nsteps, tol=1e-14):
    """Leftmost r* < 1 with beta_bar_h(r*) = 1 (bisection between the last
    point where beta_bar_h < 1 on a fine scan and 1), as in App. B."""
    rs = np.linspace(0.5, 1.0, 20001)
    vals = beta_bar_h(rs, nsteps)
    above = np.nonzero(vals >= 1.0)[0]
    j = above[0]
    if j == 0:
        raise ValueError("scan starts above 1")
    lo, hi = rs[j - 1], rs[j]
    while hi - lo > tol:
        mid = 0.5 * (lo + hi)
        if beta_bar_h([mid], nsteps)[0] >= 1.0:
            hi = mid
        else:
            lo = mid
    return hi
