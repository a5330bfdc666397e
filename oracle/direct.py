"""Direct solves of the discrete elastic Helmholtz system (oracle; test
infrastructure only).

Sec. 4.3: discretising the time-harmonic equation (eq. (elastic-frequency),
omega^2 rho v + div T(v) = f) directly in space gives
      (omega^2 M + L_h) v = W f,
and with the corrected time stepper the WaveHoltz fixed point equals this
solution exactly (Sec. 1.1; Sec. 5.2 "near machine precision").  With the
standard stepper the fixed point solves the same system with omega replaced
by wt = 2 sin(omega dt / 2) / dt (Sec. 4.3).  These are plain definitions;
the solves below are library sparse LU / dense LU of that matrix.
"""

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spl

from .operator import Operator


def helmholtz_matrix(op: Operator, omega):
    return (sp.diags(omega ** 2 * op.m) + op.Lh).tocsc()


def solve(op: Operator, omega, f):
    """v with (omega^2 M + L_h) v = W f, by sparse LU with pivoting."""
    return spl.splu(helmholtz_matrix(op, omega)).solve(op.w * np.asarray(f, np.float64))


def solve_dense(op: Operator, omega, f):
    return np.linalg.solve(helmholtz_matrix(op, omega).toarray(), op.w * np.asarray(f, np.float64))


def dense_operator(apply, n):
    """Brute force: the matrix of a linear map, column by column from unit vectors."""
    cols = []
    e = np.zeros(n)
    for j in range(n):
        e[j] = 1.0
        cols.append(apply(e))
        e[j] = 0.0
    return np.array(cols).T


def manufactured_forcing(op: Operator, omega, v):
    """f = omega^2 rho v + Ltilde v: the forcing whose discrete Helmholtz
    solution is exactly v."""
    v = np.asarray(v, np.float64)
    return omega ** 2 * op.rho_dof * v + op.apply_Ltilde(v)
