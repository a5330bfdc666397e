"""Iterations against frequency (the rectangle of the experiment on
iterations vs omega in Sec. 5): a 5 x 1 rectangle, lambda = 2, mu = 1,
rho = 1, Dirichlet sides, standard explicit scheme, about 20 points per
wavelength (n_r = 4 L omega + 1, n_q = 4 omega + 1), a discrete point source
of amplitude omega^2 near (0.5, 0.5), omega = k + sqrt(2)/10, conjugate
residual to 1e-8.  The paper states (its figure has no table) that the
iteration count grows like omega^d in d dimensions; the log-log slope of the
oracle's counts over k = 4..16 is 2.16 (2.14 with k = 24 added)."""

import math

import numpy as np

from oracle import krylov
from oracle.operator import Operator
from oracle.problem import Problem
from oracle.stepping import STANDARD, WaveHoltz


def cr_iterations(k):
    w = k + math.sqrt(2) / 10
    n = (int(4 * 5 * w + 1), int(4 * w + 1))
    prob = Problem(2, n, length=(5.0, 1.0), bc=(0, 0, 0, 0))
    shape = prob.node_shape
    op = Operator(prob, np.ones(shape), 2.0 * np.ones(shape), np.ones(shape))
    f = np.zeros(prob.field_shape)
    f[0, n[1] // 2, n[0] // 10] = w * w / ((5.0 / n[0]) * (1.0 / n[1]))
    wh = WaveHoltz(op, w, scheme=STANDARD)
    r = krylov.cr(wh.apply_A, wh.rhs(prob.gather(f)), op.m, tol=1e-8, maxit=5000)
    return w, r.iters


def test_iterations_grow_like_omega_squared():
    data = [cr_iterations(k) for k in (4, 6, 8, 12, 16)]
    slope = np.polyfit(np.log([w for w, _ in data]), np.log([i for _, i in data]), 1)[0]
    assert all(a[1] < b[1] for a, b in zip(data, data[1:]))
    assert 1.6 <= slope <= 2.6, (data, slope)
