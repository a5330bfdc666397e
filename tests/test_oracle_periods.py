"""The K-period filter (eq. many_periods_filter) on the oracle: the trend of
Table 3 on a finite-difference analogue of its bar.

Table 3 uses DG on [0,8] x [0,1] with free top, bottom and right sides and a
shaken left side.  The analogue here: the same bar, lambda = 2, mu = 1,
rho = 1, omega = 5.123, 128 x 16 cells, free top and bottom, Dirichlet left
and right (the FD operator supports free faces on the marching axis only),
forced by a Gaussian near the left end; CG to 1e-10.  The paper's point is
the efficiency N_1 / (K N_K): more periods cut the iterations, sublinearly.
"""

import json
import os

import numpy as np

from oracle import krylov
from oracle.operator import Operator
from oracle.problem import Problem
from oracle.stepping import WaveHoltz
from paper_2205_12344_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table3_periods.json")


def bar_problem(n=(128, 16)):
    length = (8.0, 1.0)
    prob = Problem(2, n, length=length, bc=(0, 0, 1, 1))
    shape = prob.node_shape
    op = Operator(prob, np.ones(shape), 2.0 * np.ones(shape), np.ones(shape))
    f = inputs.gaussian_sources(2, n, length, [(1.0, 0.5)], [0.25], [(1.0, 0.0)])
    return prob, op, f


def test_k_period_efficiency_follows_table3():
    g = json.load(open(GOLDEN))
    prob, op, f = bar_problem()
    iters = []
    for K in g["periods"]:
        wh = WaveHoltz(op, 5.123, periods=K)
        r = krylov.cg(wh.apply_A, wh.rhs(prob.gather(f)), op.m, tol=1e-10, maxit=2000)
        iters.append(r.iters)
    eff = [iters[0] / (K * n) for K, n in zip(g["periods"], iters)]
    # more periods, fewer iterations, but sublinearly: the efficiency falls
    assert all(a > b for a, b in zip(iters, iters[1:]))
    assert all(a >= b - 0.02 for a, b in zip(eff, eff[1:]))
    assert eff[-1] < 0.6
    # and it falls as in Table 3 (case 1) within 0.12 at every K
    for e, ref in zip(eff, g["case1_efficiency"]):
        assert abs(e - ref) <= 0.12, (eff, g["case1_efficiency"])
