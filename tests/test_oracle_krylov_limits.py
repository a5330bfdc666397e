"""Two properties of the warm-start workload (its problems coarsened
to 64^2 cells so the CPU oracle runs in seconds) that bound what any solver
option can gain there.

* The CG iteration count to 1e-8 hardly depends on how close the start is:
  from the exact solution plus white noise of 1 % relative size (M norm) CG
  needs about as many iterations as from zero.  The count is set by the
  cluster of small eigenvalues of A_h (modes close to omega), which CG has
  to resolve whatever the start; this caps the gain of any initial guess,
  learned or not.
* Near resonance A_h can be slightly indefinite (Sec. 4.4, remark on the
  trapezoid rule): CG meets (p, A_h p)_M <= 0, while the conjugate residual
  method, the MINRES-type remedy the remark recommends, converges.
"""

import numpy as np
import pytest

from oracle import direct, krylov
from oracle.operator import Operator
from oracle.problem import Problem
from oracle.stepping import WaveHoltz
from paper_2205_12344_amd import inputs


def _setup(seed):
    c = inputs.warmstart_problem(seed, n=64)
    prob = Problem(2, c.n, bc=c.bc)
    op = Operator(prob, c.rho, c.lam, c.mu)
    wh = WaveHoltz(op, c.omega)
    fv = prob.gather(c.f)
    return c, op, wh, wh.rhs(fv), direct.solve(op, c.omega, fv)


@pytest.mark.parametrize("seed", [4099])
def test_close_start_barely_shortens_cg(seed):
    c, op, wh, b, xs = _setup(seed)
    zero = krylov.cg(wh.apply_A, b, op.m, tol=1e-8, maxit=3000)
    rng = np.random.default_rng(0)
    e = rng.standard_normal(b.size)
    e *= 0.01 * np.sqrt(np.dot(op.m * xs, xs) / np.dot(op.m * e, e))
    near = krylov.cg(wh.apply_A, b, op.m, x0=xs + e, tol=1e-8, maxit=3000)
    assert zero.iters > 100
    # a start 100x closer than zero saves under 5 % of the iterations
    assert near.iters >= 0.95 * zero.iters


def test_indefinite_case_cg_breaks_down_cr_converges():
    c, op, wh, b, xs = _setup(4115)
    with pytest.raises(ArithmeticError, match="breakdown"):
        krylov.cg(wh.apply_A, b, op.m, tol=1e-8, maxit=3000)
    r = krylov.cr(wh.apply_A, b, op.m, tol=1e-8, maxit=3000)
    assert np.linalg.norm(r.x - xs) / np.linalg.norm(xs) <= 1e-6
