"""The boundary-condition experiment of Sec. 5.6 on the GPU at sizes the
oracle solves in seconds: the unit cube, all faces Dirichlet or traction-free
z faces, h omega = 0.4, the standard explicit scheme, conjugate residual to
1e-9 from zero.  The GPU's iteration counts equal the oracle's (+-1) and its
FP64 true residual meets the tolerance; the oracle's counts grow like
omega^3 over these sizes, as the section states (slope pinned on the CPU)."""

import sys

import numpy as np
import pytest

from oracle import krylov
from oracle import stepping as S
from oracle.operator import Operator
from oracle.problem import Problem
from paper_2205_12344_amd import inputs


def _say(*a):
    print("[gpu-cube-bc]", *a, file=sys.stderr, flush=True)


def _oracle_cr(c, tol=1e-9):
    prob = Problem(3, c.n, bc=c.bc)
    op = Operator(prob, c.rho, c.lam, c.mu)
    wh = S.WaveHoltz(op, c.omega, scheme=S.STANDARD)
    r = krylov.cr(wh.apply_A, wh.rhs(prob.gather(c.f)), op.m, tol=tol, maxit=5000)
    return r.iters, wh.nt


def test_oracle_counts_grow_like_omega_cubed():
    """CPU: the oracle's CR counts over omega = 8, 10, 12 (20^3 .. 30^3 cells)
    have a log-log slope within [2.5, 3.5] for both boundary sets, and free z
    faces need more iterations than Dirichlet ones (the softer cavity)."""
    for free in (False, True):
        ws = (8.0, 10.0, 12.0)
        its = [_oracle_cr(inputs.cube_bc_case(w, free_z=free))[0] for w in ws]
        slope = np.polyfit(np.log(ws), np.log(its), 1)[0]
        _say("oracle", "free" if free else "dirichlet", its, "slope", slope)
        assert 2.5 <= slope <= 3.5
    assert _oracle_cr(inputs.cube_bc_case(8.0, True))[0] > _oracle_cr(inputs.cube_bc_case(8.0, False))[0]


@pytest.fixture(scope="module")
def E():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_12344_amd import elwh
    return elwh


@pytest.mark.gpu
@pytest.mark.parametrize("omega", [6.0, 10.0])
@pytest.mark.parametrize("free", [False, True])
def test_gpu_counts_equal_oracle(E, omega, free):
    c = inputs.cube_bc_case(omega, free_z=free)
    ref, nt = _oracle_cr(c)
    ctx = E.context_from_case(c, scheme=E.SCHEME_STANDARD, krylov=E.KRYLOV_CR)
    assert ctx.info()["nt"] == nt
    _, info = ctx.solve(c.f, tol=1e-9, maxit=5000)
    _say("omega", omega, "free" if free else "dirichlet", "cells", c.n[0], "gpu", info["iters"], "oracle", ref,
         "relres", info["relres_fp64"])
    assert info["status"] == "OK" and info["relres_fp64"] <= 1e-9
    assert abs(info["iters"] - ref) <= 1
