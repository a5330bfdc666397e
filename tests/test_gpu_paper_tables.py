"""The paper's printed numbers reproduced through the GPU path (C ABI), not
only through the oracle: Table 1 (Sec. 5.1), the accuracy of the FD
El-WaveHoltz solution under refinement."""

import json
import math
import os
import sys

import numpy as np
import pytest

from oracle.problem import Problem

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-tables]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def E():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_12344_amd import elwh
    return elwh


def _quartic(n, om=1.0, lam=1.0, mu=1.0):
    """u = v = 16^2 x^2 (x - 1)^2 y^2 (y - 1)^2 and the forcing f with
    omega^2 u + div T(u) = f (the manufactured solution of Table 1)."""
    prob = Problem(2, (n, n))
    X, Y = prob.mesh()
    p = lambda s: s ** 2 * (s - 1) ** 2
    d1 = lambda s: 2 * s * (s - 1) ** 2 + 2 * s ** 2 * (s - 1)
    d2 = lambda s: 2 * (s - 1) ** 2 + 8 * s * (s - 1) + 2 * s ** 2
    U = 256 * p(X) * p(Y)
    uxx, uyy, uxy = 256 * d2(X) * p(Y), 256 * p(X) * d2(Y), 256 * d1(X) * d1(Y)
    A = lam + 2 * mu
    f = np.array([om ** 2 * U + A * uxx + mu * uyy + (lam + mu) * uxy,
                  om ** 2 * U + mu * uxx + A * uyy + (lam + mu) * uxy])
    return prob, np.array([U, U]), f


def test_table1_fd_accuracy(E, golden_dir):
    """Table 1: the standard leapfrog with k = 0.4 h / sqrt(3 mu + lambda),
    omega = 1, lambda = mu = rho = 1 on the Dirichlet unit square, solved by
    CG on the GPU to a residual of 1e-12 (the paper: 1e-15); the mean
    absolute nodal error over the unknowns matches the printed errors within
    2.5 percent and the printed rates to +-0.011, as the oracle does."""
    g = json.load(open(os.path.join(golden_dir, "table1_fd_accuracy.json")))
    errs = []
    for n in g["n"]:
        prob, U, f = _quartic(n)
        one = np.ones(prob.node_shape)
        k = 0.4 * prob.h[0] / math.sqrt(3.0 + 1.0)
        nt = int(math.ceil(2 * math.pi / k))
        ctx = E.Context(2, (n, n), one, one, one, 1.0, (0, 0, 0, 0), nt=nt, scheme=E.SCHEME_STANDARD)
        v, info = ctx.solve(f, tol=1e-12, maxit=500)
        assert info["status"] == "OK" and info["nt"] == nt
        errs.append(float(np.mean(np.abs(prob.gather(v.cpu().numpy()) - prob.gather(U)))))
        _say("n", n, "nt", nt, "iters", info["iters"], "error", errs[-1])
        ctx.close()
    for e, ep in zip(errs, g["error"]):
        assert e == pytest.approx(ep, rel=0.025)
    rates = [math.log2(errs[i - 1] / errs[i]) for i in range(1, len(errs))]
    _say("rates", rates, "printed", g["rate"][1:])
    for r, rp in zip(rates, g["rate"][1:]):
        assert abs(r - rp) <= 0.011
