"""The entry point that allocates nothing (elwh_dot_M_noalloc), through the C
ABI, against the context-based elwh_dot_M it varies (FP64: rel <= 1e-13,
two deterministic reduction orders) and against the oracle's M weights, on
two calls in a row, the second with a smaller grid; plus its argument
checks.  The two calls share the library's scratch array: the second must
not see anything of the first."""

import sys

import numpy as np
import pytest

from oracle.problem import Problem

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-noalloc]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def E():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_12344_amd import elwh
    return elwh


def _media(shape, seed):
    rng = np.random.default_rng(seed)
    rho = np.exp(0.25 * rng.standard_normal(shape))
    mu = np.exp(0.25 * rng.standard_normal(shape))
    return rho, 2.0 * mu, mu


CASES = [
    # (dim, n, bc): a larger grid first, then a smaller one on the same GPU
    (2, (301, 170), (0, 0, 1, 2)),
    (2, (40, 23), (0, 0, 0, 1)),
    (3, (37, 30, 25), (0, 0, 0, 0, 1, 1)),
    (3, (9, 8, 7), (0, 0, 0, 0, 0, 1)),
]


def test_noalloc_dot_matches_context_dot(E):
    import torch
    for k, (dim, n, bc) in enumerate(CASES):
        prob = Problem(dim, n, bc=tuple(min(b, 1) for b in bc))
        rho, lam, mu = _media(prob.node_shape, 10 + k)
        rng = np.random.default_rng(20 + k)
        x = rng.standard_normal(prob.field_shape)
        y = rng.standard_normal(prob.field_shape)
        ref = float(np.dot(prob.mass_diag(rho) * prob.gather(x), prob.gather(y)))
        ctx = E.Context(dim, n, rho, lam, mu, 3.0, bc)
        want = ctx.dot_M(x, y)
        td = [torch.from_numpy(a).cuda() for a in (rho, x, y)]
        got = E.dot_M_noalloc(dim, n, td[0], bc, td[1], td[2])
        again = E.dot_M_noalloc(dim, n, td[0], bc, td[1], td[2])
        _say(dim, n, bc, got, want, ref)
        assert got == again                                   # deterministic
        assert got == pytest.approx(want, rel=1e-13)
        assert got == pytest.approx(ref, rel=1e-13)
        # (x, x)_M > 0 and the M weights vanish on Dirichlet faces
        xx = E.dot_M_noalloc(dim, n, td[0], bc, td[1], td[1])
        assert xx == pytest.approx(float(np.dot(prob.mass_diag(rho) * prob.gather(x), prob.gather(x))),
                                   rel=1e-13)
        del ctx


def test_noalloc_dot_rejects_bad_arguments(E):
    import torch
    rho = torch.ones((9, 9), dtype=torch.float64, device="cuda")
    x = torch.ones((2, 9, 9), dtype=torch.float64, device="cuda")
    with pytest.raises(E.ElwhError, match="ERR_ARG"):
        E.dot_M_noalloc(2, (1, 8), rho, (0, 0, 0, 0), x, x)
    with pytest.raises(E.ElwhError, match="ERR_ARG"):
        E.dot_M_noalloc(2, (8, 8), rho, (0, 0, 7, 0), x, x)
    with pytest.raises(E.ElwhError, match="2\\^31"):
        big = (2000, 2000, 1000)          # 4e9 nodes: rejected before any device access
        E.dot_M_noalloc(3, big, rho, (0,) * 6, x, x)
