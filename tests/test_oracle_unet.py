"""Pins of the FP64 warm-start network oracle: its hand-written backward pass
against central finite differences (CPU)."""

import numpy as np
import pytest

from oracle import unet


def _setup(seed=0, B=2, H=16):
    rng = np.random.default_rng(seed)
    theta = np.zeros(unet.num_params())
    off = 0
    for ci, co, _ in unet.LAYERS:
        theta[off:off + 9 * ci * co] = rng.standard_normal(9 * ci * co) * np.sqrt(2.0 / (9 * ci))
        off += 9 * ci * co
        theta[off:off + co] = 0.1 * rng.standard_normal(co)
        off += co
    x = rng.standard_normal((B, H, H, 7))
    y = rng.standard_normal((B, H, H, 2))
    w = rng.uniform(0.5, 1.5, (B, H, H))
    return theta, x, y, w


def test_param_count():
    assert unet.num_params() == 1644578


def test_gradient_matches_finite_differences():
    theta, x, y, w = _setup()
    L, g, _ = unet.loss_and_grad(theta, x, y, w)
    rng = np.random.default_rng(1)
    # a few parameters in every layer, weights and biases
    idx = []
    off = 0
    for ci, co, _ in unet.LAYERS:
        idx += list(rng.integers(off, off + 9 * ci * co, 2))
        off += 9 * ci * co
        idx.append(off + int(rng.integers(0, co)))
        off += co
    eps = 1e-6
    for k in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[k] += eps
        tm[k] -= eps
        fd = (unet.loss_and_grad(tp, x, y, w)[0] - unet.loss_and_grad(tm, x, y, w)[0]) / (2 * eps)
        assert g[k] == pytest.approx(fd, rel=1e-5, abs=1e-9 * max(1.0, abs(L)))


def test_im2col_col2im_adjoint():
    """<im2col X, C> = <X, col2im C>: the two are transposes."""
    rng = np.random.default_rng(2)
    X = rng.standard_normal((2, 8, 6, 3))
    C = rng.standard_normal((2 * 8 * 6, 27))
    assert np.sum(unet.im2col(X) * C) == pytest.approx(np.sum(X * unet.col2im(C, X.shape)), rel=1e-12)
