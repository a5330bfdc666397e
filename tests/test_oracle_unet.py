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


def _ref_conv(X, W, b, act):
    """A 3x3 zero-padded convolution layer written independently of the
    oracle's im2col: per (input, output) channel pair a 2-D correlation
    (scipy.signal.correlate2d, mode 'same') with the kernel
    K[ky, kx] = W[(ky * 3 + kx) * cin + ci, co]."""
    from scipy.signal import correlate2d
    B, H, Wd, C = X.shape
    co_n = W.shape[1]
    out = np.zeros((B, H, Wd, co_n))
    K = W.reshape(3, 3, C, co_n)
    for bi in range(B):
        for co in range(co_n):
            acc = np.full((H, Wd), b[co])
            for ci in range(C):
                acc += correlate2d(X[bi, :, :, ci], K[:, :, ci, co], mode="same", boundary="fill")
            out[bi, :, :, co] = acc
    return out * (1.0 / (1.0 + np.exp(-out))) if act else out


def _ref_forward(theta, x):
    """The network's definition restated with the reference convolution,
    block means for pooling and Kronecker products for upsampling."""
    P = unet.unpack(theta)
    B = x.shape[0]

    def pool(h):
        b_, H, W, C = h.shape
        return h.reshape(b_, H // 2, 2, W // 2, 2, C).mean(axis=(2, 4))

    def up(h):
        return np.kron(h, np.ones((1, 2, 2, 1)))

    h, skips = x, []
    for lev in range(5):
        for l in (2 * lev, 2 * lev + 1):
            h = _ref_conv(h, *P[l], unet.LAYERS[l][2])
        skips.append(h)
        if lev < 4:
            h = pool(h)
    for lev in (3, 2, 1, 0):
        la = 10 + 2 * (3 - lev)
        h = np.concatenate([up(h), skips[lev]], axis=3)
        for l in (la, la + 1):
            h = _ref_conv(h, *P[l], unet.LAYERS[l][2])
    assert h.shape[0] == B
    return _ref_conv(h, *P[18], unet.LAYERS[18][2])


def test_conv_layer_matches_direct_correlation():
    rng = np.random.default_rng(4)
    X = rng.standard_normal((2, 8, 6, 5))
    W = rng.standard_normal((9 * 5, 3))
    b = rng.standard_normal(3)
    for act in (0, 1):
        _, got = unet._conv(X, W, b, act)
        np.testing.assert_allclose(got, _ref_conv(X, W, b, act), rtol=1e-12, atol=1e-12)


def test_forward_matches_independent_restatement():
    theta, x, _, _ = _setup(seed=3, B=1, H=16)
    got, _ = unet.forward(theta, x)
    np.testing.assert_allclose(got, _ref_forward(theta, x), rtol=1e-10, atol=1e-10)


def test_conv_pin_catches_a_flipped_kernel():
    """A convolution (flipped kernel) instead of a correlation fails the pin."""
    rng = np.random.default_rng(5)
    X = rng.standard_normal((1, 6, 6, 2))
    W = rng.standard_normal((18, 2))
    b = np.zeros(2)
    Wf = W.reshape(3, 3, 2, 2)[::-1, ::-1].reshape(18, 2)
    _, got = unet._conv(X, Wf, b, 0)
    assert np.abs(got - _ref_conv(X, W, b, 0)).max() > 1e-3
