"""FP64 NumPy forward and backward of the warm-start network (oracle; test
infrastructure only).

The network is not part of the paper: it produces an initial guess for the
Krylov solve of Sec. 4.5.  Definition (the same network the library trains):
five resolution levels; each level two 3x3 convolutions (zero padding,
bias, SiLU x * sigmoid(x)) of widths 32, 64, 96, 128, 128; 2x2 average
pooling between encoder levels; the decoder upsamples by nearest
neighbour, concatenates [upsampled, encoder skip] along channels and applies
two convolutions; a final 3x3 convolution to 2 channels without activation.
Tensors are NHWC.  Parameters are one flat vector: per layer W[9 cin][cout]
(row (ky*3+kx)*cin + ci) then bias[cout].

Loss: L = (1/B) sum_b sum w (yh - y)^2 / sum w y^2 (w per pixel).

The backward pass is written by hand and pinned by central finite
differences in the tests.
"""

import numpy as np

LAYERS = [
    (7, 32, 1), (32, 32, 1),
    (32, 64, 1), (64, 64, 1),
    (64, 96, 1), (96, 96, 1),
    (96, 128, 1), (128, 128, 1),
    (128, 128, 1), (128, 128, 1),
    (256, 128, 1), (128, 128, 1),
    (224, 96, 1), (96, 96, 1),
    (160, 64, 1), (64, 64, 1),
    (96, 32, 1), (32, 32, 1),
    (32, 2, 0),
]
WIDTH = [32, 64, 96, 128, 128]


def num_params():
    return sum(9 * ci * co + co for ci, co, _ in LAYERS)


def unpack(theta):
    out, off = [], 0
    for ci, co, _ in LAYERS:
        W = theta[off:off + 9 * ci * co].reshape(9 * ci, co)
        off += 9 * ci * co
        b = theta[off:off + co]
        off += co
        out.append((W, b))
    return out


def im2col(X):
    B, H, W, C = X.shape
    P = np.zeros((B, H + 2, W + 2, C))
    P[:, 1:-1, 1:-1, :] = X
    cols = [P[:, ky:ky + H, kx:kx + W, :] for ky in range(3) for kx in range(3)]
    return np.concatenate(cols, axis=3).reshape(B * H * W, 9 * C)


def col2im(dcol, shape):
    B, H, W, C = shape
    d = dcol.reshape(B, H, W, 9, C)
    P = np.zeros((B, H + 2, W + 2, C))
    for ky in range(3):
        for kx in range(3):
            P[:, ky:ky + H, kx:kx + W, :] += d[:, :, :, ky * 3 + kx, :]
    return P[:, 1:-1, 1:-1, :]


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def pool(X):
    return 0.25 * (X[:, 0::2, 0::2] + X[:, 1::2, 0::2] + X[:, 0::2, 1::2] + X[:, 1::2, 1::2])


def pool_back(dY):
    return 0.25 * np.repeat(np.repeat(dY, 2, axis=1), 2, axis=2)


def up(X):
    return np.repeat(np.repeat(X, 2, axis=1), 2, axis=2)


def up_back(dY):
    return dY[:, 0::2, 0::2] + dY[:, 1::2, 0::2] + dY[:, 0::2, 1::2] + dY[:, 1::2, 1::2]


def _conv(X, W, b, act):
    B, H, Wd, C = X.shape
    Z = (im2col(X) @ W + b).reshape(B, H, Wd, -1)
    return Z, (silu(Z) if act else Z)


def forward(theta, x):
    """Returns the output and a cache for backward."""
    P = unpack(theta)
    cache = {"in": {}, "Z": {}, "A": {}}

    def run(l, X):
        W, b = P[l]
        Z, A = _conv(X, W, b, LAYERS[l][2])
        cache["in"][l], cache["Z"][l], cache["A"][l] = X, Z, A
        return A

    h = x
    skips = []
    for lev in range(5):
        h = run(2 * lev, h)
        h = run(2 * lev + 1, h)
        skips.append(h)
        if lev < 4:
            h = pool(h)
    for lev in (3, 2, 1, 0):
        la = 10 + 2 * (3 - lev)
        h = np.concatenate([up(h), skips[lev]], axis=3)
        h = run(la, h)
        h = run(la + 1, h)
    y = run(18, h)
    return y, cache


def loss(yh, y, w):
    B = y.shape[0]
    num = (w[..., None] * (yh - y) ** 2).reshape(B, -1).sum(axis=1)
    den = (w[..., None] * y ** 2).reshape(B, -1).sum(axis=1)
    den = np.where(den > 0, den, 1.0)
    L = float((num / den).sum() / B)
    dyh = 2.0 / B * w[..., None] * (yh - y) / den[:, None, None, None]
    return L, dyh


def backward(theta, cache, dy):
    P = unpack(theta)
    grads = [None] * len(LAYERS)

    def back(l, dA):
        W, b = P[l]
        X, Z = cache["in"][l], cache["Z"][l]
        dZ = dA * silu_grad(Z) if LAYERS[l][2] else dA
        B, H, Wd, _ = X.shape
        dZf = dZ.reshape(B * H * Wd, -1)
        grads[l] = (im2col(X).T @ dZf, dZf.sum(axis=0))
        return col2im(dZf @ W.T, X.shape)

    d = back(18, dy)
    dskip = {}
    for lev in (0, 1, 2, 3):
        la = 10 + 2 * (3 - lev)
        d = back(la + 1, d)
        dcat = back(la, d)
        cup = dcat.shape[3] - WIDTH[lev]
        dskip[lev] = dcat[..., cup:]
        d = up_back(dcat[..., :cup])
    for lev in (4, 3, 2, 1, 0):
        if lev < 4:
            d = d + dskip[lev]
        d = back(2 * lev + 1, d)
        d = back(2 * lev, d)
        if lev > 0:
            d = pool_back(d)
    flat = []
    for gW, gb in grads:
        flat.append(gW.ravel())
        flat.append(gb)
    return np.concatenate(flat)


def loss_and_grad(theta, x, y, w):
    yh, cache = forward(theta, x)
    L, dyh = loss(yh, y, w)
    return L, backward(theta, cache, dyh), yh
