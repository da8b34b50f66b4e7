"""Pins of the FP64 reference of the warm-start surrogate (CPU only):
the convolution against brute-force loops, the adjoint identities of every
linear piece, and the whole network's gradient against central finite
differences."""
import itertools

import numpy as np
import pytest

from oracle import nn_ref as nn


def brute_conv(x, w, b):
    B, D, H, W, ci = x.shape
    co = w.shape[1]
    y = np.zeros((B, D, H, W, co))
    for bb, z, yy, xx in itertools.product(range(B), range(D), range(H), range(W)):
        for t, (dz, dy, dx) in enumerate(nn.TAPS):
            src = x[bb, (z + dz) % D, (yy + dy) % H, (xx + dx) % W]
            y[bb, z, yy, xx] += w[t] @ src
        y[bb, z, yy, xx] += b
    return y


def test_conv_matches_brute_force_loops():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(2, 3, 4, 5, 2))
    w = rng.normal(size=(27, 3, 2))
    b = rng.normal(size=3)
    assert np.allclose(nn.conv3d(x, w, b), brute_conv(x, w, b), rtol=0, atol=1e-12)


def test_conv_tap_order_is_z_major():
    # a single non-zero weight at tap (dz, dy, dx) = (1, 0, -1) reads x[z + 1, y, x - 1]
    x = np.zeros((1, 4, 4, 4, 1))
    x[0, 2, 1, 0, 0] = 1.0
    w = np.zeros((27, 1, 1))
    w[9 * 2 + 3 * 1 + 0] = 1.0
    y = nn.conv3d(x, w, np.zeros(1))
    assert y[0, 1, 1, 1, 0] == 1.0 and y.sum() == 1.0


def test_adjoint_identities():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(2, 4, 6, 4, 3))
    w = rng.normal(size=(27, 5, 3))
    dy = rng.normal(size=(2, 4, 6, 4, 5))
    lin = nn.conv3d(x, w, np.zeros(5))
    # <A x, y> = <x, A^T y> for the input, and the same for the weights
    assert np.isclose((lin * dy).sum(), (x * nn.conv3d_bwd_data(dy, w)).sum(), rtol=1e-12)
    dw, db = nn.conv3d_bwd_weight(x, dy)
    assert np.isclose((lin * dy).sum(), (w * dw).sum(), rtol=1e-12)
    assert np.allclose(db, dy.sum(axis=(0, 1, 2, 3)))
    p = rng.normal(size=(2, 2, 3, 2, 3))
    assert np.isclose((nn.pool2(x) * p).sum(), (x * nn.pool2_bwd(p)).sum(), rtol=1e-12)
    q = rng.normal(size=(2, 8, 12, 8, 3))
    assert np.isclose((nn.up2(x) * q).sum(), (x * nn.up2_bwd(q)).sum(), rtol=1e-12)


def test_network_gradient_against_finite_differences():
    spec = nn.layers(2, 3, 4)
    params = nn.init_params(spec, 5)
    rng = np.random.default_rng(6)
    params = {k: (w, rng.normal(scale=0.1, size=b.shape)) for k, (w, b) in params.items()}
    x = rng.normal(size=(1, 8, 8, 8, 2))
    target = rng.normal(size=(1, 8, 8, 8, 3))
    cw = np.array([1.0, 0.5, 2.0])

    def loss(p):
        out, _ = nn.forward(p, x, spec)
        return nn.mse(out, target, cw)[0]

    out, cache = nn.forward(params, x, spec)
    _, dout = nn.mse(out, target, cw)
    grads, dx = nn.backward(params, cache, dout, spec)
    eps = 1e-6
    for name, (t, co, ci) in [("e1a", (13, 1, 0)), ("e3a", (5, 9, 6)), ("b1", (0, 5, 7)), ("d3", (2, 10, 20)),
                              ("d2", (26, 2, 11)), ("out", (4, 2, 3))]:
        w, b = params[name]
        wp, wm = w.copy(), w.copy()
        wp[t, co, ci] += eps
        wm[t, co, ci] -= eps
        fd = (loss({**params, name: (wp, b)}) - loss({**params, name: (wm, b)})) / (2 * eps)
        assert np.isclose(grads[name][0][t, co, ci], fd, rtol=1e-5, atol=1e-10), name
    for name in ("e2b", "e3b", "d1"):
        w, b = params[name]
        bp, bm = b.copy(), b.copy()
        bp[1] += eps
        bm[1] -= eps
        fd = (loss({**params, name: (w, bp)}) - loss({**params, name: (w, bm)})) / (2 * eps)
        assert np.isclose(grads[name][1][1], fd, rtol=1e-5, atol=1e-10), name
    # and the input gradient
    xp, xm = x.copy(), x.copy()
    xp[0, 3, 4, 5, 1] += eps
    xm[0, 3, 4, 5, 1] -= eps
    op, _ = nn.forward(params, xp, spec)
    om, _ = nn.forward(params, xm, spec)
    fd = (nn.mse(op, target, cw)[0] - nn.mse(om, target, cw)[0]) / (2 * eps)
    assert np.isclose(dx[0, 3, 4, 5, 1], fd, rtol=1e-5, atol=1e-10)
