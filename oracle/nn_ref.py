"""FP64 CPU reference of the warm-start surrogate network (test
infrastructure only: tests, the smoke check and the bench's CPU leg use it;
the product path never does).

The surrogate maps a solid mask and a component-fraction field to the
steady velocity and component densities that the lattice Boltzmann solver
reaches (the learned warm start; the solver always runs on from its output
and judges it).  Everything here is the plain definition written out in
float64 with NumPy, on channel-last arrays x[b, z, y, x, c]:

* conv3d: 3 x 3 x 3 convolution with periodic padding (the lattices are
  periodic), weights w[t, co, ci] with tap t = 9 (dz + 1) + 3 (dy + 1) +
  (dx + 1), bias b[co]:
  y[p, co] = b[co] + sum_t sum_ci w[t, co, ci] x[p + d_t, ci];
* its two adjoints (gradient with respect to the input and to the weights);
* ReLU, 2 x 2 x 2 average pooling, nearest 2x upsampling, channel concat;
* the weighted mean-square loss;
* the encoder-decoder built from them (UNet below) with its forward and
  backward passes.

Pinned by tests/test_nn_oracle.py: a brute-force loop convolution, the
adjoint identities <A x, y> = <x, A^T y>, and central finite differences of
the whole network's loss.
"""
from __future__ import annotations

import numpy as np

TAPS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def shift(x, d):
    """s[p] = x[p + d] with periodic wrap over the three spatial axes."""
    dz, dy, dx = d
    return np.roll(x, shift=(-dz, -dy, -dx), axis=(1, 2, 3))


def conv3d(x, w, b):
    y = np.zeros(x.shape[:4] + (w.shape[1],))
    for t, d in enumerate(TAPS):
        y += shift(x, d) @ w[t].T
    return y + b


def conv3d_bwd_data(dy, w):
    """dx[p, ci] = sum_t sum_co w[t, co, ci] dy[p - d_t, co]."""
    dx = np.zeros(dy.shape[:4] + (w.shape[2],))
    for t, d in enumerate(TAPS):
        dx += shift(dy @ w[t], tuple(-v for v in d))
    return dx


def conv3d_bwd_weight(x, dy):
    """dw[t, co, ci] = sum_p dy[p, co] x[p + d_t, ci]; db[co] = sum_p dy[p, co]."""
    co, ci = dy.shape[-1], x.shape[-1]
    dyf = dy.reshape(-1, co)
    dw = np.stack([dyf.T @ shift(x, d).reshape(-1, ci) for d in TAPS])
    return dw, dyf.sum(axis=0)


def relu(x):
    return np.maximum(x, 0.0)


def relu_bwd(dy, y):
    return dy * (y > 0)


def pool2(x):
    b, d, h, w, c = x.shape
    return x.reshape(b, d // 2, 2, h // 2, 2, w // 2, 2, c).mean(axis=(2, 4, 6))


def pool2_bwd(dy):
    return np.repeat(np.repeat(np.repeat(dy, 2, axis=1), 2, axis=2), 2, axis=3) / 8.0


def up2(x):
    return np.repeat(np.repeat(np.repeat(x, 2, axis=1), 2, axis=2), 2, axis=3)


def up2_bwd(dy):
    b, d, h, w, c = dy.shape
    return dy.reshape(b, d // 2, 2, h // 2, 2, w // 2, 2, c).sum(axis=(2, 4, 6))


def mse(pred, target, cw):
    """L = sum_c cw[c] mean_p (pred - target)^2 and dL/dpred."""
    n = pred.size // pred.shape[-1]
    r = pred - target
    return float((cw * (r * r)).sum() / n), 2.0 * cw * r / n


# ---------------------------------------------------------------------------
# The encoder-decoder.  Layer list: (name, ci, co, relu); the skip
# connections concatenate [upsampled, encoder] channels.
# ---------------------------------------------------------------------------
def layers(cin, cout, base):
    c1, c2 = base, 2 * base
    return [
        ("e1a", cin, c1, True), ("e1b", c1, c1, True),      # full resolution
        ("e2a", c1, c2, True), ("e2b", c2, c2, True),       # 1/2
        ("b1", c2, c2, True), ("b2", c2, c2, True),         # 1/4
        ("d2", 2 * c2, c2, True),                           # 1/2: [up(b2), e2b]
        ("d1", c2 + c1, c1, True),                          # full: [up(d2), e1b]
        ("out", c1, cout, False),
    ]


def _same(a):
    return a


def forward(params, x, spec, store=_same):
    """params: {name: (w, b)}; returns (output, cache of activations).
    store(a) is applied to every stored activation (identity by default; a
    caller that emulates reduced-precision storage passes its rounding).
    The output layer's result is not passed through store."""
    spec = {l[0]: l for l in spec}
    a = {}
    def conv(name, inp):
        w, b = params[name]
        y = conv3d(inp, w, b)
        y = relu(y) if spec[name][3] else y
        return y if name == "out" else store(y)
    a["x"] = x
    a["e1a"] = conv("e1a", x)
    a["e1b"] = conv("e1b", a["e1a"])
    a["p1"] = store(pool2(a["e1b"]))
    a["e2a"] = conv("e2a", a["p1"])
    a["e2b"] = conv("e2b", a["e2a"])
    a["p2"] = store(pool2(a["e2b"]))
    a["b1"] = conv("b1", a["p2"])
    a["b2"] = conv("b2", a["b1"])
    a["c2"] = np.concatenate([up2(a["b2"]), a["e2b"]], axis=-1)
    a["d2"] = conv("d2", a["c2"])
    a["c1"] = np.concatenate([up2(a["d2"]), a["e1b"]], axis=-1)
    a["d1"] = conv("d1", a["c1"])
    a["out"] = conv("out", a["d1"])
    return a["out"], a


def backward(params, a, dout, spec, store=_same):
    """Gradients {name: (dw, db)} of the loss whose gradient with respect to
    the output is dout, and the gradient with respect to the input.
    store(g) is applied to the gradient at each convolution's output (after
    the ReLU mask) before both of its uses."""
    spec = {l[0]: l for l in spec}
    g = {}
    def conv_back(name, inp, dy):
        w, _ = params[name]
        if spec[name][3]:
            dy = relu_bwd(dy, a[name])
        dy = store(dy)
        g[name] = conv3d_bwd_weight(inp, dy)
        return conv3d_bwd_data(dy, w)
    dd1 = conv_back("out", a["d1"], dout)
    dc1 = conv_back("d1", a["c1"], dd1)
    c_up = a["d2"].shape[-1]
    dd2 = up2_bwd(dc1[..., :c_up])
    de1b = dc1[..., c_up:].copy()
    dc2 = conv_back("d2", a["c2"], dd2)
    c_up2 = a["b2"].shape[-1]
    db2 = up2_bwd(dc2[..., :c_up2])
    de2b = dc2[..., c_up2:].copy()
    db1 = conv_back("b2", a["b1"], db2)
    dp2 = conv_back("b1", a["p2"], db1)
    de2b += pool2_bwd(dp2)
    de2a = conv_back("e2b", a["e2a"], de2b)
    dp1 = conv_back("e2a", a["p1"], de2a)
    de1b += pool2_bwd(dp1)
    de1a = conv_back("e1b", a["e1a"], de1b)
    dx = conv_back("e1a", a["x"], de1a)
    return g, dx


def init_params(spec, seed):
    """He-uniform weights from a seeded generator, zero biases."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, ci, co, _ in spec:
        lim = np.sqrt(6.0 / (27 * ci))
        p[name] = (rng.uniform(-lim, lim, size=(27, co, ci)), np.zeros(co))
    return p
