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
* the encoder-decoder built from them (levels of two convolutions, 2x
  average pooling down, nearest upsampling and concatenation with the
  level's encoder output up) with its forward and backward passes.

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
# The encoder-decoder.  Layer list: (name, ci, co, relu).  Level k = 1..L
# of the encoder works at 1/2^(k-1) resolution with widths base * k; the
# bottleneck (b1, b2) at 1/2^L keeps the last width; decoder layer dk
# takes [upsampled, encoder level k output] channels at level k.
# ---------------------------------------------------------------------------
def widths(base, levels):
    return [base * (k + 1) for k in range(levels)]


def layers(cin, cout, base, levels=3):
    ch = widths(base, levels)
    spec = []
    for k in range(levels):
        spec += [(f"e{k + 1}a", cin if k == 0 else ch[k - 1], ch[k], True), (f"e{k + 1}b", ch[k], ch[k], True)]
    spec += [("b1", ch[-1], ch[-1], True), ("b2", ch[-1], ch[-1], True)]
    up = ch[-1]
    for k in range(levels, 0, -1):
        spec.append((f"d{k}", up + ch[k - 1], ch[k - 1], True))
        up = ch[k - 1]
    spec.append(("out", ch[0], cout, False))
    return spec


def levels_of(spec):
    return sum(1 for l in spec if l[0].startswith("e") and l[0].endswith("a"))


def _same(a):
    return a


def forward(params, x, spec, store=_same):
    """params: {name: (w, b)}; returns (output, cache of activations).
    store(a) is applied to every stored activation (identity by default; a
    caller that emulates reduced-precision storage passes its rounding).
    The output layer's result is not passed through store."""
    L = levels_of(spec)
    spec = {l[0]: l for l in spec}
    a = {}

    def conv(name, inp):
        w, b = params[name]
        y = conv3d(inp, w, b)
        y = relu(y) if spec[name][3] else y
        return y if name == "out" else store(y)

    a["x"] = h = x
    for k in range(1, L + 1):
        if k > 1:
            h = a[f"p{k - 1}"] = store(pool2(a[f"e{k - 1}b"]))
        a[f"e{k}a"] = conv(f"e{k}a", h)
        a[f"e{k}b"] = conv(f"e{k}b", a[f"e{k}a"])
    a[f"p{L}"] = store(pool2(a[f"e{L}b"]))
    a["b1"] = conv("b1", a[f"p{L}"])
    h = a["b2"] = conv("b2", a["b1"])
    for k in range(L, 0, -1):
        a[f"c{k}"] = np.concatenate([up2(h), a[f"e{k}b"]], axis=-1)
        h = a[f"d{k}"] = conv(f"d{k}", a[f"c{k}"])
    a["out"] = conv("out", h)
    return a["out"], a


def backward(params, a, dout, spec, store=_same):
    """Gradients {name: (dw, db)} of the loss whose gradient with respect to
    the output is dout, and the gradient with respect to the input.
    store(g) is applied to the gradient at each convolution's output (after
    the ReLU mask) before both of its uses."""
    L = levels_of(spec)
    spec = {l[0]: l for l in spec}
    g = {}

    def conv_back(name, inp, dy):
        w, _ = params[name]
        if spec[name][3]:
            dy = relu_bwd(dy, a[name])
        dy = store(dy)
        g[name] = conv3d_bwd_weight(inp, dy)
        return conv3d_bwd_data(dy, w)

    dh = conv_back("out", a["d1"], dout)
    de = {}
    for k in range(1, L + 1):
        dc = conv_back(f"d{k}", a[f"c{k}"], dh)
        below = a[f"d{k + 1}"] if k < L else a["b2"]
        c_up = below.shape[-1]
        dh = up2_bwd(dc[..., :c_up])
        de[k] = dc[..., c_up:].copy()
    db1 = conv_back("b2", a["b1"], dh)
    dp = conv_back("b1", a[f"p{L}"], db1)
    for k in range(L, 0, -1):
        de[k] += pool2_bwd(dp)
        dea = conv_back(f"e{k}b", a[f"e{k}a"], de[k])
        dp = conv_back(f"e{k}a", a[f"p{k - 1}"] if k > 1 else a["x"], dea)
    return g, dp


def init_params(spec, seed):
    """He-uniform weights from a seeded generator, zero biases."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, ci, co, _ in spec:
        lim = np.sqrt(6.0 / (27 * ci))
        p[name] = (rng.uniform(-lim, lim, size=(27, co, ci)), np.zeros(co))
    return p
