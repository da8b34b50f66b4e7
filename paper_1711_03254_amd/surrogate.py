"""The warm-start surrogate: a 3D convolutional encoder-decoder run and
trained entirely by the kernels of include/lbm_nn.h.

It maps per-site features (solid mask, fraction of component A, distance
to the nearest solid) to the fields the solver reaches at steady state
(velocity in units of u_scale g / nu_mix, density changes in units of
rho_scale).  Layout: three encoder levels of two 3^3 convolutions (widths
base, 2 base, 3 base) separated by 2x average pooling, a bottleneck of two
convolutions at 1/8 resolution, one convolution per decoder level after
nearest upsampling and concatenation with the level's encoder output, ReLU
after every convolution but the last (base 32: 1.99 M parameters); 16 input and 16 output channels (the features and
targets occupy the first ones; the rest are zero and weighted 0 in the
loss).  Weights are FP32 masters with BF16 copies for the matrix cores;
Adam updates both.  torch provides device memory only.
"""
from __future__ import annotations

import numpy as np
import torch

from . import nn

CIN = 16     # padded input channels: [solid, phi_A, distance to the nearest solid / 8, 0, ...]
COUT = 16    # padded output channels: [ux, uy, uz, rho_A, rho_B, 0, ...] (u in units of u_scale g / nu_mix)
N_FEAT, N_TARGET = 3, 5
DIST_SCALE = 8.0


LEVELS = 3   # encoder levels; the bottleneck works at 1 / 2^LEVELS resolution


def widths(base, levels=LEVELS):
    """Channels of encoder level k = 1..levels: base * k."""
    return [base * (k + 1) for k in range(levels)]


def layer_spec(base, levels=LEVELS):
    """(name, ci, co, relu) of every convolution: two per encoder level
    (e1a, e1b at full resolution, e2a, e2b at 1/2, ...), two in the
    bottleneck (b1, b2), one per decoder level (dk reads [upsampled, ekb]),
    and the linear output layer."""
    ch = widths(base, levels)
    spec = []
    for k in range(levels):
        spec += [(f"e{k + 1}a", CIN if k == 0 else ch[k - 1], ch[k], True), (f"e{k + 1}b", ch[k], ch[k], True)]
    spec += [("b1", ch[-1], ch[-1], True), ("b2", ch[-1], ch[-1], True)]
    up = ch[-1]
    for k in range(levels, 0, -1):
        spec.append((f"d{k}", up + ch[k - 1], ch[k - 1], True))
        up = ch[k - 1]
    spec.append(("out", ch[0], COUT, False))
    return spec


class Surrogate:
    def __init__(self, base=32, seed=0, device="cuda"):
        self.base = base
        self.spec = layer_spec(base)
        self.dev = torch.device(device)
        # one flat FP32 buffer of all parameters: per layer w [27, co, ci] then b [co]
        self.offsets = {}
        n = 0
        for name, ci, co, _ in self.spec:
            self.offsets[name] = (n, n + 27 * co * ci)
            n += 27 * co * ci + co
        self.n_params = n
        rng = np.random.default_rng(seed)
        host = np.zeros(n, np.float32)
        for name, ci, co, _ in self.spec:   # He-uniform weights (the linear output layer 10x smaller), zero biases
            lim = np.sqrt(6.0 / (27 * ci)) * (0.1 if name == "out" else 1.0)
            w0, b0 = self.offsets[name]
            host[w0:b0] = rng.uniform(-lim, lim, 27 * co * ci).astype(np.float32)
        self.u_scale = 1.0
        self.rho_scale = 1.0
        self._alloc_params(torch.from_numpy(host))
        self.dims = None

    # -- parameters -----------------------------------------------------------
    def _alloc_params(self, host):
        d = self.dev
        self.p = host.to(d).contiguous()
        self.g = torch.zeros_like(self.p)
        self.m = torch.zeros_like(self.p)
        self.v = torch.zeros_like(self.p)
        self.pb = torch.zeros(self.n_params, dtype=torch.int16, device=d)
        self.wt = {name: torch.zeros(27 * co * ci, dtype=torch.int16, device=d) for name, ci, co, _ in self.spec}
        self.t = 0
        nn.to_bf16(self.p, self.pb)
        self._flip()

    def _flip(self):
        for name, ci, co, _ in self.spec:
            nn.weights_flip(self.w_bf16(name), self.wt[name], ci, co)

    def w_bf16(self, name):
        w0, b0 = self.offsets[name]
        return self.pb[w0:b0]

    def bias(self, name):
        _, b0 = self.offsets[name]
        co = [s for s in self.spec if s[0] == name][0][2]
        return self.p[b0:b0 + co]

    def grads(self, name):
        w0, b0 = self.offsets[name]
        co = [s for s in self.spec if s[0] == name][0][2]
        return self.g[w0:b0], self.g[b0:b0 + co]

    def set_params(self, host_flat, u_scale=1.0, rho_scale=1.0):
        self.u_scale = float(u_scale)
        self.rho_scale = float(rho_scale)
        self._alloc_params(torch.as_tensor(np.asarray(host_flat, np.float32)))

    def params_numpy(self):
        return self.p.cpu().numpy()

    def save(self, path):
        np.savez(path, params=self.params_numpy(), base=self.base, levels=LEVELS, u_scale=self.u_scale,
                 rho_scale=self.rho_scale)

    @classmethod
    def load(cls, path, device="cuda"):
        z = np.load(path, allow_pickle=False)
        if "levels" not in z or int(z["levels"]) != LEVELS:
            raise ValueError(f"{path}: weights of a network with another number of levels")
        s = cls(base=int(z["base"]), device=device)
        s.set_params(z["params"], float(z["u_scale"]), float(z["rho_scale"]))
        return s

    # -- activations ----------------------------------------------------------
    def _alloc(self, dims):
        if self.dims == dims:
            return
        nb, d, h, w = dims
        L = LEVELS
        m = 1 << L
        assert d % m == 0 and h % m == 0 and w % m == 0, f"extents must be multiples of {m}"
        ch = widths(self.base, L)
        self.ch = ch
        # dims and positions of level k (0 = full resolution ... L = bottleneck)
        self.ldims = [(nb, d >> k, h >> k, w >> k) for k in range(L + 1)]
        P = [nb * (d >> k) * (h >> k) * (w >> k) for k in range(L + 1)]
        self.P = P
        # channels upsampled into decoder level k (1-based): b2 for the deepest, else d(k+1)
        self.up = {k: ch[k] if k < L else ch[L - 1] for k in range(1, L + 1)}
        bf = dict(dtype=torch.int16, device=self.dev)
        f32 = dict(dtype=torch.float32, device=self.dev)
        A, G = {}, {}
        A["x"] = torch.zeros(P[0] * CIN, **bf)
        G["x"] = torch.zeros(P[0] * CIN, **f32)
        for k in range(1, L + 1):
            c, cin = ch[k - 1], self.up[k] + ch[k - 1]
            A[f"e{k}a"] = torch.zeros(P[k - 1] * c, **bf)
            A[f"c{k}"] = torch.zeros(P[k - 1] * cin, **bf)      # [up(d(k+1) or b2), e(k)b]
            A[f"p{k}"] = torch.zeros(P[k] * c, **bf)
            A[f"d{k}"] = torch.zeros(P[k - 1] * c, **bf)
            G[f"e{k}a"] = torch.zeros(P[k - 1] * c, **f32)
            G[f"c{k}"] = torch.zeros(P[k - 1] * cin, **f32)
            G[f"p{k}"] = torch.zeros(P[k] * c, **f32)
            G[f"d{k}"] = torch.zeros(P[k - 1] * c, **f32)
        A["b1"] = torch.zeros(P[L] * ch[-1], **bf)
        A["b2"] = torch.zeros(P[L] * ch[-1], **bf)
        G["b1"] = torch.zeros(P[L] * ch[-1], **f32)
        G["b2"] = torch.zeros(P[L] * ch[-1], **f32)
        A["out"] = torch.zeros(P[0] * COUT, **f32)
        G["dout"] = torch.zeros(P[0] * COUT, **f32)
        work, gmax = 0, 0
        for name, ci, co, _ in self.spec:
            lv = self._level(name)
            work = max(work, nn.bwd_weight_work(self.ldims[lv], ci, co))
            gmax = max(gmax, P[lv] * co)
        G["bf"] = torch.zeros(gmax, **bf)   # bf16 gradient at a layer output
        G["work"] = torch.zeros(work, **f32)
        self.loss_buf = torch.zeros(257, dtype=torch.float64, device=self.dev)
        self.A, self.G, self.dims = A, G, dims

    @staticmethod
    def _level(name):
        """Resolution level (0 = full) a layer works at."""
        if name == "out":
            return 0
        if name in ("b1", "b2"):
            return LEVELS
        return int(name[1]) - 1

    # -- forward / backward ---------------------------------------------------
    def forward(self, x_bf16, dims):
        """x_bf16: int16 tensor [P0 * 16] (features, bf16 bits).  Returns the
        FP32 output tensor [P0 * 16] (owned by the surrogate)."""
        self._alloc(dims)
        A, ch, L, V, D = self.A, self.ch, LEVELS, nn.View, self.ldims
        A["x"].copy_(x_bf16)

        def conv(name, src, dst, lv, ci, co, relu):
            nn.conv3d_fwd(src, self.w_bf16(name), self.bias(name), dst, relu, D[lv], ci, co)

        h, hc = V(A["x"], CIN), CIN
        for k in range(1, L + 1):
            c, cin = ch[k - 1], self.up[k] + ch[k - 1]
            if k > 1:
                nn.pool2_fwd(V(A[f"c{k - 1}"], self.up[k - 1] + ch[k - 2], self.up[k - 1]), V(A[f"p{k - 1}"], ch[k - 2]),
                             D[k - 2], ch[k - 2])
                h, hc = V(A[f"p{k - 1}"], ch[k - 2]), ch[k - 2]
            conv(f"e{k}a", h, V(A[f"e{k}a"], c), k - 1, hc, c, True)
            conv(f"e{k}b", V(A[f"e{k}a"], c), V(A[f"c{k}"], cin, self.up[k]), k - 1, c, c, True)
        cL = ch[-1]
        nn.pool2_fwd(V(A[f"c{L}"], self.up[L] + cL, self.up[L]), V(A[f"p{L}"], cL), D[L - 1], cL)
        conv("b1", V(A[f"p{L}"], cL), V(A["b1"], cL), L, cL, cL, True)
        conv("b2", V(A["b1"], cL), V(A["b2"], cL), L, cL, cL, True)
        h, hc = V(A["b2"], cL), cL
        for k in range(L, 0, -1):
            c, cin = ch[k - 1], self.up[k] + ch[k - 1]
            nn.up2_fwd(h, V(A[f"c{k}"], cin, 0), D[k], hc)
            conv(f"d{k}", V(A[f"c{k}"], cin), V(A[f"d{k}"], c), k - 1, cin, c, True)
            h, hc = V(A[f"d{k}"], c), c
        conv("out", h, V(A["out"], COUT), 0, ch[0], COUT, False)
        return A["out"]

    def backward(self, need_dx=False):
        """Gradients of the loss whose output gradient is in G['dout'] into
        self.g (and the input gradient into G['x'] when asked)."""
        A, G, ch, L, V, D, P = self.A, self.G, self.ch, LEVELS, nn.View, self.ldims, self.P
        gb = G["bf"]

        def layer_back(name, x_in: nn.View, y_out, dy: nn.View, lv, ci, co, relu, dx_out):
            """dy: FP32 gradient at the layer output; dx_out: FP32 view for the
            input gradient (or None)."""
            g = V(gb, co)
            nn.relu_bwd_cast(dy, y_out, g, P[lv], co, relu)
            dw, db = self.grads(name)
            nn.conv3d_bwd_weight(x_in, g, dw, db, G["work"], D[lv], ci, co)
            if dx_out is not None:
                nn.conv3d_fwd(g, self.wt[name], None, dx_out, False, D[lv], co, ci)

        layer_back("out", V(A["d1"], ch[0]), None, V(G["dout"], COUT), 0, ch[0], COUT, False, V(G["d1"], ch[0]))
        for k in range(1, L + 1):
            c, up = ch[k - 1], self.up[k]
            cin = up + c
            layer_back(f"d{k}", V(A[f"c{k}"], cin), V(A[f"d{k}"], c), V(G[f"d{k}"], c), k - 1, cin, c, True,
                       V(G[f"c{k}"], cin))
            below = G[f"d{k + 1}"] if k < L else G["b2"]
            nn.up2_bwd(V(G[f"c{k}"], cin, 0), V(below, up), D[k], up)
        cL = ch[-1]
        layer_back("b2", V(A["b1"], cL), V(A["b2"], cL), V(G["b2"], cL), L, cL, cL, True, V(G["b1"], cL))
        layer_back("b1", V(A[f"p{L}"], cL), V(A["b1"], cL), V(G["b1"], cL), L, cL, cL, True, V(G[f"p{L}"], cL))
        for k in range(L, 0, -1):
            c, up = ch[k - 1], self.up[k]
            cin = up + c
            de = V(G[f"c{k}"], cin, up)
            nn.pool2_bwd(V(G[f"p{k}"], c), de, True, D[k - 1], c)
            layer_back(f"e{k}b", V(A[f"e{k}a"], c), V(A[f"c{k}"], cin, up), de, k - 1, c, c, True,
                       V(G[f"e{k}a"], c))
            if k > 1:
                cp = ch[k - 2]
                src, ci, dxo = V(A[f"p{k - 1}"], cp), cp, V(G[f"p{k - 1}"], cp)
            else:
                src, ci, dxo = V(A["x"], CIN), CIN, (V(G["x"], CIN) if need_dx else None)
            layer_back(f"e{k}a", src, V(A[f"e{k}a"], c), V(G[f"e{k}a"], c), k - 1, ci, c, True, dxo)

    def loss_and_grad(self, target, cw):
        """MSE of the last forward output against target (FP32 [P0 * 16]);
        its gradient goes to G['dout'].  Returns the loss (a device scalar)."""
        P0 = self.dims[0] * self.dims[1] * self.dims[2] * self.dims[3]
        nn.mse(nn.View(self.A["out"], COUT), nn.View(target, COUT), cw, nn.View(self.G["dout"], COUT), self.loss_buf,
               P0, COUT)
        return self.loss_buf[0]

    def adam_step(self, lr):
        self.t += 1
        nn.adam(self.p, self.g, self.m, self.v, self.pb, lr, self.t)
        self._flip()

    def train_step(self, x_bf16, target, cw, dims, lr):
        self.forward(x_bf16, dims)
        loss = self.loss_and_grad(target, cw)
        self.backward()
        self.adam_step(lr)
        return loss


# -- features and targets ------------------------------------------------------
DIST_RADIUS = 24   # the distance feature is exact up to this many sites along each axis


def _dev(a, dtype):
    """A device tensor of the given dtype from a numpy array or a tensor."""
    if isinstance(a, torch.Tensor):
        return a.to(device="cuda", dtype=dtype).contiguous()
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def features(solid, rho_a, rho_b):
    """bf16 input tensor [P * 16] of one sample, built on the GPU from the
    mask and the initial densities, (nz, ny, nx) arrays or device tensors:
    the mask, the fraction of A, and the mask's periodic distance to the
    nearest solid site / DIST_SCALE (nn_solid_distance, nn_features)."""
    shape = tuple(np.shape(solid))
    s = _dev(solid, torch.uint8).reshape(-1)
    a = _dev(rho_a, torch.float64).reshape(-1)
    b = _dev(rho_b, torch.float64).reshape(-1)
    n = s.numel()
    work = torch.empty(2 * n, dtype=torch.float32, device="cuda")
    dist = torch.empty(n, dtype=torch.float32, device="cuda")
    nn.solid_distance(s, work, dist, shape, DIST_RADIUS)
    out = torch.empty(n * CIN, dtype=torch.int16, device="cuda")
    nn.features(s, a, b, dist, DIST_SCALE, nn.View(out, CIN), CIN)
    return out


def targets(u, rho_a, rho_b, u_scale, mobility, base_a, base_b, rho_scale=1.0, device="cuda"):
    """FP32 target tensor [P * 16]: u / (mobility u_scale) for u (3, ...),
    and the changes (rho_A - base_a) / rho_scale, (rho_B - base_b) /
    rho_scale of the densities from the initial ones.  mobility (per site) carries the known scaling of slow flow
    with the forcing and the viscosity, g / nu_mix, so that the network
    learns the geometry's part of the flow only."""
    n = np.asarray(rho_a).size
    t = np.zeros((n, COUT), np.float32)
    u = np.asarray(u).reshape(3, -1)
    m = np.asarray(mobility, np.float64).reshape(1, -1) * u_scale
    t[:, 0:3] = np.divide(u, m, out=np.zeros_like(u), where=m > 0).T   # zero where the mobility is (solid sites)
    t[:, 3] = ((np.asarray(rho_a) - np.asarray(base_a)) / rho_scale).reshape(-1)
    t[:, 4] = ((np.asarray(rho_b) - np.asarray(base_b)) / rho_scale).reshape(-1)
    return torch.from_numpy(t.reshape(-1)).to(device)


def loss_weights(device="cuda"):
    w = np.zeros(COUT, np.float32)
    w[:N_TARGET] = 1.0
    return torch.from_numpy(w).to(device)


def decode_device(net, out, solid, rho_a0, rho_b0, nu, g, floor=1e-3):
    """The warm state on the GPU from the network's output (nn_decode_fields):
    u (3 P), rho_A, rho_B (P each) as float64 device tensors, densities
    floored and rescaled to the initial component masses."""
    s = _dev(solid, torch.uint8).reshape(-1)
    a0 = _dev(rho_a0, torch.float64).reshape(-1)
    b0 = _dev(rho_b0, torch.float64).reshape(-1)
    n = s.numel()
    u = torch.empty(3 * n, dtype=torch.float64, device="cuda")
    ra = torch.empty(n, dtype=torch.float64, device="cuda")
    rb = torch.empty(n, dtype=torch.float64, device="cuda")
    work = torch.empty(4096, dtype=torch.float64, device="cuda")
    nn.decode_fields(nn.View(out, COUT), s, a0, b0, float(nu[0]), float(nu[1]), float(g), net.u_scale, net.rho_scale,
                     floor, u, ra, rb, work)
    return u, ra, rb


def decode(out, shape, u_scale, mobility, base_a, base_b, rho_scale=1.0):
    """(u (3, ...), rho_A, rho_B) as float64 numpy arrays from the output
    (the inverse of targets)."""
    o = out.reshape(-1, COUT).double().cpu().numpy()
    u = (o[:, 0:3].T * u_scale * np.asarray(mobility).reshape(1, -1)).reshape((3,) + tuple(shape))
    return u, base_a + rho_scale * o[:, 3].reshape(shape), base_b + rho_scale * o[:, 4].reshape(shape)
