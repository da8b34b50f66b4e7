"""The warm-start surrogate: a 3D convolutional encoder-decoder run and
trained entirely by the kernels of include/lbm_nn.h.

It maps per-site features (solid mask, fraction of component A) to the
fields the solver reaches at steady state (velocity in units of
u_scale g / nu_mix, rho_A, rho_B).  Layout: two levels of 2x average
pooling, two 3^3 convolutions per level, a bottleneck at 1/4 resolution, nearest upsampling
with skip connections (channel concatenation), ReLU after every
convolution but the last; 16 input and 16 output channels (the features and
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


def layer_spec(base):
    c1, c2 = base, 2 * base
    return [("e1a", CIN, c1, True), ("e1b", c1, c1, True), ("e2a", c1, c2, True), ("e2b", c2, c2, True),
            ("b1", c2, c2, True), ("b2", c2, c2, True), ("d2", 2 * c2, c2, True), ("d1", c2 + c1, c1, True),
            ("out", c1, COUT, False)]


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
        for name, ci, co, _ in self.spec:   # He-uniform weights, zero biases
            lim = np.sqrt(6.0 / (27 * ci))
            w0, b0 = self.offsets[name]
            host[w0:b0] = rng.uniform(-lim, lim, 27 * co * ci).astype(np.float32)
        self.u_scale = 1.0
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

    def set_params(self, host_flat, u_scale=1.0):
        self.u_scale = float(u_scale)
        self._alloc_params(torch.as_tensor(np.asarray(host_flat, np.float32)))

    def params_numpy(self):
        return self.p.cpu().numpy()

    def save(self, path):
        np.savez(path, params=self.params_numpy(), base=self.base, u_scale=self.u_scale)

    @classmethod
    def load(cls, path, device="cuda"):
        z = np.load(path, allow_pickle=False)
        s = cls(base=int(z["base"]), device=device)
        s.set_params(z["params"], float(z["u_scale"]))
        return s

    # -- activations ----------------------------------------------------------
    def _alloc(self, dims):
        if self.dims == dims:
            return
        nb, d, h, w = dims
        assert d % 4 == 0 and h % 4 == 0 and w % 4 == 0, "extents must be multiples of 4"
        c1, c2 = self.base, 2 * self.base
        P0, P1, P2 = nb * d * h * w, nb * d * h * w // 8, nb * d * h * w // 64
        bf = dict(dtype=torch.int16, device=self.dev)
        f32 = dict(dtype=torch.float32, device=self.dev)
        A = {}
        A["x"] = torch.zeros(P0 * CIN, **bf)
        A["e1a"] = torch.zeros(P0 * c1, **bf)
        A["c1"] = torch.zeros(P0 * (c2 + c1), **bf)      # [up(d2), e1b]
        A["p1"] = torch.zeros(P1 * c1, **bf)
        A["e2a"] = torch.zeros(P1 * c2, **bf)
        A["c2"] = torch.zeros(P1 * 2 * c2, **bf)         # [up(b2), e2b]
        A["p2"] = torch.zeros(P2 * c2, **bf)
        A["b1"] = torch.zeros(P2 * c2, **bf)
        A["b2"] = torch.zeros(P2 * c2, **bf)
        A["d2"] = torch.zeros(P1 * c2, **bf)
        A["d1"] = torch.zeros(P0 * c1, **bf)
        A["out"] = torch.zeros(P0 * COUT, **f32)
        G = {}
        G["dout"] = torch.zeros(P0 * COUT, **f32)
        G["d1"] = torch.zeros(P0 * c1, **f32)
        G["c1"] = torch.zeros(P0 * (c2 + c1), **f32)
        G["d2"] = torch.zeros(P1 * c2, **f32)
        G["c2"] = torch.zeros(P1 * 2 * c2, **f32)
        G["b2"] = torch.zeros(P2 * c2, **f32)
        G["b1"] = torch.zeros(P2 * c2, **f32)
        G["p2"] = torch.zeros(P2 * c2, **f32)
        G["e2a"] = torch.zeros(P1 * c2, **f32)
        G["p1"] = torch.zeros(P1 * c1, **f32)
        G["e1a"] = torch.zeros(P0 * c1, **f32)
        G["x"] = torch.zeros(P0 * CIN, **f32)
        G["bf"] = torch.zeros(P0 * max(c2 + c1, COUT), **bf)   # bf16 gradient at a layer output
        work = 0
        dims1, dims2 = (nb, d // 2, h // 2, w // 2), (nb, d // 4, h // 4, w // 4)
        for name, ci, co, _ in self.spec:
            dd = dims if name in ("e1a", "e1b", "d1", "out") else (dims1 if name in ("e2a", "e2b", "d2") else dims2)
            work = max(work, nn.bwd_weight_work(dd, ci, co))
        G["work"] = torch.zeros(work, **f32)
        self.loss_buf = torch.zeros(257, dtype=torch.float64, device=self.dev)
        self.A, self.G, self.dims = A, G, dims
        self.dims1, self.dims2 = dims1, dims2

    # -- forward / backward ---------------------------------------------------
    def forward(self, x_bf16, dims):
        """x_bf16: int16 tensor [P0 * 16] (features, bf16 bits).  Returns the
        FP32 output tensor [P0 * 16] (owned by the surrogate)."""
        self._alloc(dims)
        A, c1, c2 = self.A, self.base, 2 * self.base
        A["x"].copy_(x_bf16)
        V = nn.View
        d0, d1, d2 = self.dims, self.dims1, self.dims2
        conv = lambda name, src, dst, dd, ci, co, relu: nn.conv3d_fwd(src, self.w_bf16(name), self.bias(name), dst,
                                                                      relu, dd, ci, co)
        conv("e1a", V(A["x"], CIN), V(A["e1a"], c1), d0, CIN, c1, True)
        e1b = V(A["c1"], c2 + c1, c2)
        conv("e1b", V(A["e1a"], c1), e1b, d0, c1, c1, True)
        nn.pool2_fwd(e1b, V(A["p1"], c1), d0, c1)
        conv("e2a", V(A["p1"], c1), V(A["e2a"], c2), d1, c1, c2, True)
        e2b = V(A["c2"], 2 * c2, c2)
        conv("e2b", V(A["e2a"], c2), e2b, d1, c2, c2, True)
        nn.pool2_fwd(e2b, V(A["p2"], c2), d1, c2)
        conv("b1", V(A["p2"], c2), V(A["b1"], c2), d2, c2, c2, True)
        conv("b2", V(A["b1"], c2), V(A["b2"], c2), d2, c2, c2, True)
        nn.up2_fwd(V(A["b2"], c2), V(A["c2"], 2 * c2, 0), d2, c2)
        conv("d2", V(A["c2"], 2 * c2), V(A["d2"], c2), d1, 2 * c2, c2, True)
        nn.up2_fwd(V(A["d2"], c2), V(A["c1"], c2 + c1, 0), d1, c2)
        conv("d1", V(A["c1"], c2 + c1), V(A["d1"], c1), d0, c2 + c1, c1, True)
        conv("out", V(A["d1"], c1), V(A["out"], COUT), d0, c1, COUT, False)
        return A["out"]

    def backward(self, need_dx=False):
        """Gradients of the loss whose output gradient is in G['dout'] into
        self.g (and the input gradient into G['x'] when asked)."""
        A, G, c1, c2 = self.A, self.G, self.base, 2 * self.base
        V = nn.View
        d0, d1, d2 = self.dims, self.dims1, self.dims2
        P0 = d0[0] * d0[1] * d0[2] * d0[3]
        P1, P2 = P0 // 8, P0 // 64
        gb = G["bf"]

        def layer_back(name, x_in: nn.View, y_out, dy: nn.View, dd, P, ci, co, relu, dx_out):
            """dy: FP32 gradient at the layer output; dx_out: FP32 view for the
            input gradient (or None)."""
            g = V(gb, co)
            nn.relu_bwd_cast(dy, y_out, g, P, co, relu)
            dw, db = self.grads(name)
            nn.conv3d_bwd_weight(x_in, g, dw, db, G["work"], dd, ci, co)
            if dx_out is not None:
                nn.conv3d_fwd(g, self.wt[name], None, dx_out, False, dd, co, ci)

        layer_back("out", V(A["d1"], c1), None, V(G["dout"], COUT), d0, P0, c1, COUT, False, V(G["d1"], c1))
        layer_back("d1", V(A["c1"], c2 + c1), V(A["d1"], c1), V(G["d1"], c1), d0, P0, c2 + c1, c1, True,
                   V(G["c1"], c2 + c1))
        nn.up2_bwd(V(G["c1"], c2 + c1, 0), V(G["d2"], c2), d1, c2)
        layer_back("d2", V(A["c2"], 2 * c2), V(A["d2"], c2), V(G["d2"], c2), d1, P1, 2 * c2, c2, True,
                   V(G["c2"], 2 * c2))
        nn.up2_bwd(V(G["c2"], 2 * c2, 0), V(G["b2"], c2), d2, c2)
        layer_back("b2", V(A["b1"], c2), V(A["b2"], c2), V(G["b2"], c2), d2, P2, c2, c2, True, V(G["b1"], c2))
        layer_back("b1", V(A["p2"], c2), V(A["b1"], c2), V(G["b1"], c2), d2, P2, c2, c2, True, V(G["p2"], c2))
        de2b = V(G["c2"], 2 * c2, c2)
        nn.pool2_bwd(V(G["p2"], c2), de2b, True, d1, c2)
        layer_back("e2b", V(A["e2a"], c2), V(A["c2"], 2 * c2, c2), de2b, d1, P1, c2, c2, True, V(G["e2a"], c2))
        layer_back("e2a", V(A["p1"], c1), V(A["e2a"], c2), V(G["e2a"], c2), d1, P1, c1, c2, True, V(G["p1"], c1))
        de1b = V(G["c1"], c2 + c1, c2)
        nn.pool2_bwd(V(G["p1"], c1), de1b, True, d0, c1)
        layer_back("e1b", V(A["e1a"], c1), V(A["c1"], c2 + c1, c2), de1b, d0, P0, c1, c1, True, V(G["e1a"], c1))
        layer_back("e1a", V(A["x"], CIN), V(A["e1a"], c1), V(G["e1a"], c1), d0, P0, CIN, c1, True,
                   V(G["x"], CIN) if need_dx else None)

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
def solid_distance(solid):
    """Euclidean distance of every site to the nearest solid site on the
    periodic lattice (the mask's geometry in the form that sets the local
    pore size); wide if there is no solid."""
    from scipy import ndimage
    solid = np.asarray(solid) != 0
    if not solid.any():
        return np.full(solid.shape, float(max(solid.shape)))
    pad = [min(n, 24) for n in solid.shape]
    big = np.pad(solid, [(p, p) for p in pad], mode="wrap")
    d = ndimage.distance_transform_edt(~big)
    return d[tuple(slice(p, p + n) for p, n in zip(pad, solid.shape))]


def features(solid, phi, device="cuda"):
    """bf16 input tensor [P * 16] from the mask and the A fraction of one
    sample, (nz, ny, nx) arrays: the mask, the fraction, and the mask's
    distance to solid (a function of the mask alone)."""
    s = np.asarray(solid, np.float32).reshape(-1)
    f = np.asarray(phi, np.float32).reshape(-1)
    dist = (solid_distance(solid) / DIST_SCALE).astype(np.float32).reshape(-1)
    x = torch.zeros((s.size, CIN), dtype=torch.float32, device=device)
    x[:, 0] = torch.from_numpy(s).to(device)
    x[:, 1] = torch.from_numpy(f).to(device)
    x[:, 2] = torch.from_numpy(dist).to(device)
    out = torch.zeros(s.size * CIN, dtype=torch.int16, device=device)
    nn.to_bf16(x.reshape(-1).contiguous(), out)
    return out


def targets(u, rho_a, rho_b, u_scale, mobility, base_a, base_b, device="cuda"):
    """FP32 target tensor [P * 16]: u / (mobility u_scale) for u (3, ...),
    and the changes rho_A - base_a, rho_B - base_b of the densities from the
    initial ones.  mobility (per site) carries the known scaling of slow flow
    with the forcing and the viscosity, g / nu_mix, so that the network
    learns the geometry's part of the flow only."""
    n = np.asarray(rho_a).size
    t = np.zeros((n, COUT), np.float32)
    u = np.asarray(u).reshape(3, -1)
    m = np.asarray(mobility, np.float64).reshape(1, -1) * u_scale
    t[:, 0:3] = np.divide(u, m, out=np.zeros_like(u), where=m > 0).T   # zero where the mobility is (solid sites)
    t[:, 3] = (np.asarray(rho_a) - np.asarray(base_a)).reshape(-1)
    t[:, 4] = (np.asarray(rho_b) - np.asarray(base_b)).reshape(-1)
    return torch.from_numpy(t.reshape(-1)).to(device)


def loss_weights(device="cuda"):
    w = np.zeros(COUT, np.float32)
    w[:N_TARGET] = 1.0
    return torch.from_numpy(w).to(device)


def decode(out, shape, u_scale, mobility, base_a, base_b):
    """(u (3, ...), rho_A, rho_B) as float64 numpy arrays from the output
    (the inverse of targets)."""
    o = out.reshape(-1, COUT).double().cpu().numpy()
    u = (o[:, 0:3].T * u_scale * np.asarray(mobility).reshape(1, -1)).reshape((3,) + tuple(shape))
    return u, base_a + o[:, 3].reshape(shape), base_b + o[:, 4].reshape(shape)
