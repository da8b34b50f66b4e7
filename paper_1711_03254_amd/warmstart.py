"""Learned warm start of the solver: solver-generated training data, the
measures that judge a solve, and the cold and warm solves.

The solver (include/lbm.h) is the method; the surrogate (surrogate.py)
only proposes an initial state.  A warm start takes the predicted
densities (rescaled so that the component masses equal those of the cold
initial state exactly) and velocity u_F, and restarts the solver from
them through lbm_set_fields_strain: each component's equilibrium at
u_F - F_a / (2 rho_a) (so that Eq. 8 gives back u_F) plus the
non-equilibrium part of the strain of u_F.  The plain step then runs on.

Two measures judge a solve, both taken by the library in FP64 on the
device:

* the residual r = max(||u_F(t) - u_F(t - K)|| / ||u_F(t)||,
  ||rho_A(t) - rho_A(t - K)|| / ||rho_A(t)||) over K steps (lbm_residual);
* the distance to a reference state, the same norms against the fields of
  a long cold FP64 solve (lbm_distance).

Time to steady state is compared at equal accuracy: the steps (and
seconds) each solve needs until its distance to the reference is below a
target in both u_F and rho_A, so the surrogate can only change how long a
solve takes, never what it converges to.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import inputs, lbm, surrogate

T0 = 1.0 / 3.0


def physics(g=1e-5, G=-1.0, rho_s=0.0):
    """The surrogate workload's physics: nu_A = 1/60, nu_B = 1/6 (ratio
    10), Shan-Chen coupling G (Eq. 7; -1 keeps a mixture of total density 1
    miscible, -G rho < 2), body force g along z, wall parameter rho_s.  The
    coupling layers the components at the walls; the densities then settle
    geometrically while u_F approaches its steady state only algebraically
    (a tail of slow modes)."""
    return dict(tau=(1.0 / 60.0 / T0 + 0.5, 1.0), G=G, g=(0.0, 0.0, g), rho_s=rho_s)


class Residual:
    """The residual above, taken by the library in FP64 on the device
    (lbm_residual) every K steps; the first sample only records the fields."""

    def __init__(self, ctx, shape=None):
        self.ctx, self.first = ctx, True

    def sample(self):
        du, da = lbm.lbm_residual(self.ctx)
        if self.first:
            self.first = False
            return None
        return max(du, da)


def run_to_residual(ctx, shape, tol=1e-6, every=100, max_steps=100000):
    """Steps the context until the residual is below tol (checked every
    `every` steps) or max_steps.  Returns (steps, converged, residuals)."""
    res = Residual(ctx, shape)
    res.sample()
    steps, hist = 0, []
    while steps < max_steps:
        lbm.lbm_step(ctx, every)
        steps += every
        r = res.sample()
        hist.append(r)
        if r is not None and r < tol:
            return steps, True, hist
    return steps, False, hist


def fields(ctx, shape):
    ra, rb, u = lbm.lbm_moments(ctx)
    return u.reshape((3,) + tuple(shape)), ra.reshape(shape), rb.reshape(shape)


def make_context(solid, ra, rb, phys, prec="fp32", u=None):
    n = solid.shape
    return lbm.lbm_init(lbm.Params(n[2], n[1], n[0], prec=lbm.PRECISIONS[prec], solid=solid, rho_init=(ra, rb),
                                   u_init=u, **phys))


def steady_sample(n, seed, phys, steps=60000, prec="fp64", kind="mixture", **case):
    """A subvolume and the near-steady state the plain solver reaches from
    it in `steps` steps (kind "mixture": inputs.mixture_case, "droplets":
    inputs.subvolume_case), with the residual over the last 100 steps."""
    gen = inputs.mixture_case if kind == "mixture" else inputs.subvolume_case
    solid, ra0, rb0, info = gen(n, seed, **case)
    ctx = make_context(solid, ra0, rb0, phys, prec)
    t = time.perf_counter()
    lbm.lbm_step(ctx, steps - 100)
    lbm.lbm_residual(ctx)
    lbm.lbm_step(ctx, 100)
    du, da = lbm.lbm_residual(ctx)
    wall = time.perf_counter() - t
    u, ra, rb = fields(ctx, solid.shape)
    lbm.lbm_free(ctx)
    return dict(solid=solid, ra0=ra0, rb0=rb0, info=info, u=u, ra=ra, rb=rb, steps=steps, residual=(du, da),
                seconds=wall)


def phi_of(solid, ra, rb):
    tot = ra + rb
    phi = np.where(tot > 0, ra / np.where(tot > 0, tot, 1.0), 0.0)
    return np.where(solid == 1, 0.0, phi)


def mobility(solid, ra0, rb0, phys):
    """g / nu_mix per site from the mixture viscosity of Eqs. (5)-(6) with
    p = rho_1 / rho (zero on solid sites)."""
    phi = phi_of(solid, ra0, rb0)
    nu = np.array(phys["tau"], np.float64) - 0.5
    nu *= T0
    nu_mix = phi * nu[0] + (1.0 - phi) * nu[1]
    g = float(np.linalg.norm(phys["g"]))
    return np.where(solid == 1, 0.0, g / nu_mix)


def nu_of(phys):
    """Kinematic viscosities (nu_A, nu_B) of Eq. (5)."""
    return tuple(T0 * (t - 0.5) for t in phys["tau"])


def warm_state(net, solid, ra0, rb0, phys, floor=1e-3):
    """The warm initial state for a cold one (solid, ra0, rb0), computed on
    the GPU: features, the network, and the decoded fields (the predicted
    velocity u_F and densities, floored at `floor` and rescaled to the cold
    state's component masses).  Returns float64 device tensors (u (3 P),
    rho_A, rho_B)."""
    x = surrogate.features(solid, ra0, rb0)
    out = net.forward(x, (1,) + tuple(solid.shape))
    g = float(np.linalg.norm(phys["g"]))
    return surrogate.decode_device(net, out, solid, ra0, rb0, nu_of(phys), g, floor)


def reference(solid, ra0, rb0, phys, steps):
    """The reference state: `steps` cold FP64 steps.  Returns device tensors
    (rho_A, u_F) and the residual over the last 100 steps."""
    ctx = make_context(solid, ra0, rb0, phys, "fp64")
    lbm.lbm_step(ctx, steps - 100)
    lbm.lbm_residual(ctx)
    lbm.lbm_step(ctx, 100)
    res = lbm.lbm_residual(ctx)
    n = solid.size
    ra = torch.zeros(n, dtype=torch.float64, device="cuda")
    u = torch.zeros(3 * n, dtype=torch.float64, device="cuda")
    lbm.lbm_moments(ctx, ra, None, u)
    torch.cuda.synchronize()
    lbm.lbm_free(ctx)
    return ra, u, res


def solve_to_accuracy(solid, ra, rb, phys, ref, targets, u=None, prec="fp32", every=500, max_steps=40000,
                      early=(50, 100, 200, 300, 400)):
    """One solve from (ra, rb) (and, for a warm start, u_F: restart through
    lbm_set_fields_strain; host arrays or device tensors) until its
    distance to the reference (rho_A, u_F) is below each target (eps_u,
    eps_a) in turn, or max_steps.  The distance is judged after the `early`
    step counts and then every `every` steps.  The clock runs over the
    restart and the steps (synchronized per chunk), not over context
    creation or the distance checks.  Returns per target the steps and
    seconds to reach it (None if not reached), the distance trajectory and
    the final distance."""
    ra_h = ra.cpu().numpy().reshape(solid.shape) if isinstance(ra, torch.Tensor) else ra
    rb_h = rb.cpu().numpy().reshape(solid.shape) if isinstance(rb, torch.Tensor) else rb
    ctx = make_context(solid, ra_h, rb_h, phys, prec)
    secs = 0.0
    if u is not None:
        torch.cuda.synchronize()
        t = time.perf_counter()
        lbm.lbm_set_fields_strain(ctx, ra, rb, u)
        secs = time.perf_counter() - t
    ref_a, ref_u = ref
    d0 = lbm.lbm_distance(ctx, ref_a, ref_u)
    traj = [(0, d0[0], d0[1])]
    reached = [None] * len(targets)
    steps = 0

    def mark(du, da):
        for k, (eu, ea) in enumerate(targets):
            if reached[k] is None and du <= eu and da <= ea:
                reached[k] = (steps, secs)

    mark(*d0)
    marks = [e for e in sorted(early) if 0 < e < min(every, max_steps)]
    while steps < max_steps and any(r is None for r in reached):
        nxt = min(marks.pop(0) if marks else (steps // every + 1) * every, max_steps)
        torch.cuda.synchronize()
        t = time.perf_counter()
        lbm.lbm_step(ctx, nxt - steps)
        torch.cuda.synchronize()
        secs += time.perf_counter() - t
        steps = nxt
        du, da = lbm.lbm_distance(ctx, ref_a, ref_u)
        traj.append((steps, du, da))
        mark(du, da)
    lbm.lbm_free(ctx)
    return dict(reached=[None if r is None else {"steps": r[0], "seconds": r[1]} for r in reached],
                final=traj[-1], trajectory=traj, ms_per_step=1e3 * secs / max(steps, 1))


def compare(net, case, phys, ref, targets, precs=("fp32", "fp16s"), every=500, max_steps=40000):
    """Cold and warm solves of one case (dict solid, ra0, rb0) at each
    storage precision, to each accuracy target against the reference
    (device rho_A, u_F): the cold start, the cold fields restarted
    consistently (u_F = 0), the network's velocity on the cold densities,
    and the network's velocity and densities.  A warm solve's seconds
    include the prediction (features, the network and the decoding on the
    GPU from the cold fields already in device memory, and the restart).
    Returns per precision every solve, the prediction's own distance to the
    reference, and per target the steps and time factors cold / other (None
    where a solve did not reach the target)."""
    solid, ra0, rb0 = case["solid"], case["ra0"], case["rb0"]
    solid_d = torch.from_numpy(np.ascontiguousarray(solid, np.uint8)).cuda()
    ra0_d = torch.from_numpy(np.ascontiguousarray(ra0, np.float64)).cuda()
    rb0_d = torch.from_numpy(np.ascontiguousarray(rb0, np.float64)).cuda()
    warm_state(net, solid_d, ra0_d, rb0_d, phys)    # first call: allocations
    torch.cuda.synchronize()
    t = time.perf_counter()
    u, ra, rb = warm_state(net, solid_d, ra0_d, rb0_d, phys)
    torch.cuda.synchronize()
    t_pred = time.perf_counter() - t
    fluid = solid == 0
    ref_a = ref[0].cpu().numpy().reshape(solid.shape)
    ref_u = ref[1].cpu().numpy().reshape((3,) + solid.shape)
    u_h = u.cpu().numpy().reshape((3,) + solid.shape)
    ra_h = ra.cpu().numpy().reshape(solid.shape)
    out = {"predict_seconds": t_pred,
           "prediction_distance": {
               "u": float(np.linalg.norm((u_h - ref_u)[:, fluid]) / np.linalg.norm(ref_u[:, fluid])),
               "rho_a": float(np.linalg.norm((ra_h - ref_a)[fluid]) / np.linalg.norm(ref_a[fluid]))},
           "cold_start_distance": {
               "u": 1.0, "rho_a": float(np.linalg.norm((ra0 - ref_a)[fluid]) / np.linalg.norm(ref_a[fluid]))},
           "targets": [list(t) for t in targets]}
    zero = torch.zeros_like(u)
    for prec in precs:
        arms = {
            # the method's own start: f_eq(rho0, 0) (lbm_init)
            "cold": solve_to_accuracy(solid, ra0, rb0, phys, ref, targets, None, prec, every, max_steps),
            # the same fields restarted consistently: u_F = 0, i.e. each
            # component's population momentum -F_a / 2 (what a warm start
            # gains from the restart alone, without the network)
            "cold_consistent": solve_to_accuracy(solid, ra0_d, rb0_d, phys, ref, targets, zero, prec, every,
                                                 max_steps),
            # the network's velocity on the cold densities
            "warm_u": solve_to_accuracy(solid, ra0_d, rb0_d, phys, ref, targets, u, prec, every, max_steps),
            # the network's velocity and densities
            "warm": solve_to_accuracy(solid, ra, rb, phys, ref, targets, u, prec, every, max_steps),
        }
        factors = {}
        for name in ("cold_consistent", "warm_u", "warm"):
            fs = []
            for c, w in zip(arms["cold"]["reached"], arms[name]["reached"]):
                if c is None or w is None:
                    fs.append(None)
                    continue
                ws = w["seconds"] + (t_pred if name.startswith("warm") else 0.0)
                fs.append({"steps": c["steps"] / max(w["steps"], 1), "time": c["seconds"] / ws if ws > 0 else None})
            factors[name] = fs
        for r in arms.values():
            r["trajectory"] = r["trajectory"][:: max(1, len(r["trajectory"]) // 40)]
        out[prec] = {**arms, "factors": factors}
    return out


def train(net, samples, phys, epochs, lr=5e-4, log=None, lr_end=None, time_budget=None, warmup=5):
    """Adam on the surrogate's own kernels over solver-generated samples
    (each a dict of steady_sample): the learning rate rises linearly from
    lr / warmup to lr over the first `warmup` epochs, then falls linearly
    to lr_end (default lr / 10) over the rest.  Returns the per-epoch mean
    loss."""
    cw = surrogate.loss_weights()
    data = []
    for s in samples:
        x = surrogate.features(s["solid"], s["ra0"], s["rb0"])
        t = surrogate.targets(s["u"], s["ra"], s["rb"], net.u_scale, mobility(s["solid"], s["ra0"], s["rb0"], phys),
                              s["ra0"], s["rb0"], net.rho_scale)
        data.append((x, t, (1,) + tuple(s["solid"].shape)))
    hist = []
    lr_end = lr / 10 if lr_end is None else lr_end
    t0 = time.perf_counter()
    for ep in range(epochs):
        if time_budget is not None and time.perf_counter() - t0 > time_budget:
            break
        tot = 0.0
        lr_ep = lr + (lr_end - lr) * ep / max(epochs - 1, 1)
        if ep < warmup:
            lr_ep = lr * (ep + 1) / warmup
        for x, t, dims in data:
            tot += float(net.train_step(x, t, cw, dims, lr_ep))
        hist.append(tot / len(data))
        if log:
            log(ep, hist[-1])
    return hist


def u_scale_of(samples, phys):
    """RMS over the samples' fluid sites of u / mobility: the velocity unit
    of the outputs."""
    acc, n = 0.0, 0
    for s in samples:
        f = s["solid"] == 0
        m = mobility(s["solid"], s["ra0"], s["rb0"], phys)
        acc += float(((s["u"][:, f] / m[f]) ** 2).sum())
        n += int(f.sum()) * 3
    return float(np.sqrt(acc / max(n, 1))) or 1.0


def rho_scale_of(samples):
    """RMS over the samples' fluid sites of the density changes from the
    initial state: the density unit of the outputs."""
    acc, n = 0.0, 0
    for s in samples:
        f = s["solid"] == 0
        acc += float(((s["ra"] - s["ra0"])[f] ** 2).sum() + ((s["rb"] - s["rb0"])[f] ** 2).sum())
        n += 2 * int(f.sum())
    return float(np.sqrt(acc / max(n, 1))) or 1.0
