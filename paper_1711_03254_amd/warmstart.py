"""Learned warm start of the solver: solver-generated training data, the
residual that judges convergence, and the warm-started solve.

The solver (include/lbm.h) is the method; the surrogate (surrogate.py)
only proposes an initial state.  Every solve, cold or warm, runs the plain
FP32 step until the residual

    r = max(||u_F(t) - u_F(t - K)|| / ||u_F(t)||, ||rho_A(t) - rho_A(t - K)|| / ||rho_A(t)||)

(2-norms over the lattice, K = `every` steps) falls below `tol`, so the
surrogate can only change how long that takes, never the answer's
definition.  A warm start rescales each predicted component density so
that the component masses equal those of the cold initial state exactly.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import inputs, lbm, surrogate

T0 = 1.0 / 3.0


def physics(g=1e-4, G=0.0, rho_s=0.0):
    """The surrogate workload's physics: nu_A = 1/60, nu_B = 1/6 (ratio
    10), Shan-Chen coupling G, body force g along z, wall parameter rho_s.
    The default is the miscible mixture without coupling, whose flow has a
    steady state that the residual reaches geometrically (with a coupling,
    density layers at the walls relax only algebraically)."""
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


def steady_sample(n, seed, phys, tol=1e-6, every=100, max_steps=100000, kind="mixture", prec="fp32", **case):
    """A subvolume and the steady state the plain solver reaches from it
    (kind "mixture": inputs.mixture_case, "droplets": inputs.subvolume_case)."""
    gen = inputs.mixture_case if kind == "mixture" else inputs.subvolume_case
    solid, ra0, rb0, info = gen(n, seed, **case)
    ctx = make_context(solid, ra0, rb0, phys, prec)
    t = time.perf_counter()
    steps, conv, hist = run_to_residual(ctx, solid.shape, tol, every, max_steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t
    u, ra, rb = fields(ctx, solid.shape)
    lbm.lbm_free(ctx)
    return dict(solid=solid, ra0=ra0, rb0=rb0, info=info, u=u, ra=ra, rb=rb, steps=steps, converged=conv,
                seconds=wall, residuals=hist)


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


def predict(net, solid, ra0, rb0, phys):
    """The surrogate's fields (u, rho_A, rho_B) for a cold initial state."""
    shape = solid.shape
    x = surrogate.features(solid, phi_of(solid, ra0, rb0))
    out = net.forward(x, (1,) + tuple(shape))
    return surrogate.decode(out, shape, net.u_scale, mobility(solid, ra0, rb0, phys), ra0, rb0)


def warm_state(net, solid, ra0, rb0, phys, densities=True, floor=1e-3):
    """The warm initial state for a cold one (solid, ra0, rb0): the predicted
    velocity and, with densities, the predicted densities rescaled to the
    cold state's component masses (else the cold densities)."""
    u, ra, rb = predict(net, solid, ra0, rb0, phys)
    fluid = solid == 0
    if densities:
        ra = np.where(fluid, np.maximum(ra, floor), 0.0)
        rb = np.where(fluid, np.maximum(rb, floor), 0.0)
        ra *= ra0[fluid].sum() / ra[fluid].sum()
        rb *= rb0[fluid].sum() / rb[fluid].sum()
    else:
        ra, rb = ra0, rb0
    u = np.where(fluid[None], u, 0.0)
    return (np.ascontiguousarray(u, np.float64), np.ascontiguousarray(ra, np.float64),
            np.ascontiguousarray(rb, np.float64))


def compare(net, sample, phys, tol, prec="fp32", every=100, max_steps=100000, densities=False):
    """Cold and warm solves of one sample to the same residual: steps, wall
    time of each solve and of the prediction (features on the host, the
    network on the GPU), and the difference of the two converged states
    (relative 2-norm over u and over rho_A)."""
    solid, ra0, rb0 = sample["solid"], sample["ra0"], sample["rb0"]
    cold = solve(solid, ra0, rb0, phys, None, tol, every, max_steps, prec)
    t = time.perf_counter()
    u, ra, rb = warm_state(net, solid, ra0, rb0, phys, densities)
    torch.cuda.synchronize()
    t_pred = time.perf_counter() - t
    warm = solve(solid, ra, rb, phys, u, tol, every, max_steps, prec)
    (uc, rac, _), (uw, raw, _) = cold["fields"], warm["fields"]
    du = float(np.linalg.norm(uw - uc) / np.linalg.norm(uc))
    da = float(np.linalg.norm(raw - rac) / np.linalg.norm(rac))
    pu, pa, _ = predict(net, solid, ra0, rb0, phys)
    fluid = solid == 0
    eu = float(np.linalg.norm((pu - uc)[:, fluid]) / np.linalg.norm(uc[:, fluid]))
    ea = float(np.linalg.norm((pa - rac)[fluid]) / np.linalg.norm(rac[fluid]))
    return dict(cold_steps=cold["steps"], warm_steps=warm["steps"], cold_converged=cold["converged"],
                warm_converged=warm["converged"], cold_seconds=cold["seconds"], warm_seconds=warm["seconds"],
                predict_seconds=t_pred,
                converged_u_difference=du, converged_rho_a_difference=da, prediction_u_error=eu,
                prediction_rho_a_error=ea)


def solve(solid, ra, rb, phys, u=None, tol=1e-6, every=100, max_steps=100000, prec="fp32", strain=False):
    """One solve from the fields (ra, rb, u) to the residual tol.  With
    strain, the initial populations also carry the non-equilibrium part of
    u's strain (lbm_set_fields_strain), not the equilibrium alone."""
    ctx = make_context(solid, ra, rb, phys, prec, u)
    if strain and u is not None:
        lbm.lbm_set_fields_strain(ctx, ra, rb, u)
    t = time.perf_counter()
    steps, conv, hist = run_to_residual(ctx, solid.shape, tol, every, max_steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t
    f = fields(ctx, solid.shape)
    lbm.lbm_free(ctx)
    return dict(steps=steps, converged=conv, seconds=wall, fields=f, residuals=hist)


def train(net, samples, phys, epochs, lr=1e-3, log=None, lr_end=None, time_budget=None):
    """Adam on the surrogate's own kernels over solver-generated samples
    (each a dict of steady_sample), the learning rate falling linearly from
    lr to lr_end (default lr / 10) over the epochs.  Returns the per-epoch
    mean loss."""
    cw = surrogate.loss_weights()
    data = []
    for s in samples:
        x = surrogate.features(s["solid"], phi_of(s["solid"], s["ra0"], s["rb0"]))
        t = surrogate.targets(s["u"], s["ra"], s["rb"], net.u_scale, mobility(s["solid"], s["ra0"], s["rb0"], phys),
                              s["ra0"], s["rb0"])
        data.append((x, t, (1,) + tuple(s["solid"].shape)))
    hist = []
    lr_end = lr / 10 if lr_end is None else lr_end
    t0 = time.perf_counter()
    for ep in range(epochs):
        if time_budget is not None and time.perf_counter() - t0 > time_budget:
            break
        tot = 0.0
        lr_ep = lr + (lr_end - lr) * ep / max(epochs - 1, 1)
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
