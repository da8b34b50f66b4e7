"""Critical pressure for pushing a wetting slug out of a constriction, Eq. (12).

Section 3.6 sets a slug of the second component over the junction of a
narrow channel (height D) and a wide one (height H > D) in a periodic
two-dimensional channel of length L, with walls that the slug wets
(contact angle theta <= 90 degrees measured inside the second component).
Its two menisci then differ in capillary pressure by
P_crit = 2 sigma cos(theta) (1/D - 1/H), which holds the slug in the narrow
part until a body force rho_0 g over the whole length supplies it:
g_crit = P_crit / (rho_0 L).  The paper raises g in stages of -30, -10,
-5, 0, +5, +10 and +30 % around g_crit and finds the slug moving on within
10 % of it.

Here the solver (include/lbm.h) runs that protocol on a quasi-2D lattice
(one site deep in z, walls at y = 0 and y = H + 1, the narrow part centred
in y), carrying the populations from stage to stage through the exchange
calls; sigma comes from the Laplace law of static 2D droplets (Section 3.1)
and theta from the contact-angle calibration (contact_angle.py), both
measured with the same solver and physics.
"""
from __future__ import annotations

import numpy as np

from . import inputs, lbm

T0 = 1.0 / 3.0
STAGES = (-0.30, -0.10, -0.05, 0.0, 0.05, 0.10, 0.30)


def pressure(ra, rb, G):
    """Bulk pressure of the two-component model: T0 rho - G T0 rho_1 rho_2
    (the continuum limit of the force of Eq. 7)."""
    return T0 * (ra + rb) - G * T0 * ra * rb


def surface_tension(G=-4.2, tau=1.0, radii=(8, 10, 12, 14), steps=20000, prec="fp64"):
    """sigma from the Laplace law Delta p = sigma / R of static 2D droplets
    of A in B (periodic lattices of 4R x 4R), least squares over the radii
    with an intercept.  Returns (sigma, intercept, r2)."""
    pts = []
    for R in radii:
        n = 4 * R
        shape = (1, n, n)
        ra, rb = inputs.cylinder(shape, R, center=(n / 2, n / 2))
        ctx = lbm.lbm_init(lbm.Params(n, n, 1, prec=lbm.PRECISIONS[prec], rho_init=(ra, rb), tau=(tau, tau), G=G))
        lbm.lbm_step(ctx, steps)
        a, b, _ = lbm.lbm_moments(ctx)
        lbm.lbm_free(ctx)
        a, b = a.reshape(shape), b.reshape(shape)
        P = pressure(a, b, G)
        dp = P[0, n // 2, n // 2] - P[0, 0, 0]
        ain, aout = a[0, n // 2, n // 2], a[0, 0, 0]
        reff = np.sqrt(((a - aout) / (ain - aout)).sum() / np.pi)
        pts.append((reff, dp))
    r = np.array([p[0] for p in pts])
    dp = np.array([p[1] for p in pts])
    A = np.vstack([1.0 / r, np.ones_like(r)]).T
    (sigma, icpt), *_ = np.linalg.lstsq(A, dp, rcond=None)
    fit = A @ [sigma, icpt]
    r2 = 1.0 - ((dp - fit) ** 2).sum() / ((dp - dp.mean()) ** 2).sum()
    return float(sigma), float(icpt), float(r2)


def p_crit(sigma, theta_deg, D, H):
    """Eq. (12)."""
    return 2.0 * sigma * np.cos(np.radians(theta_deg)) * (1.0 / D - 1.0 / H)


def constricted_channel(L=160, Z=52, H=40, D=10, x0=54):
    """Solid mask (1, H + 2, L): walls at y = 0 and y = H + 1; in
    x0 <= x < x0 + Z only the D rows centred between them are open."""
    ny = H + 2
    solid = np.zeros((1, ny, L), np.uint8)
    solid[:, 0, :] = 1
    solid[:, ny - 1, :] = 1
    lo = 1 + (H - D) // 2
    band = np.zeros(ny, bool)
    band[lo:lo + D] = True
    for y in range(1, ny - 1):
        if not band[y]:
            solid[:, y, x0:x0 + Z] = 1
    return solid


def slug_state(solid, x_from, x_to, major=1.0, minor=0.03):
    """Component 2 (the slug) in x_from <= x < x_to, component 1 elsewhere;
    zero on solid sites."""
    L = solid.shape[2]
    x = np.arange(L)[None, None, :] * np.ones(solid.shape)
    inside = (x >= x_from) & (x < x_to)
    ra = np.where(inside, minor, major)
    rb = np.where(inside, major, minor)
    ra[solid == 1] = 0.0
    rb[solid == 1] = 0.0
    return ra, rb


def slug_position(rb, solid, minor=0.03):
    """Centre of the slug along the periodic x axis (circular mean of the
    excess second-component density over the fluid sites)."""
    L = rb.shape[2]
    w = np.where(solid == 0, np.clip(rb - minor, 0.0, None), 0.0).sum(axis=(0, 1))
    ang = 2.0 * np.pi * np.arange(L) / L
    c, s = (w * np.cos(ang)).sum(), (w * np.sin(ang)).sum()
    return float((np.arctan2(s, c) % (2.0 * np.pi)) * L / (2.0 * np.pi))


def ramp(sigma, theta_deg, D=10, H=40, L=160, Z=52, rho_s=0.4, G=-4.2, tau=(1.0, 1.0), steps=80000,
         stages=STAGES, prec="fp32", slug=(78, 109), x0=54, wall_kind=0):
    """Runs the staged drive of Section 3.6 and reports, per stage, where
    the slug's centre is (unwrapped along x) and how far it moved.  The slug
    (400 sites of the second component, 40 sites long inside the narrow
    part) starts over the exit of the narrow part at x0 + Z; the drive
    points along +x, out of the narrow part.  rho_0 is the initial majority
    density plus the minority one (the total density the body force acts
    on)."""
    solid = constricted_channel(L, Z, H, D, x0)
    ra, rb = slug_state(solid, *slug)
    rho0 = 1.03
    pc = p_crit(sigma, theta_deg, D, H)
    gc = pc / (rho0 * L)
    rows = []
    f = None
    pos = start = slug_position(rb, solid)
    travelled = 0.0
    for k, dev in enumerate(stages):
        g = gc * (1.0 + dev)
        ctx = lbm.lbm_init(lbm.Params(L, H + 2, 1, prec=lbm.PRECISIONS[prec], solid=solid, rho_init=(ra, rb),
                                      tau=tau, G=G, g=(g, 0.0, 0.0), rho_s=rho_s, wall_kind=wall_kind))
        if f is not None:
            lbm.lbm_set_populations(ctx, f)
        lbm.lbm_step(ctx, steps)
        f = lbm.lbm_get_populations(ctx)
        _, b, _ = lbm.lbm_moments(ctx)
        lbm.lbm_free(ctx)
        new = slug_position(b.reshape(solid.shape), solid)
        move = (new - pos + L / 2) % L - L / 2   # shortest signed travel (a stage moves it less than L / 2)
        travelled += move
        rows.append({"stage": dev, "g": g, "slug_x": start + travelled, "moved": move})
        pos = new
    return {"sigma": sigma, "theta_deg": theta_deg, "D": D, "H": H, "L": L, "Z": Z, "rho_s": rho_s, "wall_kind": wall_kind,
            "exit_x": x0 + Z, "p_crit": pc, "g_crit": gc, "stages": rows}


def transition(result):
    """The stages (deviations from g_crit) between which the slug is pushed
    out of the narrow part: the last stage that ends with its centre inside
    (x < exit) and the first that ends with it outside; None where there is
    no such stage."""
    prev = None
    for row in result["stages"]:
        if row["slug_x"] >= result["exit_x"]:
            return prev, row["stage"]
        prev = row["stage"]
    return prev, None


def sweep(nus=((0.0017, 0.33), (0.33, 0.0017)), rho_s_values=(0.3, 0.5, 0.7), heights=(5, 10), G=-4.2,
          log=None):
    """The grid of Section 3.6 on the solver: per viscosity pair (nu_1, nu_2)
    (component 2 is the slug) and wall parameter, the contact angle inside
    the slug from the calibration at those viscosities, then the staged
    drive at each narrow height D.  sigma is measured once at tau = 1 (it
    does not depend on the viscosities).  Returns one row per case with
    the transition band (None where the run turned non-finite: the slug's
    position is then NaN)."""
    from . import contact_angle as ca
    sigma, _, _ = surface_tension(G=G, tau=1.0)
    rows = []
    for nu in nus:
        tau = (nu[0] / T0 + 0.5, nu[1] / T0 + 0.5)
        for rho_s in rho_s_values:
            theta2 = 180.0 - ca.measure(rho_s, G=G, tau=tau, steps=20000)["theta_deg"]
            for D in heights:
                r = ramp(sigma, theta2, D=D, rho_s=rho_s, G=G, tau=tau)
                finite = all(np.isfinite(s["slug_x"]) for s in r["stages"])
                row = {"nu": list(nu), "rho_s": rho_s, "theta2": theta2, "D": D, "g_crit": r["g_crit"],
                       "finite": finite, "transition": transition(r) if finite else None,
                       "slug_x": {s["stage"]: s["slug_x"] for s in r["stages"]}, "exit_x": r["exit_x"]}
                rows.append(row)
                if log:
                    log(row)
    return {"sigma": sigma, "rows": rows}


if __name__ == "__main__":
    import json
    lbm.load_library()
    res = sweep(log=lambda row: print(json.dumps(row), flush=True))
    print(json.dumps({"sigma": res["sigma"]}), flush=True)
