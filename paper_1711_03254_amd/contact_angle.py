"""Contact-angle calibration of the wall parameter rho^s.

The paper controls wettability with the single parameter rho^s (wall
densities rho^s_1 = max(-rho^s, 0), rho^s_2 = max(rho^s, 0) on solid sites,
the wall interaction of Eq. 11) and states that the map from rho^s to the
contact angle is an empirical fit it does not give.  This module measures
it: a cylindrical droplet of component A rests on a flat wall (a quasi-2D
lattice, one site deep in z, periodic along x, a solid row at y = 0 and
at the top), the solver runs it to rest, and a circle fitted to the
interface rho_A = rho_B away from the wall gives the angle inside the
droplet at the wall plane (halfway between the solid row and the first
fluid row, where bounce-back puts it).
"""
from __future__ import annotations

import numpy as np

from . import lbm


def droplet_on_wall(nx=160, ny=80, radius=24.0, inside=(1.0, 0.03), outside=(0.03, 1.0)):
    """Solid mask and densities (nz = 1) of a half disc of A on the wall."""
    shape = (1, ny, nx)
    solid = np.zeros(shape, np.uint8)
    solid[:, 0, :] = 1
    solid[:, ny - 1, :] = 1
    y, x = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    ins = ((x - nx / 2.0) ** 2 + (y - 0.5) ** 2 <= radius ** 2)[None]
    ra = np.where(ins, inside[0], outside[0])
    rb = np.where(ins, inside[1], outside[1])
    ra[solid == 1] = 0.0
    rb[solid == 1] = 0.0
    return solid, ra, rb


def interface_points(ra, rb, solid, y_min=4, y_max=None):
    """Points (x, y) where rho_A - rho_B changes sign between neighbouring
    fluid sites (linear interpolation), at heights y_min <= y < y_max
    (default: the lower half, which keeps out the thin films that the
    opposite wall may carry)."""
    phi = np.where(solid == 0, ra - rb, np.nan)[0]
    pts = []
    ny, nx = phi.shape
    y_max = ny // 2 if y_max is None else y_max
    for y in range(y_min, y_max):
        row = phi[y]
        for x in range(nx):
            a, b = row[x], row[(x + 1) % nx]
            if np.isfinite(a) and np.isfinite(b) and a * b < 0:
                pts.append((x + a / (a - b), y))
    for x in range(nx):
        col = phi[:, x]
        for y in range(y_min, y_max - 1):
            a, b = col[y], col[y + 1]
            if np.isfinite(a) and np.isfinite(b) and a * b < 0:
                pts.append((x, y + a / (a - b)))
    return np.array(pts, dtype=np.float64)


def fit_circle(pts):
    """Least-squares circle (Kasa fit): centre (xc, yc) and radius r."""
    x, y = pts[:, 0], pts[:, 1]
    A = np.stack([2 * x, 2 * y, np.ones_like(x)], axis=1)
    b = x * x + y * y
    (xc, yc, c), *_ = np.linalg.lstsq(A, b, rcond=None)
    return xc, yc, float(np.sqrt(c + xc * xc + yc * yc))


def angle_from_circle(yc, r, y_wall=0.5):
    """Angle inside the droplet between the wall and the interface where
    the circle meets the wall plane, in degrees."""
    h = (yc - y_wall) / r
    return float(np.degrees(np.pi / 2 + np.arcsin(np.clip(h, -1.0, 1.0))))


def measure(rho_s, G=-4.2, tau=(1.0, 1.0), steps=20000, prec="fp64", wall_kind=0, nx=160, ny=80, radius=24.0,
            stream=None):
    """Contact angle (degrees) of component A at wall parameter rho_s, with
    the fitted circle and the number of interface points (NaN when no cap
    is left to fit)."""
    solid, ra, rb = droplet_on_wall(nx, ny, radius)
    ctx = lbm.lbm_init(lbm.Params(nx, ny, 1, prec=lbm.PRECISIONS[prec], solid=solid, rho_init=(ra, rb), tau=tau,
                                  G=G, rho_s=rho_s, wall_kind=wall_kind, stream=stream))
    lbm.lbm_step(ctx, steps)
    r1, r2, _ = lbm.lbm_moments(ctx)
    lbm.lbm_free(ctx)
    pts = interface_points(r1, r2, solid)
    if len(pts) < 8:   # no cap left: the droplet spread into a film or left the wall
        return {"rho_s": rho_s, "theta_deg": float("nan"), "circle": None, "points": int(len(pts))}
    xc, yc, r = fit_circle(pts)
    return {"rho_s": rho_s, "theta_deg": angle_from_circle(yc, r), "circle": [float(xc), float(yc), r],
            "points": int(len(pts))}


def calibrate(values=(-0.4, -0.2, 0.0, 0.2, 0.4), **kw):
    """theta(rho^s) over the given wall parameters."""
    return [measure(v, **kw) for v in values]


def rho_s_for(theta_deg, table):
    """The inverse of the calibration (Section 3.3 inverts theta = L(nu_1,
    nu_2, rho^s) for the wall potential): rho^s for a target angle (inside
    component A), linear between the two table rows that bracket it.  The
    table (rows of calibrate at one pair of viscosities) must be increasing
    in theta over the rows used; rows without a fitted angle are skipped.
    Raises ValueError outside the table's range."""
    rows = sorted((r["rho_s"], r["theta_deg"]) for r in table if np.isfinite(r["theta_deg"]))
    for (r0, t0), (r1, t1) in zip(rows, rows[1:]):
        if t1 <= t0:
            raise ValueError("the calibration is not increasing in rho^s")
        if t0 <= theta_deg <= t1:
            return r0 + (theta_deg - t0) * (r1 - r0) / (t1 - t0)
    raise ValueError(f"theta = {theta_deg} lies outside the calibrated range")
