"""Seeded synthetic inputs: geometry, initial density fields and random states.

This module produces inputs only -- solid masks, initial component densities
and raw population arrays -- and holds none of the lattice Boltzmann
arithmetic, so that the GPU path and the CPU oracle can be fed identical data.
Every generator is deterministic in its seed.

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) used as a counter-based
generator: draw k of stream `seed` is mix(seed + (k + 1) * 0x9E3779B97F4A7C15),
mapped to a double in [0, 1) from its top 53 bits.

Array conventions: scalar fields (nz, ny, nx) with x fastest; solid masks are
uint8 (1 = solid); populations (2, 19, nz, ny, nx).
"""
from __future__ import annotations

import math

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, n: int, offset: int = 0) -> np.ndarray:
    """Draws offset .. offset+n-1 of SplitMix64 stream `seed` (uint64)."""
    with np.errstate(over="ignore"):
        k = np.arange(offset + 1, offset + n + 1, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + k * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform(seed: int, n: int, offset: int = 0) -> np.ndarray:
    """Uniform doubles in [0, 1)."""
    return (splitmix64(seed, n, offset) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


# --------------------------------------------------------------------------
# Random states and masks (parity tests).
# --------------------------------------------------------------------------

def random_populations(shape, seed: int, lo: float = 0.01, hi: float = 0.09) -> np.ndarray:
    """Independent uniform populations in [lo, hi): a state far from
    equilibrium, for one-step comparisons."""
    nz, ny, nx = shape
    n = 2 * 19 * nx * ny * nz
    return (lo + (hi - lo) * uniform(seed, n)).reshape((2, 19) + tuple(shape))


def random_mask(shape, fraction: float, seed: int) -> np.ndarray:
    """Each site solid with probability `fraction`."""
    n = int(np.prod(shape))
    return (uniform(seed, n) < fraction).astype(np.uint8).reshape(shape)


def smooth_random_density(shape, seed: int, mean: float = 1.0, amp: float = 0.05, modes: int = 3) -> np.ndarray:
    """A smooth periodic field: mean plus a few random low Fourier modes."""
    nz, ny, nx = shape
    r = uniform(seed, 7 * modes)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    out = np.full(shape, mean, dtype=np.float64)
    for m in range(modes):
        kx, ky, kz = (1 + int(3 * r[7 * m + k]) for k in range(3))
        ph = 2 * math.pi * r[7 * m + 3]
        a = amp * (r[7 * m + 4] - 0.5) * 2 / modes
        out += a * np.cos(2 * math.pi * (kx * x / nx + ky * y / ny + kz * z / nz) + ph)
    return out


# --------------------------------------------------------------------------
# Geometries of the workloads.
# --------------------------------------------------------------------------

def droplet(shape, radius: float, center=None, inside=(1.0, 0.03), outside=(0.03, 1.0)):
    """Sphere of component A (`inside` densities) in B (`outside`), sharp
    step: a site is inside when |x - center|^2 <= R^2 on node coordinates.
    Returns (rho_A, rho_B, solid=None)."""
    nz, ny, nx = shape
    if center is None:
        center = (nx / 2.0, ny / 2.0, nz / 2.0)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    d2 = (x - center[0]) ** 2 + (y - center[1]) ** 2 + (z - center[2]) ** 2
    ins = d2 <= radius * radius
    rA = np.where(ins, inside[0], outside[0]).astype(np.float64)
    rB = np.where(ins, inside[1], outside[1]).astype(np.float64)
    return rA, rB


def cylinder(shape, radius: float, center=None, inside=(1.0, 0.03), outside=(0.03, 1.0)):
    """Column along z of component A in B (a two-dimensional droplet)."""
    nz, ny, nx = shape
    if center is None:
        center = (nx / 2.0, ny / 2.0)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ins = (x - center[0]) ** 2 + (y - center[1]) ** 2 <= radius * radius
    rA = np.where(ins, inside[0], outside[0]).astype(np.float64)
    rB = np.where(ins, inside[1], outside[1]).astype(np.float64)
    return rA, rB


def channel_walls(shape) -> np.ndarray:
    """Solid planes at y = 0 and y = ny - 1; periodic in x and z."""
    m = np.zeros(shape, np.uint8)
    m[:, 0, :] = 1
    m[:, -1, :] = 1
    return m


def two_layer(shape, major: float = 1.0, minor: float = 0.03):
    """Two layers of equal thickness between the walls of `channel_walls`:
    A in y = 1 .. ny/2 - 1, B in y = ny/2 .. ny - 2."""
    nz, ny, nx = shape
    y = np.arange(ny)[None, :, None] * np.ones(shape)
    inA = y < ny // 2
    rA = np.where(inA, major, minor).astype(np.float64)
    rB = np.where(inA, minor, major).astype(np.float64)
    return rA, rB


def three_band(shape, half_core: float, major: float = 1.0, minor: float = 0.03):
    """A along both walls, B in a core of half-width `half_core` about the
    channel centre (walls at y = 0 and ny - 1)."""
    nz, ny, nx = shape
    yc = (ny - 1) / 2.0
    y = np.arange(ny)[None, :, None] * np.ones(shape)
    core = np.abs(y - yc) < half_core
    rA = np.where(core, minor, major).astype(np.float64)
    rB = np.where(core, major, minor).astype(np.float64)
    return rA, rB


def _periodic_pairs(centers: np.ndarray, box: float, cutoff: float):
    from scipy.spatial import cKDTree
    tree = cKDTree(np.mod(centers, box), boxsize=box)
    return tree.query_pairs(cutoff, output_type="ndarray")


def sphere_pack(n: int, radius: float, solid_fraction: float, seed: int,
                max_iter: int = 20000, tol: float = 1e-3) -> np.ndarray:
    """Centres of non-overlapping spheres of one radius in a periodic cube of
    edge n, at the requested solid volume fraction.

    Random sequential addition stalls near 0.38, so the spheres are placed at
    random and then relaxed: each overlapping pair is pushed apart along its
    centre line by half the overlap, repeatedly, until no pair overlaps by
    more than tol * radius (soft-sphere overlap removal in the manner of the
    force-biased packing algorithms; it converges below the jamming fraction
    of about 0.64).  Returns the centres, shape (count, 3), ordered (x, y, z).
    """
    vol = 4.0 / 3.0 * math.pi * radius ** 3
    count = int(round(solid_fraction * n ** 3 / vol))
    c = uniform(seed, 3 * count).reshape(count, 3) * n
    d0 = 2.0 * radius
    for _ in range(max_iter):
        pairs = _periodic_pairs(c, n, d0)
        if len(pairs) == 0:
            break
        i, j = pairs[:, 0], pairs[:, 1]
        dv = c[j] - c[i]
        dv -= n * np.round(dv / n)
        d = np.sqrt((dv ** 2).sum(1))
        over = d0 - d
        if over.max() <= tol * radius:
            break
        d = np.maximum(d, 1e-9)
        push = (0.5 * (over + 1e-3 * radius) / d)[:, None] * dv
        disp = np.zeros_like(c)
        np.add.at(disp, i, -push)
        np.add.at(disp, j, push)
        c = np.mod(c + disp, n)
    return c


def voxelize_spheres(shape, centers: np.ndarray, radius) -> np.ndarray:
    """Solid mask: a node is solid when it lies within `radius` of a centre
    (periodic images included).  `radius` is a scalar or one value per
    sphere."""
    nz, ny, nx = shape
    m = np.zeros(shape, np.uint8)
    radii = np.broadcast_to(np.asarray(radius, dtype=np.float64), (len(centers),))
    for (cx, cy, cz), r in zip(centers, radii):
        rr = int(math.ceil(r))
        xs = np.arange(int(math.floor(cx)) - rr, int(math.floor(cx)) + rr + 2)
        ys = np.arange(int(math.floor(cy)) - rr, int(math.floor(cy)) + rr + 2)
        zs = np.arange(int(math.floor(cz)) - rr, int(math.floor(cz)) + rr + 2)
        dz = (zs - cz)[:, None, None]
        dy = (ys - cy)[None, :, None]
        dx = (xs - cx)[None, None, :]
        ins = dx * dx + dy * dy + dz * dz <= r * r
        zi, yi, xi = np.nonzero(ins)
        m[zs[zi] % nz, ys[yi] % ny, xs[xi] % nx] = 1
    return m


def pore_droplets(shape, sphere_centers: np.ndarray, sphere_radius: float, drop_radius: float,
                  pore_fraction: float, seed: int, margin: float = 1.0, max_tries: int = 2_000_000):
    """Centres of droplets of one radius lying wholly in the pore space,
    filling `pore_fraction` of the pore volume, not touching each other.
    Rejection sampling with SplitMix64 draws."""
    from scipy.spatial import cKDTree
    nz, ny, nx = shape
    assert nx == ny == nz, "pore_droplets expects a cube"
    n = nx
    solid = voxelize_spheres(shape, sphere_centers, sphere_radius)
    pore = int((solid == 0).sum())
    zz, yy, xx = np.meshgrid(*(np.arange(-int(drop_radius) - 1, int(drop_radius) + 2),) * 3, indexing="ij")
    drop_vol = int((xx ** 2 + yy ** 2 + zz ** 2 <= drop_radius ** 2).sum())
    want = max(1, int(round(pore_fraction * pore / drop_vol)))
    tree = cKDTree(np.mod(sphere_centers, n), boxsize=n)
    placed = []
    k = 0
    batch = 4096
    while len(placed) < want and k < max_tries:
        r = uniform(seed, 3 * batch, offset=3 * k).reshape(batch, 3) * n
        k += batch
        dmin, _ = tree.query(r)
        ok = dmin >= sphere_radius + drop_radius + margin
        for cand in r[ok]:
            if placed:
                dv = np.asarray(placed) - cand
                dv -= n * np.round(dv / n)
                if (np.sqrt((dv ** 2).sum(1)) < 2 * drop_radius + 2 * margin).any():
                    continue
            placed.append(cand)
            if len(placed) >= want:
                break
    return np.asarray(placed).reshape(-1, 3), solid


def packed_spheres_case(n: int = 256, radius: float = 12.0, porosity: float = 0.40,
                        drop_radius: float = 4.0, drop_fraction: float = 0.01, seed: int = 3,
                        minority: float = 0.03, interface_width: float = 0.0):
    """The 1 % mixture in packed spheres: a periodic cube of edge n filled with
    non-overlapping spheres of `radius` at the given porosity (solid mask),
    droplets of component A (radius `drop_radius`, `drop_fraction` of the
    pore volume) in a carrier of component B.  With interface_width w > 0 the
    droplet profile is 1/2 (1 - tanh((d - R) / w)) in the distance d from the
    nearest droplet centre instead of a sharp step.  Returns (solid, rho_A,
    rho_B, info)."""
    shape = (n, n, n)
    centers = sphere_pack(n, radius, 1.0 - porosity, seed)
    drops, solid = pore_droplets(shape, centers, radius, drop_radius, drop_fraction, seed + 1)
    inA = voxelize_spheres(shape, drops, drop_radius).astype(bool) if len(drops) else np.zeros(shape, bool)
    if interface_width > 0 and len(drops):
        from scipy.spatial import cKDTree
        z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
        pts = np.stack([x.ravel(), y.ravel(), z.ravel()], 1).astype(np.float64)
        d, _ = cKDTree(np.mod(drops, n), boxsize=n).query(pts)
        phi = (0.5 * (1.0 - np.tanh((d - drop_radius) / interface_width))).reshape(shape)
        rA = minority + (1.0 - minority) * phi
        rB = minority + (1.0 - minority) * (1.0 - phi)
    else:
        rA = np.where(inA, 1.0, minority)
        rB = np.where(inA, minority, 1.0)
    rA[solid == 1] = 0.0
    rB[solid == 1] = 0.0
    info = {"spheres": int(len(centers)), "droplets": int(len(drops)),
            "porosity": float((solid == 0).mean()),
            "drop_fraction_of_pore": float(inA.sum() / max(1, (solid == 0).sum()))}
    return solid, rA, rB, info


def ensemble_case(count: int = 64, seed: int = 11, nu_min: float = 0.0017, g: float = 1e-6):
    """The batched ensemble: `count` square ducts (solid faces at the x and y
    edges, periodic along z) with a slug front -- A in z < nz/2, B above.
    Seeded draws: nx = ny uniform in {48, 64, ..., 128}, nz uniform in
    {96, 112, ..., 256}; viscosity ratio log-uniform in [1, 1000] with the
    lower viscosity nu_min (A is the less viscous component); the workloads'
    G uniform in [1.2, 1.6], returned in the paper's sign and weights as
    G = -3 G_w; contact angle uniform in [30, 150] degrees, mapped to the wall
    parameter linearly, rho^s = 0.4 cos(theta) / cos(30 deg) (an uncalibrated
    stand-in: 90 degrees is the neutral wall).  Returns a list of dicts with
    shape (nz, ny, nx), solid, rho_A, rho_B and the physical parameters."""
    r = uniform(seed, 6 * count).reshape(count, 6)
    T0 = 1.0 / 3.0
    out = []
    for k in range(count):
        n = 48 + 16 * int(r[k, 0] * 6)
        nz = 96 + 16 * int(r[k, 1] * 11)
        ratio = 10.0 ** (3.0 * r[k, 2])
        Gw = 1.2 + 0.4 * r[k, 3]
        theta = math.radians(30.0 + 120.0 * r[k, 4])
        rho_s = 0.4 * math.cos(theta) / math.cos(math.radians(30.0))
        shape = (nz, n, n)
        solid = np.zeros(shape, np.uint8)
        solid[:, 0, :] = solid[:, -1, :] = 1
        solid[:, :, 0] = solid[:, :, -1] = 1
        z = np.arange(nz)[:, None, None] * np.ones(shape)
        rA = np.where(z < nz // 2, 1.0, 0.03)
        rB = np.where(z < nz // 2, 0.03, 1.0)
        rA[solid == 1] = 0.0
        rB[solid == 1] = 0.0
        out.append({"shape": shape, "solid": solid, "rho_A": rA, "rho_B": rB,
                    "tau": (nu_min / T0 + 0.5, nu_min * ratio / T0 + 0.5), "G": -3.0 * Gw,
                    "g": (0.0, 0.0, g), "rho_s": rho_s, "ratio": ratio, "theta_deg": math.degrees(theta)})
    return out


def boolean_spheres(n: int, radius: float, porosity: float, seed: int) -> np.ndarray:
    """Centres of independently placed spheres (overlaps allowed: the Boolean
    model of a porous medium) in a periodic cube of edge n.  Their count is
    the one whose expected pore fraction exp(-count v / n^3) equals the
    requested porosity (v the sphere volume)."""
    vol = 4.0 / 3.0 * math.pi * radius ** 3
    count = max(1, int(round(-math.log(porosity) * n ** 3 / vol)))
    return uniform(seed, 3 * count).reshape(count, 3) * n


def subvolume_case(n: int, seed: int, radius_range=(6.0, 16.0), porosity_range=(0.3, 0.5),
                   drop_radius: float = 4.0, fraction_range=(0.01, 0.05), minority: float = 0.03,
                   interface_width: float = 1.5):
    """A packed-sphere subvolume for the warm-start surrogate: sphere radius
    and porosity drawn uniformly from the given ranges (Boolean model, so the
    low porosities are reachable), droplets of component A of `drop_radius`
    filling a drawn fraction of the pore space, tanh interfaces of the given
    width.  Returns (solid, rho_A, rho_B, info)."""
    r = uniform(seed, 3, offset=1 << 40)
    radius = radius_range[0] + (radius_range[1] - radius_range[0]) * r[0]
    porosity = porosity_range[0] + (porosity_range[1] - porosity_range[0]) * r[1]
    frac = fraction_range[0] + (fraction_range[1] - fraction_range[0]) * r[2]
    shape = (n, n, n)
    centers = boolean_spheres(n, radius, porosity, seed)
    drops, solid = pore_droplets(shape, centers, radius, drop_radius, frac, seed + 1, margin=0.5)
    phi = np.zeros(shape)
    if len(drops):
        from scipy.spatial import cKDTree
        z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
        pts = np.stack([x.ravel(), y.ravel(), z.ravel()], 1).astype(np.float64)
        d, _ = cKDTree(np.mod(drops, n), boxsize=n).query(pts)
        phi = (0.5 * (1.0 - np.tanh((d - drop_radius) / interface_width))).reshape(shape)
    rA = minority + (1.0 - minority) * phi
    rB = minority + (1.0 - minority) * (1.0 - phi)
    rA[solid == 1] = 0.0
    rB[solid == 1] = 0.0
    info = {"radius": float(radius), "porosity": float((solid == 0).mean()), "target_porosity": float(porosity),
            "droplets": int(len(drops)), "drop_fraction": float(frac)}
    return solid, rA, rB, info


def mixture_case(n: int, seed: int, radius_range=(6.0, 16.0), porosity_range=(0.3, 0.5),
                 fraction_range=(0.1, 0.9), total: float = 1.0):
    """A packed-sphere subvolume (Boolean model, radius and porosity drawn
    uniformly from the ranges) filled with a uniform mixture: component A
    holds a drawn fraction c of the total density, B the rest.  Below the
    demixing coupling the mixture stays miscible and the flow it carries has
    a steady state.  Returns (solid, rho_A, rho_B, info)."""
    r = uniform(seed, 3, offset=1 << 41)
    radius = radius_range[0] + (radius_range[1] - radius_range[0]) * r[0]
    porosity = porosity_range[0] + (porosity_range[1] - porosity_range[0]) * r[1]
    c = fraction_range[0] + (fraction_range[1] - fraction_range[0]) * r[2]
    shape = (n, n, n)
    solid = voxelize_spheres(shape, boolean_spheres(n, radius, porosity, seed), radius)
    rA = np.where(solid == 1, 0.0, c * total)
    rB = np.where(solid == 1, 0.0, (1.0 - c) * total)
    info = {"radius": float(radius), "porosity": float((solid == 0).mean()), "target_porosity": float(porosity),
            "fraction": float(c)}
    return solid, rA, rB, info
