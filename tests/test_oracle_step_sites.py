"""The oracle's per-site step (ora_step_sites), which the full-size GPU
parity tests use as their reference, against the oracle's whole-lattice step
(ora_step): the same equations in the same order, so every population of
every fluid site agrees bit for bit -- for both equilibrium kinds, both
forcing kinds and both wall kinds, on a random non-equilibrium state with
random solids, a wall plane and wetting walls (Eqs. 1-11)."""
import itertools

import numpy as np
import pytest

from paper_1711_03254_amd import inputs


def _case(seed):
    shape = (7, 9, 11)
    solid = inputs.random_mask(shape, 0.15, seed)
    solid[:, 0, :] = 1
    f0 = inputs.random_populations(shape, seed + 1)
    f0[:, :, solid == 1] = 0.0
    return shape, solid, f0


@pytest.mark.parametrize("eq_kind,force_kind,wall_kind", list(itertools.product((0, 1), (0, 1), (0, 1))))
@pytest.mark.parametrize("rho_s", [0.35, -0.2])
def test_step_sites_equals_step(ora, eq_kind, force_kind, wall_kind, rho_s):
    shape, solid, f0 = _case(40 + 4 * eq_kind + 2 * force_kind + wall_kind)
    nz, ny, nx = shape
    p = ora.Params(nx, ny, nz, tau=(0.58, 1.9), G=-2.7, g=(2e-5, -1e-5, 3e-5), rho_s=rho_s, eq_kind=eq_kind,
                   force_kind=force_kind, wall_kind=wall_kind, solid=solid)
    whole = ora.step(p, f0)
    sites = np.flatnonzero(solid.ravel() == 0)
    got = ora.step_sites(p, f0, sites)
    want = whole.reshape(2, 19, -1)[:, :, sites].transpose(2, 0, 1)
    assert np.array_equal(got, want)


def test_step_sites_refuses_solid_sites(ora):
    shape, solid, f0 = _case(60)
    nz, ny, nx = shape
    p = ora.Params(nx, ny, nz, G=-2.0, solid=solid)
    with pytest.raises(ValueError):
        ora.step_sites(p, f0, np.flatnonzero(solid.ravel() == 1)[:3])


def test_wall_kinds_differ_in_step_sites(ora):
    """The per-site step honours the wall kind: with wetting walls the
    momentum-balanced wall force (W2) changes the populations next to walls."""
    shape, solid, f0 = _case(70)
    nz, ny, nx = shape
    sites = np.flatnonzero(solid.ravel() == 0)
    out = []
    for wk in (0, 1):
        p = ora.Params(nx, ny, nz, tau=(0.8, 1.1), G=-2.5, rho_s=0.4, wall_kind=wk, solid=solid)
        out.append(ora.step_sites(p, f0, sites))
    assert np.abs(out[0] - out[1]).max() > 1e-6
