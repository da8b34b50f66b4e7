"""GPU <-> oracle parity through the C ABI (needs an MI355X: -m gpu).

Tolerances: populations and densities in the normalized max-norm
max|X_gpu - X_oracle| / max|X_oracle|; the velocity u_F as an absolute error
in lattice units (its scale is the lattice speed; normalizing by max |u_F|
would divide by a spurious current of 1e-3 in a static droplet).
FP64 storage and arithmetic 1e-12 at every horizon; FP32 1e-5.  The FP64
kernel and the oracle evaluate the same equations in a different order (and
with fused multiply-adds on the GPU), so they agree to rounding, about 1e-15
per step.  FP32 rounds every stored population to single precision and
computes in FP32: it meets 1e-5 on the macroscopic fields up to a measured
horizon (FP32_HORIZON steps of the droplet, 40 steps with walls); where it
does not (the 500-step droplet, the 20000-step channel at tau = 0.5051) the
tests say so and guard the measured figure against regressions instead.
Measured deviations are appended to $PARITY_LOG (JSON lines) when it is set.
"""
import json
import os

import numpy as np
import pytest

from paper_1711_03254_amd import inputs

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5}


def record(name, **vals):
    path = os.environ.get("PARITY_LOG")
    if path:
        with open(path, "a") as fh:
            fh.write(json.dumps({"test": name, **vals}) + "\n")


@pytest.fixture(scope="module")
def lbm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU (run them with -m gpu on an MI355X)"
    import paper_1711_03254_amd.lbm as m
    m.load_library()
    return m


def nmax(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def ragged_case(seed=7, shape=(29, 37, 70), frac=0.08):
    solid = inputs.random_mask(shape, frac, seed)
    solid[:, 0, :] = 1                       # a wall plane as well
    f0 = inputs.random_populations(shape, seed + 1)
    f0[:, :, solid == 1] = 0.0
    return solid, f0


def gpu_ctx(lbm, shape, prec, solid, **kw):
    nz, ny, nx = shape
    r = np.ones(shape)
    r[solid == 1] = 0.0 if solid is not None else 1.0
    return lbm.lbm_init(lbm.Params(nx, ny, nz, prec=lbm.PRECISIONS[prec], solid=solid, rho_init=(r, r.copy()), **kw))


PHYS = dict(tau=(0.62, 1.7), G=-3.0, g=(1e-5, -2e-5, 3e-5), rho_s=0.3)


# Every tile the library compiles; FP64 is refused the tiles of more than
# 256 threads.
TILE_CASES = [(p, t) for p in ("fp64", "fp32")
              for t in ((64, 4), (32, 8), (16, 16), (8, 32), (64, 8), (32, 16), (64, 16))
              if not (p == "fp64" and t[0] * t[1] > 256)]


@pytest.mark.parametrize("prec,tile", TILE_CASES)
@pytest.mark.parametrize("eq_kind,force_kind", [(0, 0), (1, 0), (0, 1)])
def test_one_step_from_random_state(lbm, ora, prec, tile, eq_kind, force_kind):
    """One step from seeded random populations on a 70 x 37 x 29 lattice
    (ragged against every tile shape) with random solids and a wall plane:
    all 38 populations of every site."""
    solid, f0 = ragged_case()
    shape = f0.shape[2:]
    nz, ny, nx = shape
    kw = dict(PHYS, eq_kind=eq_kind, force_kind=force_kind)
    ctx = gpu_ctx(lbm, shape, prec, solid, tile=tile, zchunk=5, **kw)
    lbm.lbm_set_populations(ctx, f0)
    if prec == "fp64":
        assert np.array_equal(lbm.lbm_get_populations(ctx), f0)
    lbm.lbm_step(ctx, 1)
    got = lbm.lbm_get_populations(ctx)
    p = ora.Params(nx, ny, nz, solid=solid, **kw)
    want = ora.step(p, f0)
    dev = nmax(got, want)
    record("one_step_random", prec=prec, tile=list(tile), eq_kind=eq_kind, force_kind=force_kind, dev=dev)
    assert dev <= TOL[prec]
    assert np.all(got[:, :, solid == 1] == 0)


@pytest.mark.parametrize("prec,tile", [("fp64", (64, 4)), ("fp64", (8, 32)), ("fp32", (64, 4)), ("fp32", (8, 32)),
                                       ("fp32", (64, 8)), ("fp32", (64, 16))])
@pytest.mark.parametrize("rho_s", [0.3, -0.25])
def test_momentum_balanced_walls(lbm, ora, prec, tile, rho_s):
    """The momentum-balanced wall force (wall_kind 1) against the oracle:
    one step from a random state with walls, and 40 steps of a smooth
    two-component state (the force terms then matter beyond rounding)."""
    solid, f0 = ragged_case(seed=17)
    shape = f0.shape[2:]
    nz, ny, nx = shape
    kw = dict(PHYS, rho_s=rho_s, wall_kind=1)
    ctx = gpu_ctx(lbm, shape, prec, solid, tile=tile, zchunk=7, **kw)
    lbm.lbm_set_populations(ctx, f0)
    lbm.lbm_step(ctx, 1)
    p = ora.Params(nx, ny, nz, solid=solid, **kw)
    dev1 = nmax(lbm.lbm_get_populations(ctx), ora.step(p, f0))
    r1 = inputs.smooth_random_density(shape, 18, mean=0.6, amp=0.25)
    r2 = 1.0 - r1
    r1[solid == 1] = 0
    r2[solid == 1] = 0
    g0 = ora.init(p, r1, r2)
    c2 = lbm.lbm_init(lbm.Params(nx, ny, nz, prec=lbm.PRECISIONS[prec], solid=solid, rho_init=(r1, r2), tile=tile,
                                 **kw))
    lbm.lbm_step(c2, 40)
    m = lbm.lbm_moments(c2)
    want = ora.moments(p, ora.run(p, g0, 40))
    devs = [nmax(m[0], want[0]), nmax(m[1], want[1]), nmax(m[2], want[2])]
    record("walls_w2", prec=prec, tile=list(tile), rho_s=rho_s, one_step=dev1, moments40=devs)
    assert dev1 <= TOL[prec]
    assert max(devs) <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_moments_and_reduce_match(lbm, ora, prec):
    solid, f0 = ragged_case(seed=11)
    shape = f0.shape[2:]
    nz, ny, nx = shape
    ctx = gpu_ctx(lbm, shape, prec, solid, **PHYS)
    lbm.lbm_set_populations(ctx, f0)
    p = ora.Params(nx, ny, nz, solid=solid, **PHYS)
    g1, g2, gu = lbm.lbm_moments(ctx)
    o1, o2, ou = ora.moments(p, f0)
    assert nmax(g1, o1) <= TOL[prec] and nmax(g2, o2) <= TOL[prec] and nmax(gu, ou) <= TOL[prec]
    gr = lbm.lbm_reduce(ctx)
    orr = ora.reduce(p, f0)
    np.testing.assert_allclose(gr[:2], orr[:2], rtol=TOL[prec])
    np.testing.assert_allclose(gr[2:], orr[2:], rtol=0, atol=TOL[prec] * (orr[0] + orr[1]))


@pytest.mark.parametrize("eq_kind", [0, 1])
def test_init_equals_oracle_equilibrium(lbm, ora, eq_kind):
    shape = (12, 10, 17)
    nz, ny, nx = shape
    solid = inputs.random_mask(shape, 0.1, 3)
    r1 = inputs.smooth_random_density(shape, 4, mean=0.6, amp=0.3)
    r2 = 1.1 - r1
    u = 0.05 * (inputs.uniform(5, 3 * r1.size).reshape((3,) + shape) - 0.5)
    r1[solid == 1] = 0
    r2[solid == 1] = 0
    ctx = lbm.lbm_init(lbm.Params(nx, ny, nz, prec=lbm.LBM_FP64, solid=solid, rho_init=(r1, r2), u_init=u,
                                  eq_kind=eq_kind))
    p = ora.Params(nx, ny, nz, solid=solid, eq_kind=eq_kind)
    assert nmax(lbm.lbm_get_populations(ctx), ora.init(p, r1, r2, u)) <= 1e-14


# Longest horizon (steps) of the 32^3 droplet at which FP32 meets the 1e-5
# bar on rho_1, rho_2 (normalized) and u_F (absolute); measured, see below.
FP32_HORIZON = 200


@pytest.fixture(scope="module")
def droplet_horizons(ora, droplet_reference):
    rA, rB, p, ref, _ = droplet_reference
    f = ora.init(p, rA, rB)
    out, done = {}, 0
    for t in (10, 50, 100, 200, 500):
        f = ora.run(p, f, t - done)
        done = t
        out[t] = ora.moments(p, f)
    return out


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_droplet_500_steps(lbm, droplet_reference, droplet_horizons, prec):
    """The 32^3 droplet (C1) against the oracle at 10, 50, 100, 200 and 500
    steps.  FP64: 1e-12 at every horizon.  FP32: the 1e-5 bar at every
    horizon up to FP32_HORIZON steps, where it holds (measured 5.5e-6 at 200
    steps); beyond it the densities drift past 1e-5 (1.4e-5 at 500 steps:
    the rounding of the stored populations accumulates in the slowly
    relaxing interface), so the 500-step figure is asserted against about
    twice its measured value as a regression guard, not as the bar."""
    rA, rB, p, ref, (red0, red500) = droplet_reference
    ctx = lbm.lbm_init(lbm.Params(32, 32, 32, prec=lbm.PRECISIONS[prec], tau=p.tau, G=p.G, rho_init=(rA, rB),
                                  check_every=50))
    devs, done = {}, 0
    for t in (10, 50, 100, 200, 500):
        lbm.lbm_step(ctx, t - done)
        done = t
        got = lbm.lbm_moments(ctx)
        want = droplet_horizons[t]
        devs[t] = [nmax(got[0], want[0]), nmax(got[1], want[1]), float(np.abs(got[2] - want[2]).max())]
    record("droplet_32", prec=prec, dev={str(k): v for k, v in devs.items()})
    for t, d in devs.items():
        if prec == "fp64":
            assert max(d) <= TOL["fp64"], (t, d)
        elif t <= FP32_HORIZON:
            assert max(d) <= TOL["fp32"], (t, d)
    if prec == "fp32":
        assert max(devs[500]) <= 3e-5, devs[500]
    red = lbm.lbm_reduce(ctx)
    # mass conservation: FP64 to rounding, FP32 to its storage precision
    drift = np.abs(red[:2] - red0[:2]) / red0[:2]
    assert drift.max() <= (1e-12 if prec == "fp64" else 1e-5)


def test_checkpoint_resume_is_bitwise(lbm):
    solid, f0 = ragged_case(seed=21)
    shape = f0.shape[2:]
    for prec in ("fp64", "fp32"):
        a = gpu_ctx(lbm, shape, prec, solid, **PHYS)
        lbm.lbm_set_populations(a, f0)
        lbm.lbm_step(a, 7)
        mid = lbm.lbm_get_populations(a)
        lbm.lbm_step(a, 6)
        end_a = lbm.lbm_get_populations(a)
        b = gpu_ctx(lbm, shape, prec, solid, **PHYS)
        lbm.lbm_set_populations(b, mid)
        lbm.lbm_step(b, 6)
        assert np.array_equal(lbm.lbm_get_populations(b), end_a)


def test_runs_are_deterministic_and_tiles_agree(lbm):
    solid, f0 = ragged_case(seed=31)
    shape = f0.shape[2:]
    outs = []
    for tile in [(64, 4), (64, 4), (32, 8), (8, 32), (64, 8), (64, 8), (32, 16), (64, 16), (64, 16)]:
        c = gpu_ctx(lbm, shape, "fp32", solid, tile=tile, **PHYS)
        lbm.lbm_set_populations(c, f0)
        lbm.lbm_step(c, 9)
        outs.append(lbm.lbm_get_populations(c))
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


def test_translation_commutes_bitwise(lbm):
    solid, f0 = ragged_case(seed=41, shape=(20, 24, 33))
    shape = f0.shape[2:]
    sh = (3, -5, 11)
    a = gpu_ctx(lbm, shape, "fp64", solid, **PHYS)
    lbm.lbm_set_populations(a, f0)
    lbm.lbm_step(a, 4)
    b = gpu_ctx(lbm, shape, "fp64", np.roll(solid, sh, axis=(0, 1, 2)).copy(), **PHYS)
    lbm.lbm_set_populations(b, np.roll(f0, sh, axis=(2, 3, 4)).copy())
    lbm.lbm_step(b, 4)
    assert np.array_equal(np.roll(lbm.lbm_get_populations(a), sh, axis=(2, 3, 4)), lbm.lbm_get_populations(b))


@pytest.mark.parametrize("shape", [(1, 1, 1), (3, 3, 3), (1, 40, 1), (48, 48, 1), (5, 1, 70), (2, 130, 9)])
def test_degenerate_and_thin_lattices(lbm, ora, shape):
    """Lattices of extent 1 or 2 in some direction (every neighbour wraps onto
    the site itself or its twin), nx = 1 with the 8 x 32 tile, wide rows."""
    nz, ny, nx = shape
    f0 = inputs.random_populations(shape, 51)
    solid = None
    if ny >= 9:
        solid = np.zeros(shape, np.uint8)
        solid[:, 0, :] = 1
        f0[:, :, solid == 1] = 0.0
    ctx = gpu_ctx(lbm, shape, "fp64", solid if solid is not None else np.zeros(shape, np.uint8), **PHYS)
    lbm.lbm_set_populations(ctx, f0)
    lbm.lbm_step(ctx, 3)
    p = ora.Params(nx, ny, nz, solid=solid, **PHYS)
    assert nmax(lbm.lbm_get_populations(ctx), ora.run(p, f0, 3)) <= 1e-12


def test_zero_steps_is_a_no_op(lbm):
    solid, f0 = ragged_case(seed=61, shape=(6, 9, 10))
    c = gpu_ctx(lbm, f0.shape[2:], "fp64", solid, **PHYS)
    lbm.lbm_set_populations(c, f0)
    lbm.lbm_step(c, 0)
    assert np.array_equal(lbm.lbm_get_populations(c), f0)
    assert lbm.lbm_info(c)["steps_done"] == 0


def test_error_paths(lbm):
    shape = (8, 8, 8)
    r = np.ones(shape)
    with pytest.raises(lbm.LBMError) as e:
        lbm.lbm_init(lbm.Params(8, 8, 8, rho_init=(r, r), solid=np.ones(shape, np.uint8)))
    assert e.value.code == lbm.LBM_EINVAL and "no fluid" in str(e.value)
    bad = r.copy()
    bad[1, 2, 3] = -0.1
    with pytest.raises(lbm.LBMError) as e:
        lbm.lbm_init(lbm.Params(8, 8, 8, rho_init=(bad, r)))
    assert e.value.code == lbm.LBM_EINVAL
    # a NaN planted in the state is caught by the periodic check
    c = lbm.lbm_init(lbm.Params(8, 8, 8, rho_init=(r, r), check_every=4))
    f = lbm.lbm_get_populations(c)
    f[0, 3, 4, 4, 4] = np.nan
    lbm.lbm_set_populations(c, f)
    with pytest.raises(lbm.LBMError) as e:
        lbm.lbm_step(c, 10)
    assert e.value.code == lbm.LBM_ENONFINITE
    assert lbm.lbm_info(c)["steps_done"] == 4
    # an impossible mass tolerance trips the drift check
    rA, rB = inputs.droplet(shape, 2.5)
    c = lbm.lbm_init(lbm.Params(8, 8, 8, rho_init=(rA, rB), G=-3.0, check_every=3, mass_tol=1e-300))
    with pytest.raises(lbm.LBMError) as e:
        lbm.lbm_step(c, 30)
    assert e.value.code == lbm.LBM_EMASSDRIFT


@pytest.mark.parametrize("on_device", [False, True])
def test_restart_field_checks(lbm, on_device):
    """A restart (lbm_set_fields after lbm_init) checks its fields on the
    device with the verdicts of the first load: the lowest fluid site with
    invalid densities is named with its values (solid sites are not looked
    at), a non-finite velocity is refused, a refused restart leaves the state
    as it was, and a valid one goes through; host and device inputs."""
    import torch
    shape = (8, 9, 10)
    nz, ny, nx = shape
    solid = np.zeros(shape, np.uint8)
    solid[:, 0, :] = 1
    r = np.where(solid == 1, 0.0, 1.0)
    c = lbm.lbm_init(lbm.Params(nx, ny, nz, rho_init=(r, r.copy()), solid=solid, G=-1.0))
    lbm.lbm_step(c, 3)
    before = lbm.lbm_get_populations(c)
    arg = (lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()) if on_device else (lambda x: x)
    bad = r.copy()
    bad.ravel()[700] = np.nan
    bad.ravel()[500] = -0.5           # fluid (y = 5): the lowest invalid site
    bad[solid == 1] = -7.0            # solid sites are not checked
    with pytest.raises(lbm.LBMError) as e:
        lbm.lbm_set_fields(c, arg(bad), arg(r.copy()))
    assert e.value.code == lbm.LBM_EINVAL
    assert "fluid site 500:" in str(e.value) and "rho1=-0.5" in str(e.value)
    u = np.zeros((3,) + shape)
    u[1].ravel()[300] = np.inf
    with pytest.raises(lbm.LBMError) as e:
        lbm.lbm_set_fields(c, arg(r.copy()), arg(r.copy()), arg(u))
    assert e.value.code == lbm.LBM_EINVAL and "non-finite initial velocity" in str(e.value)
    assert np.array_equal(lbm.lbm_get_populations(c), before)
    lbm.lbm_set_fields(c, arg(r.copy()), arg(r.copy()))
    assert lbm.lbm_info(c)["n_fluid"] == int((solid == 0).sum())
    lbm.lbm_free(c)


def test_index_tiles_at_the_z_limit(lbm, ora):
    """A tile column's index tiles are read with 32-bit byte offsets, so
    nz (tx + 4)(ty + 4) 4 must stay below 4 GiB: with 64 x 16 tiles on a
    1 x 1 x nz lattice at FP32 (whose population halves allow about 1.5 M
    such planes), nz = 790 000 is refused (LBM_EINVAL) and nz = 789 000
    (index-tile offsets up to 4.292e9) steps like any lattice: one step from
    a seeded random state, 1500 sites of the last planes and 500 anywhere
    recomputed by the oracle to 1e-5."""
    per_plane = 4 * (64 + 4) * (16 + 4)
    bad, good = 790_000, 789_000
    assert bad * per_plane >= 2 ** 32 > good * per_plane
    r = np.ones(bad)
    with pytest.raises(lbm.LBMError) as e:
        lbm.lbm_init(lbm.Params(1, 1, bad, prec=lbm.LBM_FP32, rho_init=(r, r.copy()), tile=(64, 16)))
    assert e.value.code == lbm.LBM_EINVAL and "index tiles" in str(e.value)
    shape = (good, 1, 1)
    rA = (0.7 + 0.1 * inputs.uniform(311, good)).reshape(shape)
    rB = (0.3 + 0.1 * inputs.uniform(312, good)).reshape(shape)
    phys = dict(tau=(0.8, 1.2), G=-1.0, g=(0.0, 0.0, 1e-5))
    ctx = lbm.lbm_init(lbm.Params(1, 1, good, prec=lbm.LBM_FP32, rho_init=(rA, rB), tile=(64, 16), check_every=0,
                                  **phys))
    p = ora.Params(1, 1, good, **phys)
    f0 = ora.init(p, rA, rB)
    lbm.lbm_step(ctx, 1)
    got_all = lbm.lbm_get_populations(ctx)
    pick = np.concatenate([good - 1 - (inputs.uniform(313, 1500) * 4000).astype(np.int64),
                           (inputs.uniform(314, 500) * good).astype(np.int64)])
    got = got_all.reshape(2, 19, -1)[:, :, pick].transpose(2, 0, 1)
    want = ora.step_sites(p, f0, pick)
    dev = nmax(got, want)
    record("index_tiles_z_limit", nz=good, dev=dev, sites=int(len(pick)))
    lbm.lbm_free(ctx)
    assert dev <= TOL["fp32"]


def test_device_pointers_and_stream(lbm, ora):
    """Inputs and outputs as torch tensors on the GPU, on a torch stream."""
    import torch
    shape = (16, 12, 20)
    nz, ny, nx = shape
    rA, rB = inputs.droplet(shape, 4.0)
    s = torch.cuda.Stream()
    dA = torch.from_numpy(rA).cuda()
    dB = torch.from_numpy(rB).cuda()
    torch.cuda.synchronize()
    ctx = lbm.lbm_init(lbm.Params(nx, ny, nz, prec=lbm.LBM_FP64, G=-3.0, rho_init=(dA, dB), stream=s))
    lbm.lbm_step(ctx, 5)
    o1 = torch.empty(shape, dtype=torch.float64, device="cuda")
    o2 = torch.empty(shape, dtype=torch.float64, device="cuda")
    ou = torch.empty((3,) + shape, dtype=torch.float64, device="cuda")
    lbm.lbm_moments(ctx, o1, o2, ou)
    p = ora.Params(nx, ny, nz, G=-3.0)
    w1, w2, wu = ora.moments(p, ora.run(p, ora.init(p, rA, rB), 5))
    assert nmax(o1.cpu().numpy(), w1) <= 1e-12 and nmax(ou.cpu().numpy(), wu) <= 1e-12
    fd = torch.empty((2, 19) + shape, dtype=torch.float64, device="cuda")
    lbm.lbm_get_populations(ctx, fd)
    assert np.array_equal(fd.cpu().numpy(), lbm.lbm_get_populations(ctx))


# Arms of the 20000-step channel: storage precision and tau_crit (sites whose
# mixture relaxation time is below it form the collision's second moments in
# FP64; 0.55 covers the low-viscosity layer, tau = 0.5051).
CHANNEL_ARMS = {"fp64": ("fp64", 0.0), "fp32": ("fp32", 0.0), "fp32_fp64flux": ("fp32", 0.55),
                "fp16s": ("fp16s", 0.0), "fp16s_fp64flux": ("fp16s", 0.55)}
_channel_oracle = {}


@pytest.mark.parametrize("arm", list(CHANNEL_ARMS))
@pytest.mark.parametrize("nuA,nuB", [(0.0017, 1.7), (1.7, 0.0017), (0.0017, 0.17), (0.0017, 0.017)])
def test_two_layer_channel_20000_steps(lbm, ora, arm, nuA, nuB):
    """The two-layer channel workload: 8 x 64 x 256, walls at y = 0 and 63,
    A in y = 1..31 and B in y = 32..62 with minority densities near their
    coexistence value, g = 1e-6 along z, G = -4.2, viscosity ratios 1000,
    1/1000, 100 and 10 with the lower viscosity 0.0017 (tau = 0.5051),
    20000 steps.  The state stays uniform in x and z, so the oracle runs the
    exactly equivalent 1 x 64 x 1 column.

    FP64 matches to 1e-12.  FP32 does not meet the 1e-5 bar at this horizon
    (densities 3.7e-4 to 5.8e-4 off, normalized; u_F 4e-6 to 1e-5 in lattice
    units): at tau = 0.5051 the collision maps the non-equilibrium part to
    1 - 1/tau = -0.98 times itself, so the rounding of the stored populations
    is hardly damped, and the flow develops over a viscous time far beyond
    20000 steps.  Forming the collision's second moments in FP64
    (tau_crit = 0.55, the low-viscosity layer) changes these figures by a few
    per cent either way: the storage rounding, not the arithmetic, sets them.
    FP16S fails here outright (densities 11-20 % off, u_F wrong by its own
    size, component masses drifting by up to 11 %, so its periodic check
    runs with a tolerance of 1): each component's density is 1 in its layer
    and 0.005 in the other, so its deviation from the one shift reference is
    half its density everywhere and FP16 keeps 11 bits of that.  The figures are asserted
    against about twice their measured values, as regression guards, and
    recorded (PARITY_LOG)."""
    prec, tau_crit = CHANNEL_ARMS[arm]
    T0 = 1.0 / 3.0
    nz, ny, nx = 256, 64, 8
    kw = dict(tau=(nuA / T0 + 0.5, nuB / T0 + 0.5), G=-4.2, g=(0.0, 0.0, 1e-6))
    col = np.zeros((1, ny, 1), np.uint8)
    col[0, 0, 0] = col[0, -1, 0] = 1
    r1, r2 = inputs.two_layer((1, ny, 1), 1.0, 0.005)
    r1[col == 1] = 0
    r2[col == 1] = 0
    if (nuA, nuB) not in _channel_oracle:
        ora.set_threads(1)
        p = ora.Params(1, ny, 1, solid=col, **kw)
        _channel_oracle[(nuA, nuB)] = ora.moments(p, ora.run(p, ora.init(p, r1, r2), 20000))
        ora.set_threads(8)
    o1, o2, ou = _channel_oracle[(nuA, nuB)]
    shape = (nz, ny, nx)
    solid = np.broadcast_to(col, shape).copy()
    ctx = lbm.lbm_init(lbm.Params(nx, ny, nz, prec=lbm.PRECISIONS[prec], solid=solid,
                                  rho_init=(np.broadcast_to(r1, shape).copy(), np.broadcast_to(r2, shape).copy()),
                                  check_every=1000, tau_crit=tau_crit,
                                  mass_tol=0.0 if prec in ("fp64", "fp32") else 1.0, **kw))
    m0 = lbm.lbm_info(ctx)["mass0"]
    lbm.lbm_step(ctx, 20000)
    g1, g2, gu = lbm.lbm_moments(ctx)
    red = lbm.lbm_reduce(ctx)
    drift = [abs(red[k] - m0[k]) / m0[k] for k in range(2)]
    devs = [nmax(g1, np.broadcast_to(o1, shape)), nmax(g2, np.broadcast_to(o2, shape)),
            nmax(gu, np.broadcast_to(ou, (3,) + shape))]
    # x and z stay uniform on the GPU too
    spread = float(np.abs(gu[2] - gu[2][:1, :, :1]).max() / np.abs(gu[2]).max())
    uabs = float(np.abs(gu - np.broadcast_to(ou, (3,) + shape)).max())
    record("channel_8x64x256", arm=arm, prec=prec, tau_crit=tau_crit, nuA=nuA, nuB=nuB, dev=devs, u_abs=uabs,
           xz_spread=spread, mass_drift=drift)
    assert np.isfinite(gu).all()
    if prec == "fp64":
        assert max(devs[:2]) <= TOL["fp64"] and uabs <= TOL["fp64"]
        assert spread <= 1e-13
    elif prec == "fp32":
        assert max(devs[:2]) <= 1.2e-3 and uabs <= 2e-5   # regression guard; not the 1e-5 bar (see above)
        assert spread <= 1e-5
    else:
        assert max(devs[:2]) <= 0.4 and uabs <= 0.04      # regression guard; the form fails this case


@pytest.fixture(scope="module")
def packed_spheres():
    """The benchmark workload: 256^3 packed spheres (radius 12, porosity
    0.40), 1 % droplets of A, nu ratio 10, G = -4.2, g = 1e-6 along z,
    rho^s = 0.25."""
    solid, rA, rB, info = inputs.packed_spheres_case(n=256, radius=12.0, porosity=0.40, drop_radius=4.0,
                                                     drop_fraction=0.01, seed=3, minority=0.03)
    phys = dict(tau=(1.0 / 60.0 / (1.0 / 3.0) + 0.5, 1.0), G=-4.2, g=(0.0, 0.0, 1e-6), rho_s=0.25)
    return solid, rA, rB, phys


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16s", "bf16s"])
def test_full_size_sampled_sites(lbm, ora, packed_spheres, prec):
    """At the benchmark's full size and launch configuration (default tile
    and z-chunk), two steps: the first from the known initial state, the
    second from the GPU's own state after one step.  4000 seeded fluid sites
    (half of them next to a wall) are recomputed one by one by the oracle.
    FP64 to 1e-12, FP32 to 1e-5.  FP16S and BF16S: each stored population
    carries one rounding of its deviation f - w rho_ref (relative 2^-11 or
    2^-8, the deviation at most max |f|) on entry and on store, and the entry
    rounding propagates through the step: bound 4 x 2^-11 or 4 x 2^-8 of
    max |f| (as for the one-step 16-bit test)."""
    import torch
    solid, rA, rB, phys = packed_spheres
    n = solid.shape[0]
    ctx = lbm.lbm_init(lbm.Params(n, n, n, prec=lbm.PRECISIONS[prec], solid=solid, rho_init=(rA, rB),
                                  check_every=100, **phys))
    tol = {"fp64": TOL["fp64"], "fp32": TOL["fp32"], "fp16s": 4 * 2.0 ** -11, "bf16s": 4 * 2.0 ** -8}[prec]
    p = ora.Params(n, n, n, solid=solid, **phys)
    fluid = np.flatnonzero(solid.ravel() == 0)
    near = np.zeros(solid.shape, bool)
    for ax in range(3):
        for sh in (1, -1):
            near |= np.roll(solid, sh, axis=ax) == 1
    nearwall = np.flatnonzero((solid.ravel() == 0) & near.ravel())
    pick = np.concatenate([fluid[(inputs.uniform(91, 2000) * len(fluid)).astype(np.int64)],
                           nearwall[(inputs.uniform(92, 2000) * len(nearwall)).astype(np.int64)]])
    f_prev = ora.init(p, rA, rB)
    fd = torch.empty((2, 19) + solid.shape, dtype=torch.float64, device="cuda")
    idx = torch.from_numpy(pick).cuda()
    for step in range(2):
        lbm.lbm_step(ctx, 1)
        lbm.lbm_get_populations(ctx, fd)
        got = fd.view(2, 19, -1)[:, :, idx].permute(2, 0, 1).cpu().numpy()
        want = ora.step_sites(p, f_prev, pick)
        dev = nmax(got, want)
        record("packed_spheres_256_sampled", prec=prec, tile=list(lbm.lbm_info(ctx)["tile"]), step=step + 1,
               dev=dev, sites=int(len(pick)))
        assert dev <= tol
        if step == 0:
            f_prev = fd.cpu().numpy()
    del fd


@pytest.mark.parametrize("prec,gpu_kw,ora_kw", [
    ("fp32", dict(eq_kind=1, wall_kind=1), dict(eq_kind=1, wall_kind=1)),
    ("fp16s", dict(tau_crit=0.6), {}),
    ("bf16s", dict(tau_crit=0.6), {})])
def test_full_size_variants_sampled_sites(lbm, ora, packed_spheres, prec, gpu_kw, ora_kw):
    """The benchmark workload at its launch shape with the paper's variants:
    at FP32 the full equilibrium and the momentum-balanced wall force; at 16
    bits the instance that forms P_ab in FP64 where tau_mix < 0.6 (the A-rich
    sites, tau_A = 0.55).  One step, 4000 seeded sites (half next to a wall)
    against the oracle; bounds as in test_full_size_sampled_sites."""
    import torch
    solid, rA, rB, phys = packed_spheres
    n = solid.shape[0]
    ctx = lbm.lbm_init(lbm.Params(n, n, n, prec=lbm.PRECISIONS[prec], solid=solid, rho_init=(rA, rB),
                                  check_every=100, **phys, **gpu_kw))
    tol = {"fp32": TOL["fp32"], "fp16s": 4 * 2.0 ** -11, "bf16s": 4 * 2.0 ** -8}[prec]
    p = ora.Params(n, n, n, solid=solid, **phys, **ora_kw)
    fluid = np.flatnonzero(solid.ravel() == 0)
    near = np.zeros(solid.shape, bool)
    for ax in range(3):
        for sh in (1, -1):
            near |= np.roll(solid, sh, axis=ax) == 1
    nearwall = np.flatnonzero((solid.ravel() == 0) & near.ravel())
    pick = np.concatenate([fluid[(inputs.uniform(97, 2000) * len(fluid)).astype(np.int64)],
                           nearwall[(inputs.uniform(98, 2000) * len(nearwall)).astype(np.int64)]])
    f0 = ora.init(p, rA, rB)
    fd = torch.empty((2, 19) + solid.shape, dtype=torch.float64, device="cuda")
    lbm.lbm_step(ctx, 1)
    lbm.lbm_get_populations(ctx, fd)
    got = fd.view(2, 19, -1)[:, :, torch.from_numpy(pick).cuda()].permute(2, 0, 1).cpu().numpy()
    del fd
    want = ora.step_sites(p, f0, pick)
    dev = nmax(got, want)
    record("packed_spheres_256_variants", prec=prec, kw=gpu_kw, tile=list(lbm.lbm_info(ctx)["tile"]), dev=dev)
    lbm.lbm_free(ctx)
    assert dev <= tol


@pytest.mark.parametrize("prec", ["fp32", "fp16s"])
def test_full_size_all_fluid_sampled_sites(lbm, ora, prec):
    """The benchmark's all-fluid lattice (256^3, a droplet of A of radius 40
    in B, no solids, G = -3, tau = 1) at its default launch shape: two
    steps, 4000 seeded sites (half within two sites of the interface, where
    the force is largest) recomputed one by one by the oracle; bounds as in
    the packed-sphere test."""
    import torch
    n = 256
    shape = (n, n, n)
    rA, rB = inputs.droplet(shape, n / 6.4)
    solid = np.zeros(shape, np.uint8)
    phys = dict(tau=(1.0, 1.0), G=-3.0, g=(0.0, 0.0, 0.0), rho_s=0.0)
    ctx = lbm.lbm_init(lbm.Params(n, n, n, prec=lbm.PRECISIONS[prec], solid=solid, rho_init=(rA, rB),
                                  check_every=100, **phys))
    tol = {"fp32": TOL["fp32"], "fp16s": 4 * 2.0 ** -11}[prec]
    p = ora.Params(n, n, n, solid=solid, **phys)
    z, y, x = np.indices(shape, dtype=np.float64)
    c = n / 2.0   # the droplet's centre (inputs.droplet)
    rr = np.sqrt((x - c) ** 2 + (y - c) ** 2 + (z - c) ** 2)
    del x, y, z
    band = np.flatnonzero(np.abs(rr.ravel() - n / 6.4) < 2.0)
    del rr
    pick = np.concatenate([(inputs.uniform(95, 2000) * solid.size).astype(np.int64),
                           band[(inputs.uniform(96, 2000) * len(band)).astype(np.int64)]])
    f_prev = ora.init(p, rA, rB)
    fd = torch.empty((2, 19) + shape, dtype=torch.float64, device="cuda")
    idx = torch.from_numpy(pick).cuda()
    for step in range(2):
        lbm.lbm_step(ctx, 1)
        lbm.lbm_get_populations(ctx, fd)
        got = fd.view(2, 19, -1)[:, :, idx].permute(2, 0, 1).cpu().numpy()
        want = ora.step_sites(p, f_prev, pick)
        dev = nmax(got, want)
        record("all_fluid_256_sampled", prec=prec, tile=list(lbm.lbm_info(ctx)["tile"]), step=step + 1, dev=dev,
               sites=int(len(pick)))
        assert dev <= tol
        if step == 0:
            f_prev = fd.cpu().numpy()
    del fd
    lbm.lbm_free(ctx)


@pytest.mark.parametrize("prec,nz,zfar", [("fp64", 192, 188), ("fp32", 384, 376)])
def test_population_offsets_beyond_2_gib(lbm, ora, prec, nz, zfar):
    """A half of the population storage may reach 4 GiB, so byte offsets
    within a half of 2 GiB and more (negative as 32-bit ints) must address
    fluid sites like any other.  A 256 x 256 x nz lattice, fluid but for a
    wall row, one step from a seeded random state at the default launch
    shape: FP64 runs the single-pass step, FP32 the pipelined one that the
    16-bit forms share.  2000 sites of planes >= zfar (all of whose offsets
    are past 2 GiB), 500 next to the wall and 500 anywhere are recomputed by
    the oracle (FP64 to 1e-12, FP32 to 1e-5)."""
    import torch
    ny = nx = 256
    shape = (nz, ny, nx)
    solid = np.zeros(shape, np.uint8)
    solid[:, 0, :] = 1
    n = solid.size
    rA = (0.7 + 0.1 * inputs.uniform(301, n)).reshape(shape)
    rB = (0.3 + 0.1 * inputs.uniform(302, n)).reshape(shape)
    rA[solid == 1] = 0
    rB[solid == 1] = 0
    phys = dict(tau=(0.8, 1.2), G=-1.0, g=(0.0, 0.0, 1e-5), rho_s=0.2)
    # Sites are numbered plane by plane, so a site of plane z has slot
    # k >= (fluid sites of the planes below); its offset in its half is at
    # least (11 k - 352) pair sizes (11 direction runs of 32 pairs a group).
    pb = {"fp64": 16, "fp32": 8}[prec]
    k_min = zfar * nx * (ny - 1)
    assert (11 * k_min - 352) * pb >= 2 ** 31
    ctx = lbm.lbm_init(lbm.Params(nx, ny, nz, prec=lbm.PRECISIONS[prec], solid=solid, rho_init=(rA, rB),
                                  check_every=0, **phys))
    p = ora.Params(nx, ny, nz, solid=solid, **phys)
    plane = nx * ny
    far = zfar * plane + (inputs.uniform(303, 2000) * ((nz - zfar) * plane)).astype(np.int64)
    wall = (inputs.uniform(304, 500) * nz).astype(np.int64) * plane + nx + \
        (inputs.uniform(305, 500) * nx).astype(np.int64)
    anyw = (inputs.uniform(306, 500) * n).astype(np.int64)
    far = far[solid.ravel()[far] == 0]
    pick = np.concatenate([far, anyw[solid.ravel()[anyw] == 0], wall])
    f0 = ora.init(p, rA, rB)
    lbm.lbm_step(ctx, 1)
    fd = torch.empty((2, 19) + shape, dtype=torch.float64, device="cuda")
    lbm.lbm_get_populations(ctx, fd)
    got = fd.view(2, 19, -1)[:, :, torch.from_numpy(pick).cuda()].permute(2, 0, 1).cpu().numpy()
    del fd
    want = ora.step_sites(p, f0, pick)
    del f0
    dev = nmax(got, want)
    dev_far = nmax(got[:len(far)], want[:len(far)])
    record("offsets_beyond_2gib", prec=prec, shape=list(shape), tile=list(lbm.lbm_info(ctx)["tile"]), dev=dev,
           dev_far=dev_far, sites=int(len(pick)))
    lbm.lbm_free(ctx)
    assert dev <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16s", "bf16s"])
def test_resume_into_placeholder_context(lbm, prec):
    """A checkpoint resumed into a context created from placeholder fields
    (uniform densities far from the state's): the periodic mass check then
    compares against the resumed state's masses (no false drift error), at
    16 bits the default shift becomes the resumed state's mean density, and
    the run continues as the original context's does -- bit for bit at FP64
    and FP32, within the storage rounding at 16 bits."""
    shape = (18, 20, 26)
    nz, ny, nx = shape
    solid = np.zeros(shape, np.uint8)
    solid[:, 0, :] = 1
    rA, rB = inputs.droplet(shape, 5.0, center=(13.0, 10.0, 9.0))
    rA[solid == 1] = 0
    rB[solid == 1] = 0
    kw = dict(prec=lbm.PRECISIONS[prec], solid=solid, tau=(0.8, 1.2), G=-3.0, g=(0.0, 0.0, 1e-5), rho_s=0.2,
              check_every=5, mass_tol=1e-6 if prec in ("fp64", "fp32") else 1e-2)
    a = lbm.lbm_init(lbm.Params(nx, ny, nz, rho_init=(rA, rB), **kw))
    lbm.lbm_step(a, 10)
    mid = lbm.lbm_get_populations(a)
    lbm.lbm_step(a, 20)
    end_a = lbm.lbm_moments(a)
    ph = np.where(solid == 1, 0.0, 5.0)
    b = lbm.lbm_init(lbm.Params(nx, ny, nz, rho_init=(ph, ph.copy()), **kw))
    lbm.lbm_set_populations(b, mid)
    mass_mid = [float(mid[d][:, solid == 0].sum()) for d in range(2)]
    m0 = lbm.lbm_info(b)["mass0"]
    # the check sums densities formed in the storage's arithmetic (FP32 at FP32)
    np.testing.assert_allclose(m0, mass_mid, rtol={"fp64": 1e-12, "fp32": 1e-6}.get(prec, 2e-3))
    lbm.lbm_step(b, 20)   # periodic checks against the resumed masses
    end_b = lbm.lbm_moments(b)
    devs = [nmax(x, y) for x, y in zip(end_b, end_a)]
    record("resume_placeholder", prec=prec, dev=devs)
    if prec in ("fp64", "fp32"):
        assert all(np.array_equal(x, y) for x, y in zip(end_b, end_a))
    else:
        assert max(devs[:2]) <= 8 * (2.0 ** -11 if prec == "fp16s" else 2.0 ** -8)
