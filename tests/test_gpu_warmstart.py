"""The learned warm start (needs an MI355X): the library calls it rests on
(the restart from fields with the strain's non-equilibrium part, the FP64
residual and distance), and the warm start end to end at a small size."""
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def record(name, **vals):
    path = os.environ.get("PARITY_LOG")
    if path:
        with open(path, "a") as fh:
            fh.write(json.dumps({"test": name, **vals}) + "\n")


def _channel(ny=34, nx=4, nz=4):
    """A z-channel with walls at y = 0 and y = ny - 1 (the wall planes sit
    half a site inside the fluid's first row, halfway bounce-back)."""
    solid = np.zeros((nz, ny, nx), np.uint8)
    solid[:, 0, :] = 1
    solid[:, ny - 1, :] = 1
    return solid


D3Q19 = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
                  [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0], [1, 0, 1], [-1, 0, -1], [1, 0, -1], [-1, 0, 1],
                  [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1]])


def test_strain_start_sets_the_viscous_flux():
    """lbm_set_fields_strain on a parabolic channel profile: the shear moment
    sum_i c_y c_z f_i of each component must equal its density share of the
    Chapman-Enskog flux -rho T0 tau_mix du_z/dy exactly (three-point
    differences are exact on a parabola, also at the half-site walls), while
    the mass and momentum moments stay those of the fields."""
    from paper_1711_03254_amd import lbm
    lbm.load_library()
    ny = 34
    solid = _channel(ny)
    y = np.arange(ny, dtype=np.float64)
    prof = 4e-3 * (y - 0.5) * (ny - 1.5 - y)
    ra = np.where(solid == 1, 0.0, 0.7)
    rb = np.where(solid == 1, 0.0, 0.3)
    u = np.zeros((3,) + solid.shape)
    u[2] = np.where(solid == 1, 0.0, prof[None, :, None])
    tau = (0.8, 1.3)
    ctx = lbm.lbm_init(lbm.Params(4, ny, 4, prec=lbm.LBM_FP64, tau=tau, solid=solid, rho_init=(ra, rb), u_init=u))
    lbm.lbm_set_fields_strain(ctx, ra, rb, u)
    f = lbm.lbm_get_populations(ctx)
    c = D3Q19.astype(np.float64)
    fl = solid == 0
    tmix = (0.7 * tau[0] + 0.3 * tau[1]) / 1.0
    dudy = 4e-3 * (ny - 1.5 - y - (y - 0.5))
    want = -(1.0 / 3.0) * tmix * dudy[None, :, None] * np.ones(solid.shape)
    for a, share in ((0, 0.7), (1, 0.3)):
        pyz = np.einsum("i,i...->...", c[:, 1] * c[:, 2], f[a])
        np.testing.assert_allclose(pyz[fl], (share * want)[fl], rtol=1e-12, atol=1e-16)
        mass = f[a].sum(0)
        np.testing.assert_allclose(mass[fl], share, rtol=1e-13)
        jz = np.einsum("i,i...->...", c[:, 2], f[a])
        np.testing.assert_allclose(jz[fl], (share * u[2])[fl], rtol=1e-12, atol=1e-17)
    lbm.lbm_free(ctx)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_strain_start_is_near_steady(prec):
    """A miscible mixture in a body-force-driven channel started from its
    steady Poiseuille profile: with the strain's non-equilibrium part the
    first steps barely change u (the viscous stress already balances the
    force); from the equilibrium alone the force accelerates the fluid
    unopposed until the stress has built up.  tau_mix = 0.61: at tau_mix = 1
    the collision discards the non-equilibrium part whatever it is, and
    the two starts coincide after one step.  The profile is given as u_F,
    as lbm_moments reports it."""
    from paper_1711_03254_amd import lbm
    lbm.load_library()
    ny = 34
    solid = _channel(ny)
    y = np.arange(ny, dtype=np.float64)
    tau = (0.55, 0.7)
    phi = 0.6
    nu = (1.0 / 3.0) * ((phi * tau[0] + (1 - phi) * tau[1]) - 0.5)
    g = 1e-6
    prof = g / (2 * nu) * (y - 0.5) * (ny - 1.5 - y)
    ra = np.where(solid == 1, 0.0, phi)
    rb = np.where(solid == 1, 0.0, 1 - phi)
    u = np.zeros((3,) + solid.shape)
    u[2] = np.where(solid == 1, 0.0, prof[None, :, None])
    change = {}
    for strain in (False, True):
        u0 = u.copy()
        u0[2] -= np.where(solid == 1, 0.0, g / 2)    # lbm_init takes the population velocity
        ctx = lbm.lbm_init(lbm.Params(4, ny, 4, prec=lbm.PRECISIONS[prec], tau=tau, g=(0.0, 0.0, g), solid=solid,
                                      rho_init=(ra, rb), u_init=u0))
        if strain:
            lbm.lbm_set_fields_strain(ctx, ra, rb, u)
        lbm.lbm_residual(ctx)
        lbm.lbm_step(ctx, 10)
        change[strain] = lbm.lbm_residual(ctx)[0]
        lbm.lbm_free(ctx)
    record(f"strain_start_{prec}", eq_change=change[False], strain_change=change[True])
    assert change[True] < 0.2 * change[False]


@pytest.mark.parametrize("wall_kind,rho_s", [(0, 0.0), (0, 0.3), (1, -0.3)])
def test_restart_gives_back_its_velocity(wall_kind, rho_s):
    """lbm_set_fields_strain takes u_F of Eq. (8): the populations it sets
    carry each component's momentum rho_a u_F - F_a / 2 with F_a from its own
    force routine, so lbm_moments, which forms u_F = (j + F / 2) / rho with
    the step's force, must give u_F back to rounding -- with solids, a wall
    potential of either sign, both wall forms, coupling and gravity (the
    strain part carries no momentum, and the equilibrium's third-order
    terms none either on D3Q19)."""
    from paper_1711_03254_amd import inputs, lbm
    lbm.load_library()
    shape = (12, 16, 20)
    rng = np.random.default_rng(40 + wall_kind)
    solid = inputs.random_mask(shape, 0.2, 41)
    ra = np.where(solid == 1, 0.0, inputs.smooth_random_density(shape, 42, mean=0.7, amp=0.1))
    rb = np.where(solid == 1, 0.0, inputs.smooth_random_density(shape, 43, mean=0.3, amp=0.1))
    u = np.where(solid[None] == 1, 0.0, rng.normal(scale=1e-3, size=(3,) + shape))
    ctx = lbm.lbm_init(lbm.Params(shape[2], shape[1], shape[0], prec=lbm.LBM_FP64, tau=(0.7, 1.2), G=-1.5,
                                  g=(1e-5, -2e-5, 3e-5), rho_s=rho_s, wall_kind=wall_kind, solid=solid,
                                  rho_init=(ra, rb)))
    lbm.lbm_set_fields_strain(ctx, ra, rb, u)
    ga, gb, gu = lbm.lbm_moments(ctx)
    lbm.lbm_free(ctx)
    np.testing.assert_allclose(ga, ra, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(gb, rb, rtol=1e-13, atol=1e-15)
    assert np.abs(gu - u).max() <= 1e-12 * np.abs(u).max()


def test_residual_matches_the_fields():
    """lbm_residual against the same norms taken on the host from
    lbm_moments, on a coupled mixture in a porous subvolume."""
    from paper_1711_03254_amd import inputs, lbm, warmstart as ws
    lbm.load_library()
    solid, ra0, rb0, _ = inputs.mixture_case(32, 901, radius_range=(1.5, 4.0))
    ctx = ws.make_context(solid, ra0, rb0, ws.physics(G=-1.0), "fp64")
    assert lbm.lbm_residual(ctx) == (1.0, 1.0)    # against zero fields
    a0, _, u0 = lbm.lbm_moments(ctx)
    lbm.lbm_step(ctx, 7)
    du, da = lbm.lbm_residual(ctx)
    a1, _, u1 = lbm.lbm_moments(ctx)
    np.testing.assert_allclose(du, np.linalg.norm(u1 - u0) / np.linalg.norm(u1), rtol=1e-10)
    np.testing.assert_allclose(da, np.linalg.norm(a1 - a0) / np.linalg.norm(a1), rtol=1e-10)
    assert lbm.lbm_residual(ctx) == (0.0, 0.0)    # nothing stepped since the last call
    lbm.lbm_free(ctx)


def test_restart_from_fields_follows_the_state():
    """A coupled mixture (G = -1) in a porous subvolume stepped 3000 steps at
    FP64, restarted from its fields (rho1, rho2, u_F) into fresh contexts:
    through lbm_set_fields_strain the restart follows the original run
    (the force shift and the strain's non-equilibrium part set the
    populations the fields imply); the plain equilibrium of u_F (lbm_set_fields)
    does not.  lbm_distance of a state against its own fields is 0."""
    from paper_1711_03254_amd import inputs, lbm, warmstart as ws
    lbm.load_library()
    solid, ra0, rb0, _ = inputs.mixture_case(32, 902, radius_range=(1.5, 4.0))
    phys = ws.physics()
    ctx = ws.make_context(solid, ra0, rb0, phys, "fp64")
    lbm.lbm_step(ctx, 3000)
    u, ra, rb = ws.fields(ctx, solid.shape)
    assert lbm.lbm_distance(ctx, ra, u) == (0.0, 0.0)
    strain = ws.make_context(solid, ra, rb, phys, "fp64")
    lbm.lbm_set_fields_strain(strain, ra, rb, u)
    plain = ws.make_context(solid, ra, rb, phys, "fp64")
    lbm.lbm_set_fields(plain, ra, rb, u)
    for c in (ctx, strain, plain):
        lbm.lbm_step(c, 200)
    u1, ra1, _ = ws.fields(ctx, solid.shape)
    d_strain = lbm.lbm_distance(strain, ra1, u1)
    d_plain = lbm.lbm_distance(plain, ra1, u1)
    record("restart_from_fields", strain=d_strain, plain=d_plain)
    assert d_strain[0] < 0.1 * d_plain[0]
    assert d_strain[0] < 1e-2 and d_strain[1] < 1e-4
    for c in (ctx, strain, plain):
        lbm.lbm_free(c)


def test_warm_start_end_to_end():
    """Solver-generated samples with the coupling on, the surrogate trained
    on them by its own kernels, and a held-out case solved cold and warm at
    FP32 and FP16S storage to the same accuracy against a long cold FP64
    solve.  Asserted: training lowers the loss, the FP32 cold solve
    reaches the target, and the FP32 warm solve moves towards the same
    state (its distance to the reference falls).  Whether and by how much
    the warm start is faster (steps and time to the target) is recorded,
    not assumed: on this tiny, tortuous case a poor prediction can also be
    slower, and at FP16S storage cold and warm solves alike stall where the
    per-step corrections fall below the 16-bit resolution of the
    populations (the flow in these small pores is slow: u_F about 1e-4)."""
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1711_03254_amd import inputs, lbm, surrogate, warmstart as ws
    lbm.load_library()
    phys = ws.physics()
    rr = (1.5, 4.0)
    train = [ws.steady_sample(32, 700 + k, phys, steps=6000, radius_range=rr) for k in range(6)]
    net = surrogate.Surrogate(base=16, seed=2)
    net.u_scale = ws.u_scale_of(train, phys)
    net.rho_scale = ws.rho_scale_of(train)
    hist = ws.train(net, train, phys, epochs=200, lr=1e-3)
    assert np.isfinite(hist[-1]) and hist[-1] < hist[0] / 3
    solid, ra0, rb0, info = inputs.mixture_case(32, 900, radius_range=rr)
    ref_a, ref_u, _ = ws.reference(solid, ra0, rb0, phys, 20000)
    targets = [(0.05, 0.005)]
    r = ws.compare(net, dict(solid=solid, ra0=ra0, rb0=rb0), phys, (ref_a, ref_u), targets, every=500,
                   max_steps=30000)
    assert r["fp32"]["cold"]["reached"][0] is not None, r["fp32"]["cold"]["final"]
    w = r["fp32"]["warm"]["trajectory"]
    assert w[-1][1] < 0.5 * w[0][1] or r["fp32"]["warm"]["reached"][0] is not None, (w[0], w[-1])
    record("warm_start_32", loss_first=hist[0], loss_last=hist[-1], prediction=r["prediction_distance"],
           factors={p: r[p]["factors"] for p in ("fp32", "fp16s")},
           reached={p: {a: r[p][a]["reached"][0] for a in ("cold", "warm")} for p in ("fp32", "fp16s")},
           final={p: {a: r[p][a]["final"] for a in ("cold", "warm")} for p in ("fp32", "fp16s")})


def test_trained_surrogate_shortens_the_solve_at_128():
    """What the committed surrogate gains over the method without it, on a
    held-out 128^3 coupled subvolume (seed 10100, not among the training
    seeds): steps to the accuracy target (4e-2 in u_F, 4e-3 in rho_A against
    100 000 cold FP64 steps) from the cold start and from the warm start, at
    FP32 and FP16S storage.  Asserted: the warm start reaches the target in
    fewer steps at both (measured with the 200 000-step reference: 500
    against 2500 at FP32, 500 against 6000 at FP16S), and the prediction is
    closer to the reference than the cold state in both fields."""
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1711_03254_amd import inputs, lbm, surrogate, warmstart as ws
    lbm.load_library()
    here = os.path.dirname(os.path.abspath(__file__))
    net = surrogate.Surrogate.load(os.path.join(here, "..", "paper_1711_03254_amd", "weights",
                                                "surrogate_coupled_128.npz"))
    phys = ws.physics()
    solid, ra0, rb0, _ = inputs.mixture_case(128, 10100)
    ref_a, ref_u, _ = ws.reference(solid, ra0, rb0, phys, 100000)
    r = ws.compare(net, dict(solid=solid, ra0=ra0, rb0=rb0), phys, (ref_a, ref_u), [(0.04, 0.004)], every=500,
                   max_steps=20000)
    steps = {p: {a: (r[p][a]["reached"][0] or {}).get("steps") for a in ("cold", "warm")} for p in ("fp32", "fp16s")}
    record("warm_start_128", prediction=r["prediction_distance"], cold_start=r["cold_start_distance"], steps=steps,
           predict_seconds=r["predict_seconds"], factors={p: r[p]["factors"]["warm"] for p in ("fp32", "fp16s")})
    assert r["prediction_distance"]["u"] < r["cold_start_distance"]["u"]
    assert r["prediction_distance"]["rho_a"] < r["cold_start_distance"]["rho_a"]
    for p in ("fp32", "fp16s"):
        assert steps[p]["cold"] is not None and steps[p]["warm"] is not None, (p, steps)
        assert steps[p]["warm"] < steps[p]["cold"], (p, steps)
