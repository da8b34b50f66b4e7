"""Invariants and symmetries of the oracle's full step (Eqs. 1-11): exact
mass conservation, momentum balance, the uniform-state special case, and
metamorphic symmetries (translation, cube symmetries, component swap)."""
import numpy as np
import pytest

from paper_1711_03254_amd import inputs

T0 = 1.0 / 3.0


def _smooth_state(ora, p, seed, u_amp=0.02):
    shape = p.shape
    r1 = inputs.smooth_random_density(shape, seed, mean=0.6, amp=0.5)
    r2 = 1.2 - r1 + inputs.smooth_random_density(shape, seed + 7, mean=0.0, amp=0.05)
    u = u_amp * (inputs.uniform(seed + 3, 3 * int(np.prod(shape))).reshape((3,) + shape) - 0.5)
    return ora.init(p, r1, r2, u)


def test_mass_conserved_with_walls_and_wetting(ora):
    """Each component's mass is conserved exactly (up to rounding): collision
    keeps rho_alpha (sum f_eq = rho_alpha, sum f' = 0, sum F_i = 0) and
    streaming with bounce-back permutes populations (Eq. 1, Section 2 walls)."""
    shape = (10, 9, 11)
    solid = inputs.random_mask(shape, 0.12, seed=5)
    p = ora.Params(11, 9, 10, tau=(0.6, 1.3), G=-2.5, g=(1e-4, -2e-4, 3e-4), rho_s=0.4, solid=solid)
    f = _smooth_state(ora, p, 11)
    m0 = ora.reduce(p, f)
    n = 200
    g = ora.run(p, f, n)
    m1 = ora.reduce(p, g)
    assert abs(m1[0] - m0[0]) <= n * 5e-15 * m0[0]
    assert abs(m1[1] - m0[1]) <= n * 5e-15 * m0[1]
    assert np.isfinite(g).all()


def test_momentum_balance_periodic(ora):
    """No solids: the Shan-Chen forces of Eq. (7) cancel pairwise over the
    lattice, so total momentum grows by exactly (sum rho) g per step.  The
    reported sum of rho u_F is that momentum plus half the step's force
    (Eq. 8)."""
    shape = (8, 7, 9)
    gv = np.array([2e-5, -1e-5, 3e-5])
    p = ora.Params(9, 7, 8, tau=(0.7, 1.1), G=-2.5, g=tuple(gv))
    f = _smooth_state(ora, p, 21, u_amp=0.05)
    M = None
    prev = None
    for _ in range(6):
        r = ora.reduce(p, f)
        mass = r[0] + r[1]
        if prev is not None:
            np.testing.assert_allclose(r[2:] - prev, mass * gv, rtol=0, atol=1e-13 * mass)
        prev = r[2:]
        M = mass
        f = ora.step(p, f)
    assert M > 0


def test_momentum_conserved_without_body_force(ora):
    shape = (6, 8, 7)
    p = ora.Params(7, 8, 6, tau=(0.55, 2.0), G=-3.0)
    f = _smooth_state(ora, p, 31, u_amp=0.05)
    r0 = ora.reduce(p, f)
    r1 = ora.reduce(p, ora.run(p, f, 25))
    np.testing.assert_allclose(r1[2:], r0[2:], atol=1e-13 * (r0[0] + r0[1]))


@pytest.mark.parametrize("tau", [(0.7, 1.9), (0.5051, 5.6)])
def test_uniform_state_accelerates_exactly(ora, tau):
    """Uniform state with a body force (Eq. 3 as printed): the interaction
    force vanishes, the non-equilibrium flux stays zero, and the bare velocity
    grows as u(t) = u0 + g t, so the reported u_F = u0 + g (t + 1/2)
    (Eq. 8)."""
    shape = (4, 5, 3)
    gv = np.array([1e-4, 2e-4, -1e-4])
    u0 = np.array([0.01, -0.02, 0.005])
    p = ora.Params(3, 5, 4, tau=tau, G=-4.2, g=tuple(gv))
    r1 = np.full(shape, 0.7)
    r2 = np.full(shape, 0.3)
    u = np.broadcast_to(u0[:, None, None, None], (3,) + shape)
    f = ora.init(p, r1, r2, u)
    for t in range(0, 40):
        if t % 13 == 0:
            a, b, uF = ora.moments(p, f)
            np.testing.assert_allclose(a, 0.7, atol=1e-15)
            np.testing.assert_allclose(b, 0.3, atol=1e-15)
            want = u0 + gv * (t + 0.5)
            np.testing.assert_allclose(uF.reshape(3, -1), np.repeat(want[:, None], a.size, 1), atol=2e-15)
        f = ora.step(p, f)


def test_translation_is_bitwise(ora):
    """Periodic translation commutes with the step, bit for bit."""
    shape = (6, 7, 8)
    solid = inputs.random_mask(shape, 0.1, seed=9)
    p = ora.Params(8, 7, 6, tau=(0.6, 1.4), G=-2.5, g=(1e-5, 0, 2e-5), rho_s=-0.3, solid=solid)
    f = _smooth_state(ora, p, 41)
    f[:, :, solid == 1] = 0.0
    sh = (2, -3, 5)
    ps = ora.Params(8, 7, 6, tau=p.tau, G=p.G, g=p.g, rho_s=p.rho_s, solid=np.roll(solid, sh, axis=(0, 1, 2)))
    a = np.roll(ora.run(p, f, 3), sh, axis=(2, 3, 4))
    b = ora.run(ps, np.roll(f, sh, axis=(2, 3, 4)), 3)
    assert np.array_equal(a, b)


def test_uniform_directions_reduce_to_column(ora):
    """A state that is uniform in x and z evolves exactly as the same column
    on a 1 x ny x 1 lattice."""
    ny = 12
    solid_col = np.zeros((1, ny, 1), np.uint8)
    solid_col[0, 0, 0] = solid_col[0, -1, 0] = 1
    r1 = inputs.two_layer((1, ny, 1))[0]
    r2 = inputs.two_layer((1, ny, 1))[1]
    r1[solid_col == 1] = 0
    r2[solid_col == 1] = 0
    kw = dict(tau=(0.9, 1.6), G=-2.5, g=(0, 0, 1e-5), rho_s=0.2)
    pc = ora.Params(1, ny, 1, solid=solid_col, **kw)
    fc = ora.run(pc, ora.init(pc, r1, r2), 20)
    shape = (5, ny, 4)
    pb = ora.Params(4, ny, 5, solid=np.broadcast_to(solid_col, shape).copy(), **kw)
    fb = ora.run(pb, ora.init(pb, np.broadcast_to(r1, shape).copy(), np.broadcast_to(r2, shape).copy()), 20)
    for z in range(5):
        for x in range(4):
            assert np.array_equal(fb[:, :, z, :, x], fc[:, :, 0, :, 0])


def _direction_permutation(c, R):
    rc = c @ R.T
    perm = np.empty(19, int)
    for i in range(19):
        perm[i] = int(np.nonzero((c == rc[i]).all(1))[0][0])
    return perm  # direction i maps onto direction perm[i]


@pytest.mark.parametrize("axes,flips", [((1, 0, 2), (1, 1, 1)), ((0, 1, 2), (-1, 1, 1)),
                                        ((2, 0, 1), (1, -1, 1)), ((1, 2, 0), (-1, -1, -1))])
def test_cube_symmetries_commute(ora, axes, flips):
    """Rotations and reflections of the cubic lattice commute with the step
    (D3Q19 is invariant under the cube group)."""
    n = 7
    shape = (n, n, n)
    solid = inputs.random_mask(shape, 0.1, seed=13)
    gv = np.array([1e-4, -2e-4, 3e-5])
    p = ora.Params(n, n, n, tau=(0.58, 1.7), G=-2.5, g=tuple(gv), rho_s=0.35, solid=solid)
    f = _smooth_state(ora, p, 51)
    f[:, :, solid == 1] = 0
    c, _, _ = ora.lattice()
    # new coordinate d = flips[d] * old coordinate axes[d]; arrays are (z, y, x)
    R = np.zeros((3, 3), int)
    for d in range(3):
        R[d, axes[d]] = flips[d]
    perm = _direction_permutation(c, R)

    def tf_scalar(a):
        # a is (z, y, x); build new array b[x'] with x'_d = flips_d * x_{axes_d}
        spatial_axes = [2 - axes[d] for d in (2, 1, 0)]  # new (z, y, x) axis order in old array terms
        b = np.transpose(a, spatial_axes)
        for d in range(3):
            if flips[d] < 0:
                b = np.flip(b, axis=2 - d)
        return np.ascontiguousarray(b)

    def tf_pop(F):
        out = np.empty_like(F)
        for a in range(2):
            for i in range(19):
                out[a, perm[i]] = tf_scalar(F[a, i])
        return out

    pr = ora.Params(n, n, n, tau=p.tau, G=p.G, g=tuple(R @ gv), rho_s=p.rho_s, solid=tf_scalar(solid))
    a = tf_pop(ora.run(p, f, 4))
    b = ora.run(pr, tf_pop(f), 4)
    np.testing.assert_allclose(b, a, rtol=0, atol=2e-15)


def test_component_swap_symmetry(ora):
    """Swapping the components together with tau_1 <-> tau_2 and
    rho^s -> -rho^s swaps the result (Eqs. 6, 7, 11 are symmetric in the
    component labels)."""
    shape = (6, 7, 5)
    solid = inputs.random_mask(shape, 0.1, seed=17)
    p = ora.Params(5, 7, 6, tau=(0.53, 2.5), G=-2.5, g=(0, 1e-4, 0), rho_s=0.45, solid=solid)
    q = ora.Params(5, 7, 6, tau=(2.5, 0.53), G=-2.5, g=(0, 1e-4, 0), rho_s=-0.45, solid=solid)
    f = _smooth_state(ora, p, 61)
    a = ora.run(p, f, 5)
    b = ora.run(q, f[::-1].copy(), 5)
    np.testing.assert_allclose(b[::-1], a, rtol=0, atol=1e-14)
