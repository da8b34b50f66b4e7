"""Pins of the oracle's lattice, equilibrium and regularization against closed
forms (Section 2: D3Q19 with fourth-order isotropy, Eq. 3, Eq. 10)."""
import itertools

import numpy as np
import pytest

T0 = 1.0 / 3.0


def test_lattice_identities(ora):
    """D3Q19 weight moments: sum w = 1, odd moments vanish, second moment
    T0 delta, fourth moment T0^2 (dd + dd + dd)  (Section 2, D3Q19 with
    fourth-order isotropy)."""
    c, w, opp = ora.lattice()
    assert c.shape == (19, 3)
    assert len({tuple(v) for v in c}) == 19
    assert abs(w.sum() - 1.0) < 4e-16
    np.testing.assert_allclose(np.einsum("i,ia->a", w, c), 0.0, atol=4e-16)
    np.testing.assert_allclose(np.einsum("i,ia,ib->ab", w, c, c), T0 * np.eye(3), atol=4e-16)
    np.testing.assert_allclose(np.einsum("i,ia,ib,ic->abc", w, c, c, c), 0.0, atol=4e-16)
    m4 = np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c)
    d = np.eye(3)
    iso = T0 ** 2 * (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
                     + np.einsum("ad,bc->abcd", d, d))
    np.testing.assert_allclose(m4, iso, atol=4e-16)
    assert abs(np.sum(w * c[:, 0] ** 4) - 3 * T0 ** 2) < 4e-16
    assert abs(np.sum(w * c[:, 0] ** 2 * c[:, 1] ** 2) - T0 ** 2) < 4e-16
    # opposite index table
    np.testing.assert_array_equal(c[opp], -c)
    # the fixed direction order: rest, +x -x +y -y +z -z, then xy, xz, yz diagonals
    assert (c[0] == 0).all()
    np.testing.assert_array_equal(c[1:7], [[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]])
    assert (c[7:11, 2] == 0).all() and (c[11:15, 1] == 0).all() and (c[15:19, 0] == 0).all()
    speeds = (c ** 2).sum(1)
    np.testing.assert_allclose(w[speeds == 0], 1 / 3)
    np.testing.assert_allclose(w[speeds == 1], 1 / 18)
    np.testing.assert_allclose(w[speeds == 2], 1 / 36)


def _random_cases(n, seed):
    rng = np.random.default_rng(seed)
    for _ in range(n):
        yield rng.uniform(0.01, 2.0), rng.uniform(-0.15, 0.15, 3)


@pytest.mark.parametrize("eq_kind", [0, 1])
def test_equilibrium_moments(ora, eq_kind):
    """Eq. (3): sum f_eq = rho; sum c f_eq = rho u (the cubic terms cancel by
    fourth-order isotropy); sum c c f_eq = rho T0 delta for the printed Stokes
    form, plus rho u u when the second-order terms are included."""
    c, w, _ = ora.lattice()
    for rho, u in _random_cases(50, 1):
        fe = ora.feq(rho, u, eq_kind)
        assert abs(fe.sum() - rho) <= 1e-15 * rho * 4
        np.testing.assert_allclose(c.T @ fe, rho * u, atol=2e-15 * rho)
        second = np.einsum("ia,ib,i->ab", c, c, fe)
        want = rho * T0 * np.eye(3) + (rho * np.outer(u, u) if eq_kind == 1 else 0.0)
        np.testing.assert_allclose(second, want, atol=2e-15 * rho)
    # at rest the equilibrium is rho w_i
    np.testing.assert_allclose(ora.feq(0.7, [0, 0, 0], eq_kind), 0.7 * w, rtol=1e-15)


def test_regularization_projection(ora):
    """Eq. (10): f' = Phi:Pi has zero mass and momentum, its second moment is
    the non-equilibrium momentum flux Pi itself, and projecting f' again
    returns f' (Phi is a projector)."""
    c, w, _ = ora.lattice()
    rng = np.random.default_rng(2)
    for rho, u in _random_cases(40, 3):
        fe = ora.feq(rho, u)
        f = fe * (1 + 0.3 * rng.uniform(-1, 1, 19))
        fp, Pi = ora.regularize(f, fe)
        scale = np.abs(f - fe).sum()
        np.testing.assert_allclose(Pi, np.einsum("ia,ib,i->ab", c, c, f - fe), atol=1e-15 * scale)
        assert abs(fp.sum()) < 1e-15 * scale * 4
        np.testing.assert_allclose(c.T @ fp, 0.0, atol=1e-15 * scale * 4)
        np.testing.assert_allclose(np.einsum("ia,ib,i->ab", c, c, fp), Pi, atol=1e-15 * scale * 4)
        fpp, _ = ora.regularize(fp, np.zeros(19))
        np.testing.assert_allclose(fpp, fp, atol=1e-15 * scale * 4)


def test_regularization_kills_higher_hermite_content(ora):
    """A deviation with no second moment (momentum and third-order Hermite
    content only) has no regularized part."""
    c, w, _ = ora.lattice()
    fe = ora.feq(1.0, [0.05, -0.02, 0.01])
    # third-order Hermite direction c_x c_y c_z is zero on D3Q19; use c_x (c_y^2 - c_z^2)
    d = w * (2.0 * c[:, 1] + c[:, 0] * (c[:, 1] ** 2 - c[:, 2] ** 2))
    fp, Pi = ora.regularize(fe + 0.01 * d, fe)
    np.testing.assert_allclose(Pi, 0.0, atol=1e-17)
    np.testing.assert_allclose(fp, 0.0, atol=1e-17)
