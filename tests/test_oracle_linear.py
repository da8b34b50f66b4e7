"""Linear analysis pins of the oracle.

A single Fourier mode on a uniform mixture at rest evolves, to first order in
its amplitude, under a linear map that can be written down from the
mathematics of Section 2 alone -- here in Fourier space, as a 19x19 (G = 0)
or 38x38 (G != 0) matrix built with NumPy -- and compared with the oracle's
lattice-space run:

* G = 0, equal relaxation times, uniform total density: the map is exact (the
  cubic equilibrium terms vanish because u stays 0), so the oracle must
  follow it to rounding.  At tau = 1 the decay factor per step of a
  concentration mode has the closed form sum_i w_i cos(k . c_i).
* G != 0: the linearized map includes the Shan-Chen force of Eq. (7), the
  velocity shift of Eq. (8) and the forcing term; for an amplitude eps the
  oracle agrees to O(eps^2).  The growth or decay rate of the mode pins the
  sign, size and stencil of the interaction force.
"""
import numpy as np
import pytest

T0 = 1.0 / 3.0


def _lattice(ora):
    c, w, _ = ora.lattice()
    return c.astype(float), w


def _hermite(c):
    return np.einsum("ia,ib->iab", c, c) - T0 * np.eye(3)[None]


def _mode(shape, k, x0=0.0):
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return k[0] * x + k[1] * y + k[2] * z + x0


def _map_g0(c, w, k, omega):
    """f_hat(t+1) = M f_hat(t) for one component, G = 0, u = 0."""
    H = _hermite(c)
    HH = np.einsum("iab,jab->ij", H, H)
    collide = w[:, None] * (1.0 + (1.0 - omega) / (2 * T0 * T0) * HH)
    phase = np.exp(-1j * (c @ k))
    return phase[:, None] * collide


@pytest.mark.parametrize("tau", [1.0, 0.62, 1.8])
def test_concentration_mode_exact(ora, tau):
    c, w = _lattice(ora)
    shape = (5, 6, 8)
    k = 2 * np.pi * np.array([1 / 8, 1 / 6, 2 / 5])
    eps = 0.2
    arg = _mode(shape, k)
    r1 = 0.5 + eps * np.cos(arg)
    r2 = 0.5 - eps * np.cos(arg)
    p = ora.Params(8, 6, 5, tau=(tau, tau), G=0.0)
    f = ora.init(p, r1, r2)
    M = _map_g0(c, w, k, 1.0 / tau)
    v = w.astype(complex) * eps
    for t in range(1, 31):
        f = ora.step(p, f)
        v = M @ v
        if t in (1, 2, 7, 30):
            got = ora.moments(p, f)[0] - 0.5
            want = np.real(np.sum(v) * np.exp(1j * arg))
            np.testing.assert_allclose(got, want, rtol=0, atol=2e-15)
    if tau == 1.0:
        lam = np.sum(w * np.cos(c @ k))
        assert abs(np.sum(v).real - eps * lam ** 30) < 1e-15
        np.testing.assert_allclose(np.sum(M @ w), lam, rtol=1e-14)


def _map_sc(c, w, k, omega, G, rbar):
    """Linearized two-component map about (rbar_1, rbar_2, u = 0), state
    vector [f^1_0..18, f^2_0..18] in Fourier space."""
    H = _hermite(c)
    HH = np.einsum("iab,jab->ij", H, H)
    rho = rbar[0] + rbar[1]
    S = np.einsum("i,ia->a", w, c * np.sin(c @ k)[:, None])  # sum w c sin(k.c)
    ones = np.ones(19)
    # linear functionals: density of each component, momentum of the mixture
    D = [np.concatenate([ones, 0 * ones]), np.concatenate([0 * ones, ones])]
    J = np.concatenate([c.T, c.T], axis=1)  # (3, 38)
    # force on component a (3 x 38): G rbar_a (i S) delta rho_b
    F = [G * rbar[0] * 1j * np.outer(S, D[1]), G * rbar[1] * 1j * np.outer(S, D[0])]
    uF = J / rho + (F[0] + F[1]) / (2 * rho)
    M = np.zeros((38, 38), complex)
    phase = np.exp(-1j * (c @ k))
    for a in range(2):
        blk = slice(19 * a, 19 * a + 19)
        rows = np.zeros((19, 38), complex)
        rows += np.outer(w, D[a])                          # w_i rho_a
        rows += 3 * rbar[a] * (w[:, None] * (c @ uF))      # w_i rho_a c.u_F / T0
        sel = np.zeros((19, 38))
        sel[:, blk] = np.eye(19)
        rows += (1 - omega) / (2 * T0 * T0) * (w[:, None] * HH) @ sel  # w/(2T0^2) H:Pi
        rows += 1.5 * (w[:, None] * (c @ F[a]))            # w_i c.F / (2 T0)
        M[blk] = phase[:, None] * rows
    return M


@pytest.mark.parametrize("kvec", [(1 / 12, 1 / 5, 0.0), (1 / 12, 0.0, 0.0)])
@pytest.mark.parametrize("G,tau1,tau2", [(-1.5, 0.8, 0.8), (-3.0, 1.0, 1.0), (-2.2, 0.7, 1.6), (1.0, 0.9, 0.9)])
def test_shan_chen_mode_linearized(ora, G, tau1, tau2, kvec):
    c, w = _lattice(ora)
    shape = (4, 5, 12)
    k = 2 * np.pi * np.array(kvec)
    rbar = (0.45, 0.55)
    eps = 1e-5
    arg = _mode(shape, k)
    r1 = rbar[0] + eps * np.cos(arg)
    r2 = rbar[1] - 0.5 * eps * np.cos(arg)
    p = ora.Params(12, 5, 4, tau=(tau1, tau2), G=G)
    f = ora.init(p, r1, r2)
    pbar = rbar[0] / (rbar[0] + rbar[1])
    tau = pbar * tau1 + (1 - pbar) * tau2
    M = _map_sc(c, w, k, 1.0 / tau, G, rbar)
    v = np.concatenate([w * eps, -0.5 * w * eps]).astype(complex)
    for t in range(1, 25):
        f = ora.step(p, f)
        v = M @ v
    got1 = ora.moments(p, f)[0] - rbar[0]
    want1 = np.real(np.sum(v[:19]) * np.exp(1j * arg))
    amp = np.abs(want1).max()
    assert amp > 0
    err = np.abs(got1 - want1).max()
    assert err <= 2e-4 * amp + 1e-14
    # The separating instability: a long-wave concentration mode grows when
    # -G exceeds the spinodal value (1/rbar_1 + 1/rbar_2) / 2 of the
    # continuum limit of Eq. (7), and decays otherwise.
    if kvec[1] == 0.0:
        growth = np.abs(np.linalg.eigvals(M)).max()
        spinodal = 0.5 * (1 / rbar[0] + 1 / rbar[1])
        assert (growth > 1.0) == (-G > spinodal)
