"""Host-side pieces of the Eq. (12) protocol: the closed form, the
constricted channel, the slug's initial state and its periodic centre."""
import numpy as np

from paper_1711_03254_amd import critical_pressure as cp


def test_eq12_closed_form():
    # 2 sigma cos(theta) (1/D - 1/H): zero without a constriction or at 90 degrees, linear in sigma
    assert cp.p_crit(0.1, 40.0, 40, 40) == 0.0
    assert abs(cp.p_crit(0.1, 90.0, 10, 40)) < 1e-17
    assert np.isclose(cp.p_crit(0.1, 60.0, 10, 40), 2 * 0.1 * 0.5 * (0.1 - 0.025))
    assert np.isclose(cp.p_crit(0.2, 60.0, 10, 40), 2 * cp.p_crit(0.1, 60.0, 10, 40))
    assert cp.p_crit(0.1, 120.0, 10, 40) < 0    # a non-wetting slug is pulled out, not held


def test_constricted_channel_geometry():
    s = cp.constricted_channel(L=160, Z=52, H=40, D=10, x0=54)
    assert s.shape == (1, 42, 160)
    assert s[0, 0].all() and s[0, 41].all()
    assert (s[0, 1:41, :54] == 0).all() and (s[0, 1:41, 106:] == 0).all()
    open_rows = np.nonzero(s[0, :, 80] == 0)[0]
    assert len(open_rows) == 10 and open_rows[0] == 16 and open_rows[-1] == 25   # centred band of height D
    assert (s[0, 1:41, 54:106].sum(axis=0) == 30).all()


def test_slug_state_and_periodic_centre():
    s = cp.constricted_channel()
    ra, rb = cp.slug_state(s, 78, 109)
    assert (ra[s == 1] == 0).all() and (rb[s == 1] == 0).all()
    fluid = s == 0
    assert np.isclose((rb[fluid] > 0.5).sum(), 28 * 10 + 3 * 40)   # 400 slug sites
    # the centre of a slug that straddles the periodic seam
    ra2, rb2 = cp.slug_state(s, 150, 160)
    _, rb3 = cp.slug_state(s, 0, 10)
    c = cp.slug_position(np.maximum(rb2, rb3), s)
    assert abs((c + 0.5) % 160) < 1e-9          # x = 150 .. 159 and 0 .. 9: centred at -0.5
    # weighted by slug sites per column: 28 columns of 10 (x = 78 .. 105), 3 of 40 (x = 106 .. 108);
    # the circular mean matches the arithmetic one up to the slug's spread relative to the period
    xs = np.r_[np.arange(78, 106).repeat(10), np.arange(106, 109).repeat(40)]
    assert abs(cp.slug_position(rb, s) - xs.mean()) < 0.2
