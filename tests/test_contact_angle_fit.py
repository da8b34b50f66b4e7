"""Host-side pieces of the contact-angle calibration: interface location,
circle fit and the angle at the wall plane, on synthetic fields."""
import numpy as np
import pytest

from paper_1711_03254_amd import contact_angle as ca


def synthetic(xc, yc, r, nx=160, ny=80):
    y, x = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    d = np.sqrt((x - xc) ** 2 + (y - yc) ** 2)
    phi = np.tanh((r - d) / 2.0)          # +1 inside, -1 outside
    ra = (1 + phi)[None] / 2
    rb = (1 - phi)[None] / 2
    solid = np.zeros((1, ny, nx), np.uint8)
    solid[:, 0, :] = 1
    return ra, rb, solid


def test_circle_fit_recovers_a_known_circle():
    ra, rb, solid = synthetic(80.3, 10.7, 20.2)
    pts = ca.interface_points(ra, rb, solid)
    xc, yc, r = ca.fit_circle(pts)
    assert abs(xc - 80.3) < 0.05 and abs(yc - 10.7) < 0.05 and abs(r - 20.2) < 0.05


def test_angle_at_the_wall_plane():
    assert abs(ca.angle_from_circle(0.5, 10.0) - 90.0) < 1e-12          # centre on the wall: half disc
    assert abs(ca.angle_from_circle(0.5 + 5.0, 10.0) - 120.0) < 1e-9    # sin(30 deg) above: 90 + 30
    assert abs(ca.angle_from_circle(0.5 - 5.0, 10.0) - 60.0) < 1e-9
    # a circle centred far above the wall touches it only at 180 degrees
    assert ca.angle_from_circle(100.0, 10.0) == 180.0


def test_inverse_interpolates_between_bracketing_rows():
    table = [{"rho_s": -0.3, "theta_deg": 55.0}, {"rho_s": -0.2, "theta_deg": 65.0},
             {"rho_s": 0.0, "theta_deg": float("nan")}, {"rho_s": 0.2, "theta_deg": 115.0}]
    assert abs(ca.rho_s_for(60.0, table) - (-0.25)) < 1e-12
    assert abs(ca.rho_s_for(65.0, table) - (-0.2)) < 1e-12
    assert abs(ca.rho_s_for(90.0, table) - 0.0) < 1e-12       # across the gap left by the unfitted row
    with pytest.raises(ValueError):
        ca.rho_s_for(150.0, table)
    with pytest.raises(ValueError):
        ca.rho_s_for(60.0, [{"rho_s": 0.1, "theta_deg": 70.0}, {"rho_s": 0.2, "theta_deg": 50.0}])
