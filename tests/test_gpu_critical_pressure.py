"""Critical pressure of a wetting slug in a constriction against Eq. (12)
(needs an MI355X: -m gpu).

The protocol of Section 3.6 runs on the solver: a slug of the second
component over the exit of a narrow part (D = 10) of a periodic channel
(H = 40, L = 160, Z = 52), body forces stepped through -30 ... +30 % of
g_crit = 2 sigma cos(theta) (1/D - 1/H) / (rho_0 L), 80 000 steps per stage.
sigma is measured from the Laplace law of static droplets and theta (inside
the second component) from the contact-angle calibration, both with the
same solver and physics (G = -4.2, tau = 1).  The paper finds the slug
pushed out of the narrow part within 10 % of g_crit; so must we: still
inside at -10 %, out by +10 %, at three wall potentials (theta about 55,
46 and 38 degrees).
"""
import json
import os

import pytest

pytestmark = pytest.mark.gpu


def test_slug_leaves_the_constriction_within_ten_percent_of_eq12():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1711_03254_amd import contact_angle as ca, critical_pressure as cp, lbm
    lbm.load_library()
    sigma, _, r2 = cp.surface_tension(G=-4.2, tau=1.0)
    assert r2 >= 0.999 and sigma > 0
    rows = []
    for rho_s in (0.3, 0.4, 0.5):
        theta2 = 180.0 - ca.measure(rho_s, steps=20000)["theta_deg"]
        assert theta2 < 90.0        # the wall wets the slug
        r = cp.ramp(sigma, theta2, D=10, rho_s=rho_s)
        at = {row["stage"]: row["slug_x"] for row in r["stages"]}
        rows.append({"rho_s": rho_s, "theta2": theta2, "g_crit": r["g_crit"], "slug_x": at,
                     "transition": cp.transition(r)})
        assert at[-0.10] < r["exit_x"], (rho_s, at)
        assert at[0.10] >= r["exit_x"], (rho_s, at)
    path = os.environ.get("PARITY_LOG")
    if path:
        with open(path, "a") as fh:
            fh.write(json.dumps({"test": "critical_pressure", "sigma": sigma, "cases": rows}) + "\n")
