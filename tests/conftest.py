import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (run with -m gpu)")
    config.addinivalue_line("markers", "slow: longer CPU run (still part of the default suite)")


@pytest.fixture(scope="session")
def ora():
    from oracle import oracle as o
    o.build(force=False)
    return o


@pytest.fixture(scope="session")
def droplet_reference(ora):
    """Config 1: 32^3 periodic, sphere R = 8 of A (1, 0.03) in B (mirror),
    tau = 1, G = -4.2 (the configuration's G = 1.4 in unit-second-moment
    weights), 500 steps; oracle moments at 10 and 500 steps."""
    from paper_1711_03254_amd import inputs
    shape = (32, 32, 32)
    rA, rB = inputs.droplet(shape, 8.0, center=(16.0, 16.0, 16.0))
    p = ora.Params(32, 32, 32, tau=(1.0, 1.0), G=-4.2)
    f = ora.init(p, rA, rB)
    f10 = ora.run(p, f, 10)
    f500 = ora.run(p, f10, 490)
    return rA, rB, p, {10: ora.moments(p, f10), 500: ora.moments(p, f500)}, (ora.reduce(p, f), ora.reduce(p, f500))


