import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


@pytest.fixture(scope="session")
def jitter4():
    """Jittered 4^3 Kuhn cube (384 tets), its complex and operators."""
    import qh_inputs as qi
    from oracle.complex_ import Complex
    from oracle.whitney import Operators
    m = qi.make_mesh(qi.CONFIGS["jitter4"])
    cx = Complex(m.xyz, m.tets)
    op = Operators(cx, qi.EPS0, qi.MU0)
    return m, cx, op
