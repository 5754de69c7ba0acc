import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: oracle runs of a minute or more")


@pytest.fixture(scope="session")
def sphere32():
    """Oracle hierarchy of the 32^3 sphere workload (box minus the sphere r = 0.25,
    Dirichlet, sin 2 pi x sin 2 pi y sin 2 pi z), shared by the oracle tests."""
    from oracle.fields import Field
    from oracle.multigrid import Hierarchy
    from paper_2410_05865_amd import inputs
    dom, phi = inputs.sphere_workload(32)
    return Hierarchy(dom), Field(phi)
