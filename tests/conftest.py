import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an AMD GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def mesh_4():
    from afe_inputs.mesh import jittered_lattice_seeds, periodic_voronoi
    return periodic_voronoi(jittered_lattice_seeds(4, 0.2, 0))


@pytest.fixture(scope="session")
def mesh_3():
    from afe_inputs.mesh import jittered_lattice_seeds, periodic_voronoi
    return periodic_voronoi(jittered_lattice_seeds(3, 0.2, 0))
