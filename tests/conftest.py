import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device)")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


@pytest.fixture(scope="session")
def cfg0_hier():
    import workloads as W
    from oracle.hierarchy import Hierarchy
    c = W.make_config(0)
    return c, Hierarchy(c["coords"], c["elems"], c["kappa"], check_literal=True)


@pytest.fixture(scope="session")
def graded_small():
    import workloads as W
    from oracle.hierarchy import Hierarchy
    c = W.make_config(1, scale=0.004)
    return c, Hierarchy(c["coords"], c["elems"], c["kappa"], check_literal=True)
