import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built library")
    config.addinivalue_line("markers", "slow: longer CPU test")


@pytest.fixture(scope="session")
def mech_h2():
    import chemgen
    return chemgen.make_mechanism("h2")


@pytest.fixture(scope="session")
def mech_ch4():
    import chemgen
    return chemgen.make_mechanism("ch4")


@pytest.fixture(scope="session")
def om_h2(mech_h2):
    import oracle
    return oracle.OracleMech(mech_h2)


@pytest.fixture(scope="session")
def om_ch4(mech_ch4):
    import oracle
    return oracle.OracleMech(mech_ch4)


def state_vector(T, Y, i):
    return np.concatenate([[T[i]], Y[:, i]])
