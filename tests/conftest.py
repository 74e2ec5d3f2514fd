import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    if not os.path.exists(oracle.LIB):
        oracle.build(force=False)
    return oracle


@pytest.fixture(scope="session")
def ssp2000():
    return synth.ssp_grid(2000)


@pytest.fixture(scope="session")
def filt6():
    return synth.filters()


@pytest.fixture(scope="session")
def orc(oracle_mod, ssp2000, filt6):
    o = oracle_mod.Oracle(ssp2000, filt6)
    o.build_ztable(64, 0.1, 3.0)
    return o


@pytest.fixture(scope="session")
def ssp_small():
    """Reduced wavelength sampling for quick CPU checks (same grid shape otherwise)."""
    return synth.ssp_grid(400)


@pytest.fixture(scope="session")
def orc_small(oracle_mod, ssp_small, filt6):
    o = oracle_mod.Oracle(ssp_small, filt6)
    o.build_ztable(64, 0.1, 3.0)
    return o


def rng(seed=0):
    return np.random.default_rng(seed)
