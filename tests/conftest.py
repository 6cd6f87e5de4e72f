import os
import sys

import pytest

try:   # imported at collection so that its first (slow) load is not charged to a test
    import torch  # noqa: F401
except Exception:  # noqa: BLE001
    torch = None

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C-ABI library)")
    config.addinivalue_line("markers", "slow: longer CPU test")


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    oracle.lib()
    return oracle


@pytest.fixture(scope="session")
def tiny(oracle_mod):
    import workloads
    c = workloads.tiny_code()
    return c, oracle_mod.OCode(c)


@pytest.fixture(scope="session")
def code1(oracle_mod):
    import workloads
    c = workloads.table5_code1()
    return c, oracle_mod.OCode(c)


@pytest.fixture(scope="session")
def tiny_search(oracle_mod, tiny):
    """Oracle impulse search on the tiny code: singles + pairs within distance 4,
    OMS int8, 20 iterations, 3 dB, grid k/16 up to 32, a_max 6."""
    c, oc = tiny
    pats = oracle_mod.pattern_list(oc, [oracle_mod.PAT_SINGLES, oracle_mod.PAT_PAIRS])
    res = oracle_mod.search(oc, pats, a_max=6)
    return pats, res
