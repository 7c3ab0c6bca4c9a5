import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")


def load_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append(line.split())
    return rows


@pytest.fixture(scope="session")
def oracle():
    from oracle import oracle as O
    O.lib()
    return O


@pytest.fixture(scope="session")
def c1_market(oracle):
    """Config-1 caplet market completed with oracle model vols + noise."""
    from paper_2408_01470_amd import inputs as I
    m, truth, noise = I.caplet_market()
    mv, _, _, ok = oracle.model_values(m, 0, truth[0])
    assert ok
    return I.complete_market(m, mv, noise), truth


def complete_with_oracle(oracle, m, truth, noise):
    """Market vols = oracle model vols (vol mode) at the true parameters + noise."""
    from paper_2408_01470_amd import inputs as I
    vm = I.as_vol_market(m)
    M = oracle.Market(vm)
    vols = []
    for i in range(M.n_inst):
        mv, _, _, ok = oracle.model_values(M, i, truth[i])
        assert ok, f"true parameters of instance {i} outside the model domain"
        vols.append(mv)
    return I.complete_market(m, np.concatenate(vols), noise)


@pytest.fixture(scope="session")
def c2_market(oracle):
    from paper_2408_01470_amd import inputs as I
    m, truth, noise = I.lmm_market()
    return complete_with_oracle(oracle, m, truth, noise), truth
