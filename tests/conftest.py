import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# a planted oracle mistake, for the child runs of tests/test_oracle_mutations.py
if os.environ.get("HC_ORACLE_MUTANT"):
    from tests.oracle_mutants import install
    install(os.environ["HC_ORACLE_MUTANT"])


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: takes more than a few seconds")


def xyz_close(got, ref, rel=2e-5, floor=1e-7):
    """Per-component |got - ref| <= rel * |ref| + floor; returns the worst
    ratio of error to allowance (<= 1 passes)."""
    import numpy as np
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    allow = rel * np.abs(ref) + floor
    return float((np.abs(got - ref) / allow).max()) if ref.size else 0.0


@pytest.fixture
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")
