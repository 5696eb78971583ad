import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: full-size case (minutes on the CPU)")


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def fig1_pattern():
    """Lower pattern of the Fig. 1 factor as (n, colptr, rowind), 0-based."""
    import numpy as np
    import scipy.sparse as sp
    rows, cols = [], []
    with open(os.path.join(ROOT, "tests", "golden", "fig1_pattern.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            t = [int(x) for x in line.split()]
            i = t[0] - 1
            rows.append(i)
            cols.append(i)
            for c in t[1:]:
                rows.append(i)
                cols.append(c - 1)
    A = sp.csc_matrix((np.ones(len(rows)), (rows, cols)), shape=(15, 15))
    A.sort_indices()
    return 15, A.indptr.astype(np.int64), A.indices.astype(np.int64)


@pytest.fixture(scope="session")
def fig1_facts():
    facts = {}
    with open(os.path.join(ROOT, "tests", "golden", "fig1_facts.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            t = line.split()
            facts.setdefault(t[0], []).append(t[1:])
    return facts
