import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


def read_table(name):
    """Whitespace table from tests/golden, '#' comments skipped; returns list of rows (strings)."""
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append(line.split())
    return rows


class DiagCSR:
    """CSR view of a diagonal matrix."""

    def __init__(self, d):
        d = np.asarray(d, dtype=np.float64)
        n = d.size
        self.rowptr = np.arange(n + 1, dtype=np.int64)
        self.col = np.arange(n, dtype=np.int32)
        self.val = d.copy()
        self.n_rows = n


class DenseCSR:
    """CSR view of a dense matrix (all stored entries nonzero)."""

    def __init__(self, a):
        import scipy.sparse as sp

        s = sp.csr_matrix(np.asarray(a, dtype=np.float64))
        s.sort_indices()
        self.rowptr = s.indptr.astype(np.int64)
        self.col = s.indices.astype(np.int32)
        self.val = s.data.astype(np.float64)
        self.n_rows = s.shape[0]


@pytest.fixture
def diag_csr():
    return DiagCSR


@pytest.fixture
def dense_csr():
    return DenseCSR
