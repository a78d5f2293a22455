"""GPU checks of the operator storage: symmetric stored diagonals, the sliced
remainder, and every case that must fall back to the sliced layout.

Each case is a small CSR matrix built on the host; the operator application
through the C ABI is compared row by row with the oracle's CSR product
(|y - y_ref| <= 8 eps sum_j |a_ij x_j|), and the storage the library chose is
checked against what the selection rule gives for that matrix.
"""
import numpy as np
import pytest

import oracle as O
from paper_2208_01339_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2208_01339_amd import binding

    binding.lib()
    return binding


def from_coo(n, rows, cols, vals, sort=True):
    """CSR from triplets, keeping duplicates (entries of one row in column order when sort)."""
    rows, cols, vals = np.asarray(rows), np.asarray(cols), np.asarray(vals, dtype=np.float64)
    order = np.lexsort((cols, rows)) if sort else np.argsort(rows, kind="stable")
    rows, cols, vals = rows[order], cols[order], vals[order]
    rp = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rp, rows + 1, 1)
    rp = np.cumsum(rp)
    return W.CSR(n, n, rp, cols.astype(np.int32), vals)


def to_coo(a):
    rows = np.repeat(np.arange(a.n_rows), np.diff(a.rowptr))
    return rows, a.col.astype(np.int64), a.val.copy()


def apply_check(B, a, flags=0):
    op = B.Operator(a=a, flags=flags)
    x = W.rhs_uniform(a.n_rows, 11)
    y = torch.empty(a.n_rows, dtype=torch.float64, device="cuda")
    B.pp_operator_apply(op.handle, torch.from_numpy(x).cuda(), y)
    torch.cuda.synchronize()
    got = y.cpu().numpy()
    ref = O.csr_matvec(a, x)
    bound = abs(a.to_scipy()) @ np.abs(x)
    tol = 8 * EPS * bound + 1e-300
    assert np.all(np.abs(got - ref) <= tol), np.max(np.abs(got - ref) / tol)
    st = B.pp_get_stats(op.handle)
    op.close()
    return st


def test_stencil_uses_diagonals(B):
    st = apply_check(B, W.poisson3d(11))
    assert st["diagonals"] == 4 and st["nnz_stored"] == 0


def test_asymmetric_value_falls_back(B):
    r, c, v = to_coo(W.poisson3d(9))
    k = np.nonzero((c == r + 9) & (r == 40))[0][0]
    v[k] = -1.0000000000000002  # one ulp away from its mirror
    st = apply_check(B, from_coo(729, r, c, v))
    assert st["diagonals"] == 0


def _split(r, c, v, i, j):
    """Split a_ij into two entries of the same column (CSR sums duplicates)."""
    k = np.nonzero((r == i) & (c == j))[0][0]
    r, c, v = np.append(r, i), np.append(c, j), np.append(v, 0.25)
    v[k] -= 0.25
    return r, c, v


def test_duplicate_entries_fall_back(B):
    r, c, v = to_coo(W.poisson3d(8))
    # both mirrors duplicated: the offset counts stay paired, the fill finds the duplicates
    r, c, v = _split(*_split(r, c, v, 100, 101), 101, 100)
    st = apply_check(B, from_coo(512, r, c, v))
    assert st["diagonals"] == 0


def test_one_sided_duplicate_unpairs_offset(B):
    r, c, v = to_coo(W.poisson3d(8))
    # one extra entry at offset +1 only: offset 1 leaves the stored set
    st = apply_check(B, from_coo(512, *_split(r, c, v, 100, 101)))
    assert st["diagonals"] == 3 and st["nnz_stored"] > 0


def test_many_offsets_falls_back(B):
    rng = np.random.default_rng(5)
    n = 4000
    i = rng.integers(0, n, 6000)
    j = rng.integers(0, n, 6000)
    keep = i != j
    i, j = i[keep], j[keep]
    w = -rng.uniform(0.1, 1.0, len(i))
    rows = np.concatenate([i, j, np.arange(n)])
    cols = np.concatenate([j, i, np.arange(n)])
    vals = np.concatenate([w, w, np.full(n, 20.0)])
    st = apply_check(B, from_coo(n, rows, cols, vals))
    assert st["diagonals"] == 0


def test_hybrid_remainder(B):
    """A stencil plus a few symmetric long-range couplings: the stencil offsets
    are stored diagonals, the couplings go to the sliced remainder."""
    a = W.poisson3d(12)
    r, c, v = to_coo(a)
    rng = np.random.default_rng(8)
    i = rng.integers(0, 1728, 40)
    j = (i + rng.integers(500, 1200, 40)) % 1728
    keep = np.abs(i - j) > 200
    i, j = i[keep], j[keep]
    w = -0.01 * np.ones(len(i))
    h = from_coo(1728, np.concatenate([r, i, j]), np.concatenate([c, j, i]), np.concatenate([v, w, w]))
    # merge possible duplicates of the random pairs into single entries
    S = h.to_scipy().tocsr()
    S.sum_duplicates()
    S.sort_indices()
    h = W.CSR(1728, 1728, S.indptr.astype(np.int64), S.indices.astype(np.int32), S.data)
    st = apply_check(B, h)
    assert st["diagonals"] == 4 and st["nnz_stored"] > 0
    # and the solve through both storages matches the oracle
    orc = O.Operator(h, jacobi=True)
    lmin, lmax = O.lanczos_bounds(orc, 20)
    b = W.rhs_uniform(1728, 3)
    xo, sto = O.pcg(orc, 6, lmin, lmax, 0.0, b, tol=0.0, maxit=8)
    op = B.Operator(a=h, flags=B.PP_JACOBI)
    B.pp_setup(op.handle, 6, lmin, lmax, 0.0)
    x = torch.zeros(1728, dtype=torch.float64, device="cuda")
    B.pcg_solve(op.handle, torch.from_numpy(b).cuda(), x, 0.0, 8)
    torch.cuda.synchronize()
    assert np.linalg.norm(x.cpu().numpy() - xo) <= 1e-10 * np.linalg.norm(xo)
    op.close()


def test_unpaired_offset_goes_to_remainder(B):
    """An entry above the diagonal without a mirror makes its offset unpaired:
    that offset leaves the stored set (its entries go to the slice part)."""
    r, c, v = to_coo(W.poisson3d(10))
    # row 9 ends an x-line: (9, 10) is not a stencil neighbour
    h = from_coo(1000, np.append(r, 9), np.append(c, 10), np.append(v, -0.5))
    st = apply_check(B, h)
    assert st["diagonals"] == 3 and st["nnz_stored"] > 0


def test_explicit_zero_without_mirror(B):
    """An explicit zero above the diagonal with no mirror is symmetric in value."""
    r, c, v = to_coo(W.poisson3d(10))
    h = from_coo(1000, np.append(r, 9), np.append(c, 10), np.append(v, 0.0))
    st = apply_check(B, h)
    assert st["diagonals"] == 4 and st["nnz_stored"] == 0


def test_unsorted_rows(B):
    """Column order inside a row does not matter to either storage."""
    r, c, v = to_coo(W.hetero_diffusion(9, 1.0, 3))
    perm = np.random.default_rng(1).permutation(len(r))
    h = from_coo(729, r[perm], c[perm], v[perm], sort=False)
    st = apply_check(B, h)
    assert st["diagonals"] == 4
    assert apply_check(B, h, B.PP_SLICED)["diagonals"] == 0


def test_tiny_and_single_row(B):
    # n = 1 and a 2 x 2 system: offsets beyond the matrix end
    apply_check(B, W.CSR(1, 1, np.array([0, 1], dtype=np.int64), np.array([0], dtype=np.int32),
                         np.array([3.0])))
    st = apply_check(B, from_coo(2, [0, 0, 1, 1], [0, 1, 0, 1], [2.0, -1.0, -1.0, 2.0]))
    assert st["diagonals"] == 2
