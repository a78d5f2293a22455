"""GPU parity of the LDS-staged x tiles of the slice kernel (k_cheb_lt).

Operators held in slices only: the 7-point box under PP_SLICED (every tile
staged), and the same box with the rows of its last tile coupled to columns
spread over the whole matrix (that tile touches more than 6144 values of x
and gathers from memory while the others stage).  The staged kernel sums in
the order of the plain one: pp_apply with the tiles and without them
(PP_OPT_LDS_TILES = 0) agree bit for bit, and both match the oracle to 1e-12;
PCG at equal iteration counts within 1e-10.
"""
import numpy as np
import pytest

import oracle as O
from paper_2208_01339_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2208_01339_amd import binding

    binding.lib()
    return binding


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def wide_last_tile(N=40):
    """Heterogeneous 7-point box plus symmetric couplings -0.1 between row n-1024+i and
    column 30 i (i < 1024), each coupled row's diagonal raised by 0.1 (SPD by dominance)."""
    import scipy.sparse as sp

    a = W.hetero_diffusion(N, 1.0, 2)
    n = a.n_rows
    A = a.to_scipy().tolil()
    for i in range(1024):
        r, c = n - 1024 + i, 30 * i
        if r == c:
            continue
        A[r, c] = A[r, c] - 0.1
        A[c, r] = A[c, r] - 0.1
        A[r, r] = A[r, r] + 0.1
        A[c, c] = A[c, c] + 0.1
    A = sp.csr_matrix(A)
    A.sort_indices()
    return W.CSR(n, n, A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data.astype(np.float64))


CASES = {"box40_sliced": lambda: W.hetero_diffusion(40, 2.0, 1), "wide_last_tile": wide_last_tile}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("jacobi", [True, False])
def test_lds_tiles_parity(B, name, jacobi):
    a = CASES[name]()
    n = a.n_rows
    fl = (B.PP_JACOBI if jacobi else 0) | B.PP_SLICED
    op = B.Operator(a=a, flags=fl)
    st = B.pp_get_stats(op.handle)
    assert st["lds_tiles"] == 1 and st["diagonals"] == 0
    orc = O.Operator(a, jacobi=jacobi)
    lmin, lmax = O.lanczos_bounds(orc, 20)
    r = W.rhs_uniform(n, 3)
    outs = []
    for k in (1, 2, 9):
        B.pp_setup(op.handle, k, lmin, lmax, 1e-3)
        z = torch.empty(n, dtype=torch.float64, device="cuda")
        for use in (1, 0):
            B.pp_set_option(op.handle, B.PP_OPT_LDS_TILES, use)
            B.pp_apply(op.handle, dev(r), z)
            outs.append(host(z))
        assert np.array_equal(outs[-2], outs[-1]), k  # staged and plain: bit for bit
        ref = O.cheb_apply(orc, k, lmin, lmax, 1e-3, r)
        assert np.linalg.norm(outs[-1] - ref) <= 1e-12 * np.linalg.norm(ref)
    B.pp_set_option(op.handle, B.PP_OPT_LDS_TILES, 1)
    B.pp_set_option(op.handle, B.PP_OPT_DRIVER, 0)  # the staged kernel runs in the stream-driven solve
    b = W.rhs_uniform(n, 1)
    xo, sto = O.pcg(orc, 9, lmin, lmax, 1e-3, b, tol=1e-8, maxit=3000)
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    s, it, _ = B.pcg_solve(op.handle, dev(b), x, 1e-8, 3000)
    assert s == B.PP_OK and abs(it - sto["iters"]) <= 2
    x.zero_()
    B.pcg_solve(op.handle, dev(b), x, 0.0, sto["iters"])
    assert np.linalg.norm(host(x) - xo) <= 1e-10 * np.linalg.norm(xo)
    op.close()


def test_lds_tiles_off_for_scattered_lanes(B):
    """A renumbered irregular operator: its lanes read scattered columns, so create
    plans no tiles (measured slower there)."""
    op = B.Operator(a=W.irregular_fe(24, seed=3), flags=B.PP_JACOBI)
    st = B.pp_get_stats(op.handle)
    assert st["reordered"] == 1 and st["lds_tiles"] == 0
    op.close()
