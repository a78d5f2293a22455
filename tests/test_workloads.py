"""Invariants of the seeded input generators (no method arithmetic involved)."""
import numpy as np

from paper_2208_01339_amd import workloads as W


def test_hetero_sigma0_is_poisson():
    a = W.poisson3d(9)
    b = W.hetero_diffusion(9, 0.0, 123)
    assert np.array_equal(a.rowptr, b.rowptr)
    assert np.array_equal(a.col, b.col)
    assert np.array_equal(a.val, b.val)


def test_poisson32_shape():
    a, b = W.config_poisson32()
    assert a.n_rows == 32768 and a.nnz == 223232
    assert b.shape == (32768,) and b.min() >= -1 and b.max() < 1
    assert np.array_equal(b, np.random.default_rng(0).uniform(-1, 1, 32768))


def test_hetero_symmetric_spd_and_sorted():
    a = W.hetero_diffusion(7, 2.0, 5)
    S = a.to_scipy()
    assert abs(S - S.T).max() == 0
    assert np.linalg.eigvalsh(S.toarray()).min() > 0
    for i in range(a.n_rows):
        c = a.col[a.rowptr[i]:a.rowptr[i + 1]]
        assert np.all(np.diff(c) > 0)
    # M-matrix: off-diagonals negative, rows weakly diagonally dominant
    d = S.diagonal()
    off = np.asarray(abs(S).sum(axis=1)).ravel() - d
    assert np.all(d >= off - 1e-12)


def test_hetero_nnz_formula():
    for N in (4, 7, 10):
        a = W.hetero_diffusion(N, 1.0, 0)
        assert a.nnz == N ** 3 + 6 * N * N * (N - 1)


def test_dfn_shapes():
    s = W.dfn_schur(n_frac=30, G=16, n_traces=60, L_lo=3, L_hi=12, sigma=1.5, seed=0)
    assert s.n == 30 * 256
    assert s.a.nnz == 30 * (256 * 5 - 4 * 16)
    assert s.c.nnz == 2 * s.nt
    assert 60 * 3 <= s.nt <= 60 * 12
    assert np.all(s.m >= 0.5) and np.all(s.m <= 2.0)
    # C rows: +1 and -1 on cells of two different fractures
    c = s.c.col.reshape(-1, 2)
    v = s.c.val.reshape(-1, 2)
    assert np.all(c[:, 0] < c[:, 1])
    assert np.all(v.sum(axis=1) == 0) and np.all(np.abs(v) == 1)
    assert np.all(c[:, 0] // 256 != c[:, 1] // 256)
    # block diagonal A_ff: no entry leaves its fracture
    rows = np.repeat(np.arange(s.n), np.diff(s.a.rowptr))
    assert np.all(rows // 256 == s.a.col // 256)


def test_dfn_full_size_counts():
    s = W.dfn_schur()
    assert s.n == 8_192_000 and s.a.nnz == 40_448_000
    assert 150_000 < s.nt < 200_000
    # spanning tree: every fracture touched by some trace
    touched = np.unique(s.c.col // 4096)
    assert touched.size == 2000


def test_batch_sizes():
    sides = W.batch_sizes()
    assert sides.size == 256 and sides.min() >= 21 and sides.max() <= 126


def test_dfn_su_structure():
    """Blocks of the DFN system: A and G^h fracture-local within distance G of
    the diagonal, C columns inside their owner fracture, B = C + E with E on the
    other side of the trace, G^u pairing the two sides; deterministic per seed."""
    P = W.dfn_su(n_frac=7, G=9, n_traces=12, L_lo=2, L_hi=9, seed=2)
    nf = P.grid ** 2
    for M in (P.a, P.gh):
        S = M.to_scipy().tocoo()
        assert np.all(S.row // nf == S.col // nf)
        assert np.all(np.abs(S.row - S.col) <= P.grid)
        D = M.to_scipy().toarray()
        assert np.array_equal(D, D.T)
    own = np.searchsorted(P.u_off, np.arange(P.n_u), side="right") - 1
    Cc = P.c.to_scipy().tocoo()
    assert np.all(Cc.row // nf == own[Cc.col]) and Cc.nnz == P.n_u
    E = (P.b.to_scipy() - P.c.to_scipy()).tocoo()
    E.eliminate_zeros()
    assert E.nnz == P.n_u and np.all(E.row // nf != own[E.col]) and np.all(E.data == -1.0)
    Gu = P.gu.to_scipy().toarray()
    assert np.array_equal(Gu, Gu.T) and np.all(Gu.sum(axis=1) == 2 * 10.0)
    Q = W.dfn_su(n_frac=7, G=9, n_traces=12, L_lo=2, L_hi=9, seed=2)
    assert np.array_equal(P.b.val, Q.b.val) and np.array_equal(P.a.val, Q.a.val)
