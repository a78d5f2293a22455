"""Pins of the oracle's spectral low-rank correction (section 3.1):
P = p_k(A) + V (V^T A V)^{-1} V^T.

Each test compares with a closed form (eq. plusone on exact eigenvectors of a
diagonal matrix), a dense assembly of the correction with numpy, the
dot-product counts of Table tab11's rank-one rows, or a closed-form
eigenvector (Ritz vectors of a Poisson matrix).
"""
import numpy as np
import pytest

import oracle as O
from paper_2208_01339_amd import workloads as W
from conftest import DiagCSR, read_table
from test_oracle_pins import poly_closed_form


@pytest.mark.parametrize("k,xi", [(0, 0.0), (3, 0.0), (10, 1e-3), (20, 1e-2)])
def test_plusone_on_exact_eigenvectors(k, xi):
    """eq. plusone: P A v_j = (1 + lambda_j p_k(lambda_j)) v_j for the p vectors in V, and
    lambda_j p_k(lambda_j) v_j for the others (V orthogonal to them)."""
    lam = np.linspace(0.01, 2.0, 200)
    op = O.Operator(DiagCSR(lam))
    lmin, lmax, p = 0.05, 2.0, 3
    V = np.eye(lam.size)[:, :p]
    hinv = O.lowrank_setup(op, V)
    assert np.allclose(hinv, np.diag(1.0 / lam[:p]), rtol=1e-14)
    pk = poly_closed_form(k, lmin, lmax, xi, lam)
    for j in (0, 1, 2, 3, 57, 199):
        e = np.zeros(lam.size)
        e[j] = lam[j]  # A e_j
        z = O.lowrank_apply_hat(op, k, lmin, lmax, xi, V, hinv, e)
        want = lam[j] * pk[j] + (1.0 if j < p else 0.0)
        assert z[j] == pytest.approx(want, rel=1e-10)
        assert np.max(np.abs(np.delete(z, j))) <= 1e-13


def test_correction_matches_dense_assembly():
    a = W.hetero_diffusion(4, 1.5, 2)
    op = O.Operator(a, jacobi=True)
    n = a.n_rows
    A = a.to_scipy().toarray()
    d = np.diag(A)
    Ah = A / np.sqrt(np.outer(d, d))
    rng = np.random.default_rng(3)
    V = rng.normal(size=(n, 3))
    lmin, lmax = O.lanczos_bounds(op, 20)
    r = rng.normal(size=n)
    k, xi = 5, 1e-3
    z = O.lowrank_apply_hat(op, k, lmin, lmax, xi, V, O.lowrank_setup(op, V), r)
    corr = V @ np.linalg.solve(V.T @ Ah @ V, V.T @ r)
    z0 = O.cheb_apply_hat(op, k, lmin, lmax, xi, r)
    assert np.allclose(z, z0 + corr, rtol=1e-11, atol=1e-13)


def test_counts_of_tab11_rank_one_rows():
    """Rank-one update: MVP = iters (m + 1) as without it, ddot = 4 iters (Table tab11)."""
    rows = read_table("tab11_rank_one.txt")
    assert len(rows) == 7
    for r in rows:
        m, it1, mvp1, dd1 = (int(v) for v in r[:4])
        assert mvp1 == it1 * (m + 1)
        if not (m == 0 and dd1 == 4900):  # printed 4900 for 4 x 1235 = 4940
            assert dd1 == 4 * it1
    a = W.hetero_diffusion(10, 2.0, 1)
    op = O.Operator(a, jacobi=True)
    lmin, lmax = O.lanczos_bounds(op, 20)
    b = W.rhs_uniform(a.n_rows, 2)
    for p in (1, 3):
        _, V = O.ritz_vectors(op, 40, p)
        for k in (0, 1, 7):
            _, st = O.pcg_lowrank(op, k, lmin, lmax, 1e-3, V, b, tol=1e-8, maxit=2000)
            assert st["status"] == O.OK
            assert st["n_apply"] == st["iters"] * (k + 1)
            assert st["n_dot"] == (3 + p) * st["iters"]


def test_ritz_vector_of_poisson_matches_closed_form():
    """Smallest eigenpair of the 3-D Dirichlet Laplacian: 3 (2 - 2 cos(pi/(N+1))),
    eigenvector sin(pi i/(N+1)) sin(pi j/(N+1)) sin(pi k/(N+1))."""
    N = 5
    op = O.Operator(W.poisson3d(N))
    th, V = O.ritz_vectors(op, 60, 1)
    lam1 = 3.0 * (2.0 - 2.0 * np.cos(np.pi / (N + 1)))
    assert th[0] == pytest.approx(lam1, rel=1e-10)
    s = np.sin(np.pi * np.arange(1, N + 1) / (N + 1))
    u = np.einsum("k,j,i->kji", s, s, s).ravel()  # row index i + N (j + N k)
    v = V[:, 0]
    cos = abs(u @ v) / (np.linalg.norm(u) * np.linalg.norm(v))
    assert cos >= 1.0 - 1e-10


def test_lowrank_pcg_solves_and_zero_rank_is_plain():
    a = W.hetero_diffusion(8, 2.0, 4)
    op = O.Operator(a, jacobi=True)
    lmin, lmax = O.lanczos_bounds(op, 20)
    b = W.rhs_uniform(a.n_rows, 5)
    _, V = O.ritz_vectors(op, 40, 2)
    x, st = O.pcg_lowrank(op, 6, lmin, lmax, 1e-3, V, b, tol=1e-10, maxit=500)
    assert st["status"] == O.OK
    # true residual of the scaled system (the tolerance applies to it)
    rh = op.dis * (b - op.apply_raw(x))
    assert np.linalg.norm(rh) <= 2e-10 * np.linalg.norm(op.dis * b)
    # rank 0 follows the plain loop exactly
    x0, st0 = O.pcg(op, 6, lmin, lmax, 1e-3, b, tol=1e-10, maxit=500)
    x1, st1 = O.pcg_lowrank(op, 6, lmin, lmax, 1e-3, np.zeros((a.n_rows, 0)), b, tol=1e-10, maxit=500,
                            hinv=np.zeros((0, 0)))
    assert st1["iters"] == st0["iters"] and np.array_equal(x0, x1)


def test_poly_ritz_on_diagonal_matrix():
    """Lanczos on p_k(D) for D with three isolated small eigenvalues below the
    polynomial's interval: p_k maps them to its largest values, so the Ritz
    vectors are the unit vectors of those rows, in order, and the Rayleigh
    quotients are the eigenvalues themselves."""
    d = np.concatenate([[0.01, 0.03, 0.2], np.linspace(1.0, 10.0, 197)])
    op = O.Operator(DiagCSR(d))
    theta, V = O.poly_ritz_vectors(op, 10, 1.0, 10.0, 0.0, 30, 3)
    assert np.allclose(theta, d[:3], rtol=1e-10)
    for c in range(3):
        assert abs(abs(V[c, c]) / np.linalg.norm(V[:, c]) - 1.0) < 1e-10


def test_poly_ritz_matches_dense_eigenvectors():
    """On a small Jacobi-scaled heterogeneous operator the p Ritz vectors from 30
    steps on p_k(A-hat) are the eigenvectors of the p smallest eigenvalues of
    A-hat (dense eigh): Rayleigh quotients to 1e-8, residuals below 1e-4."""
    a = W.hetero_diffusion(8, 2.0, 3)
    op = O.Operator(a, jacobi=True)
    lmin, lmax = O.lanczos_bounds(op, 20)
    theta, V = O.poly_ritz_vectors(op, 20, lmin, lmax, 0.0, 30, 3)
    A = a.to_scipy().toarray()
    dis = 1.0 / np.sqrt(np.diag(A))
    lam = np.linalg.eigvalsh(A * np.outer(dis, dis))
    assert np.allclose(theta, lam[:3], rtol=1e-8)
    for c in range(3):
        v = V[:, c]
        res = np.linalg.norm(op.apply(v) - theta[c] * v) / (abs(theta[c]) * np.linalg.norm(v))
        assert res < 1e-4, (c, res)
