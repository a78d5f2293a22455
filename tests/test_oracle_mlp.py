"""Pins of the CPU MLP reference: the analytic gradient against central finite
differences, and the features against direct dense computations."""
import numpy as np
import pytest

import oracle as O
from oracle import mlp as M
from paper_2208_01339_amd import workloads as W


@pytest.mark.parametrize("shape", [(4, 6, 2, 3), (16, 32, 3, 3)])
def test_mlp_gradient_finite_differences(shape):
    n_in, hidden, depth, n_out = shape
    shapes = M.layer_shapes(n_in, hidden, depth, n_out)
    rng = np.random.default_rng(0)
    npar = sum(fi * fo + fo for fi, fo in shapes)
    p = rng.normal(0, 0.3, npar)
    X = rng.normal(size=(7, n_in))
    T = rng.normal(size=(7, n_out))
    L, g = M.loss_grad(p, shapes, X, T)
    assert L == pytest.approx(M.loss(p, shapes, X, T), rel=1e-14)
    idx = rng.choice(npar, 40, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros(npar)
        e[i] = h
        fd = (M.loss(p + e, shapes, X, T) - M.loss(p - e, shapes, X, T)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 + 1e-5 * abs(fd)


def test_adam_matches_definition():
    p = np.array([1.0, -2.0])
    g = np.array([0.5, 0.25])
    p1, m1, v1 = M.adam(p, g, np.zeros(2), np.zeros(2), 1, 0.1)
    # first step: mhat = g, vhat = g^2 -> p - lr * sign(g) (up to eps)
    assert np.allclose(p1, p - 0.1 * np.sign(g), atol=1e-6)


def test_features_against_dense():
    a = W.hetero_diffusion(6, 2.0, 3)
    op = O.Operator(a, jacobi=True)
    f = M.features(op, a, power_steps=8)
    A = a.to_scipy().toarray()
    d = np.diag(A)
    Ah = A / np.sqrt(np.outer(d, d))
    lam = np.linalg.eigvalsh(Ah)
    assert f[0] == pytest.approx(np.log10(A.shape[0]))
    assert f[2] == pytest.approx(np.log10(d).mean())
    # Gershgorin bounds enclose the spectrum; Rayleigh quotients are lower bounds of lambda_max
    assert f[6] >= lam[-1] - 1e-12 and f[8] <= lam[0] + 1e-12
    assert f[6] == pytest.approx(np.abs(Ah).sum(axis=1).max())
    assert np.all(f[9:13] <= lam[-1] + 1e-12) and np.all(np.diff(f[9:13]) >= -1e-12)
    # the shifted power estimate is an upper bound of lambda_min (a Rayleigh quotient of c I - A)
    assert f[13] >= lam[0] - 1e-12
    assert f[14] == 7


def test_features_schur_bounds():
    s = W.dfn_schur(n_frac=4, G=6, n_traces=7, L_lo=2, L_hi=5, sigma=1.5, seed=3)
    op = O.Operator(s.a, s.c, s.m, jacobi=True)
    f = M.features(op, s.a, s.c, s.m, power_steps=8)
    A = s.a.to_scipy().toarray()
    Cm = s.c.to_scipy().toarray()
    S = A + Cm.T @ np.diag(1 / s.m) @ Cm
    d = np.diag(S)
    Sh = S / np.sqrt(np.outer(d, d))
    lam = np.linalg.eigvalsh(Sh)
    assert f[6] >= np.abs(Sh).sum(axis=1).max() - 1e-12  # row-sum bound of |S-hat|
    assert f[8] <= lam[0] + 1e-12
    assert np.all(f[9:13] <= lam[-1] + 1e-12)


def _power_rq(lam, Q, v0, t, shift=None):
    """Rayleigh quotient of A^t v0 (or of (c I - A)^t v0 with c = shift), from the
    eigendecomposition A = Q diag(lam) Q^T: sum c_i^2 mu_i^(2t+1) / sum c_i^2 mu_i^(2t)."""
    mu = lam if shift is None else shift - lam
    c2 = (Q.T @ v0) ** 2
    return float((c2 * mu ** (2 * t + 1)).sum() / (c2 * mu ** (2 * t)).sum())


@pytest.mark.parametrize("jacobi", [True, False])
def test_features_closed_forms_csr(jacobi):
    """Every feature of the CSR form against a dense computation written from its
    definition: nnz/n, the log-diagonal statistics (numpy's std, not the
    E[x^2] - E[x]^2 form of the oracle), the mean off-diagonal row sum, the
    minimum diagonal dominance, the power-step Rayleigh quotients and the
    shifted-power estimate from the eigendecomposition (sum c_i^2 l_i^(2t+1) /
    sum c_i^2 l_i^(2t)), and the log condition estimate built from them."""
    a = W.hetero_diffusion(6, 2.0, 5)
    op = O.Operator(a, jacobi=jacobi)
    P = 8
    f = M.features(op, a, power_steps=P)
    A = a.to_scipy().toarray()
    n = A.shape[0]
    d = np.diag(A).copy()
    dis = 1 / np.sqrt(d) if jacobi else np.ones(n)
    Ah = A * np.outer(dis, dis)
    ld = np.log10(d)
    assert f[1] == pytest.approx(np.count_nonzero(A) / n, rel=1e-15)
    assert f[2] == pytest.approx(ld.mean(), rel=1e-13)
    assert f[3] == pytest.approx(np.std(ld), rel=1e-9)
    assert f[4] == pytest.approx(ld.min(), rel=1e-15)
    assert f[5] == pytest.approx(ld.max(), rel=1e-15)
    off = np.abs(Ah).sum(axis=1) - np.abs(np.diag(Ah))
    assert f[6] == pytest.approx(np.abs(Ah).sum(axis=1).max(), rel=1e-13)
    assert f[7] == pytest.approx(off.mean(), rel=1e-13)
    assert f[8] == pytest.approx((np.diag(Ah) - off).min(), rel=1e-12, abs=1e-14)
    lam, Q = np.linalg.eigh(Ah)
    v0 = O.fmix32_start(n)
    for j, t in enumerate([P // 4, P // 2, 3 * P // 4, P]):
        assert f[9 + j] == pytest.approx(_power_rq(lam, Q, v0, t - 1), rel=1e-11)
    lmin_est = f[6] - _power_rq(lam, Q, v0, P - 1, shift=f[6])
    assert f[13] == pytest.approx(lmin_est, rel=1e-9, abs=1e-12)
    assert f[14] == 7
    assert f[15] == pytest.approx(np.log10(_power_rq(lam, Q, v0, P - 1) / abs(lmin_est)), rel=1e-9)


def test_features_closed_forms_schur():
    """The Schur form: nnz/n of A_ff, the diagonal statistics of diag(S), and the
    row sums of |A_ff-hat| + |C-hat|^T M^{-1} |C-hat| (the bound the features use
    for S-hat) against dense matrices, the Rayleigh quotients against the
    eigendecomposition of the assembled S-hat."""
    s = W.dfn_schur(n_frac=4, G=6, n_traces=7, L_lo=2, L_hi=5, sigma=1.5, seed=3)
    op = O.Operator(s.a, s.c, s.m, jacobi=True)
    P = 8
    f = M.features(op, s.a, s.c, s.m, power_steps=P)
    A = s.a.to_scipy().toarray()
    Cm = s.c.to_scipy().toarray()
    S = A + Cm.T @ np.diag(1 / s.m) @ Cm
    n = S.shape[0]
    d = np.diag(S).copy()
    dis = 1 / np.sqrt(d)
    Ah = A * np.outer(dis, dis)
    Ch = Cm * dis[None, :]
    rowabs = (np.abs(Ah) + np.abs(Ch).T @ np.diag(1 / s.m) @ np.abs(Ch)).sum(axis=1)
    ld = np.log10(d)
    assert f[1] == pytest.approx(np.count_nonzero(A) / n, rel=1e-15)
    assert f[3] == pytest.approx(np.std(ld), rel=1e-9)
    assert f[4] == pytest.approx(ld.min(), rel=1e-15) and f[5] == pytest.approx(ld.max(), rel=1e-15)
    assert f[6] == pytest.approx(rowabs.max(), rel=1e-13)
    assert f[7] == pytest.approx((rowabs - np.diag(Ah)).mean(), rel=1e-13)
    Sh = S * np.outer(dis, dis)
    lam, Q = np.linalg.eigh(Sh)
    v0 = O.fmix32_start(n)
    assert f[12] == pytest.approx(_power_rq(lam, Q, v0, P - 1), rel=1e-11)
    lmin_est = f[6] - _power_rq(lam, Q, v0, P - 1, shift=f[6])
    assert f[13] == pytest.approx(lmin_est, rel=1e-9, abs=1e-12)
    assert f[15] == pytest.approx(np.log10(_power_rq(lam, Q, v0, P - 1) / abs(lmin_est)), rel=1e-9)
