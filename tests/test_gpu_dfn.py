"""GPU parity of the DFN Schur complement S_u (sections 4.2-4.3) against the oracle.

Both sides get the same generated blocks.  Relative bounds: the operator
apply (Algorithm 3 with the device Cholesky factor), the reduced right-hand
side and the recovery of h, p to 1e-11 (FP64; the factor and the solves sum
in a different order than the oracle); p_k(S-hat) r with D_S from Algorithm 4
to 1e-10; PCG on the same right-hand side at equal iteration counts to
1e-10; the whole pipeline (rhs, PCG to 1e-8, recovery) to iteration counts
within 2 and, at equal iteration counts, solutions to 1e-8 (the library's
right-hand side differs from the oracle's by 1e-11, times kappa(S-hat)).  Shapes: odd and
even grids, the grids whose sweeps are compiled for their exact width (16,
32, 48, 64) and others, the largest grid (64), more than 64 unknowns per
fracture (two workgroups of Algorithm 4), alpha != 1.
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


CASES = {
    "f6g8": dict(n_frac=6, G=8, n_traces=10, L_lo=3, L_hi=8, seed=0),
    "f9g5_alpha0.5": dict(n_frac=9, G=5, n_traces=14, L_lo=1, L_hi=5, seed=3, alpha=0.5),
    "f4g11_odd": dict(n_frac=4, G=11, n_traces=7, L_lo=4, L_hi=11, seed=5),
    "f3g64_max": dict(n_frac=3, G=64, n_traces=4, L_lo=20, L_hi=64, seed=6),
    "f2g30_many_u": dict(n_frac=2, G=30, n_traces=6, L_lo=20, L_hi=30, seed=8),  # > 64 unknowns per fracture
    # grids with a sweep compiled for exactly their width, and one just below
    "f3g16": dict(n_frac=3, G=16, n_traces=5, L_lo=4, L_hi=16, seed=11),
    "f2g32": dict(n_frac=2, G=32, n_traces=4, L_lo=8, L_hi=32, seed=12),
    "f2g48": dict(n_frac=2, G=48, n_traces=4, L_lo=10, L_hi=40, seed=10),
    "f2g47_odd": dict(n_frac=2, G=47, n_traces=4, L_lo=10, L_hi=40, seed=13),
    # the widest line (64 steps) padded with zero coefficients, one-line lookahead
    "f2g56": dict(n_frac=2, G=56, n_traces=4, L_lo=10, L_hi=50, seed=14),
}

# Shapes whose 20-step Lanczos estimate of lambda_min is far from converged and
# moves by percents under small changes of the operator's rounding.  On the
# CPU, for f2g56: a symmetric perturbation of the dense S-hat by 1e-15 (1e-13)
# of its largest entry moves it by 0.03 % (0.3 %), the dense product in place
# of the oracle's expansion by 0.9 %; the library's S_u agrees with the
# oracle's to 1e-11, and its estimate differs by about 6 %.  For f2g48 a
# 1e-15 perturbation already moves it by 1 %.
SENSITIVE_MIN = {"f2g48": 0.05, "f2g56": 0.1}

_cache = {}


def case(name):
    if name not in _cache:
        P = W.dfn_su(**CASES[name])
        _cache[name] = (P, O.DfnOperator(P, jacobi=False), O.DfnOperator(P, jacobi=True))
    return _cache[name]


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("name", list(CASES))
def test_apply_rhs_recover(B, name):
    P, orc, _ = case(name)
    op = B.Operator(dfn=P)
    rng = np.random.default_rng(1)
    x = rng.standard_normal(P.n_u)
    y = torch.empty(P.n_u, dtype=torch.float64, device="cuda")
    B.pp_operator_apply(op.handle, dev(x), y)
    assert rel(host(y), orc.apply(x)) <= 1e-11
    q = W.rhs_uniform(P.n_h, 2)
    r = torch.empty(P.n_u, dtype=torch.float64, device="cuda")
    B.pp_dfn_rhs(op.handle, dev(q), r)
    assert rel(host(r), orc.rhs(q)) <= 1e-11
    u = rng.standard_normal(P.n_u)
    h = torch.empty(P.n_h, dtype=torch.float64, device="cuda")
    p = torch.empty_like(h)
    B.pp_dfn_recover(op.handle, dev(q), dev(u), h, p)
    h0, p0 = orc.recover(q, u)
    assert rel(host(h), h0) <= 1e-11 and rel(host(p), p0) <= 1e-11
    st = B.pp_get_stats(op.handle)
    assert st["n"] == P.n_u and st["two_step"] == 0
    op.close()


@pytest.mark.parametrize("name", ["f6g8", "f4g11_odd", "f3g64_max", "f2g30_many_u", "f2g48", "f2g56"])
@pytest.mark.parametrize("k,xi", [(1, 0.0), (6, 1e-3), (15, 1e-2)])
def test_polynomial_apply(B, name, k, xi):
    """pp_apply = D^{-1/2} p_k(S-hat) D^{-1/2} r with D_S from Algorithm 4."""
    P, _, orj = case(name)
    op = B.Operator(dfn=P)
    lmin, lmax = O.lanczos_bounds(orj, 20)
    B.pp_setup(op.handle, k, lmin, lmax, xi)
    r = W.rhs_uniform(P.n_u, 7)
    z = torch.empty(P.n_u, dtype=torch.float64, device="cuda")
    B.pp_apply(op.handle, dev(r), z)
    assert rel(host(z), O.cheb_apply(orj, k, lmin, lmax, xi, r)) <= 1e-10
    op.close()


@pytest.mark.parametrize("name", ["f6g8", "f9g5_alpha0.5", "f3g64_max", "f2g48", "f2g56"])
def test_pipeline_pcg(B, name):
    """rhs -> PCG on S-hat -> recovery, against the oracle's pipeline; the
    recovered (h, u, p) satisfy the three block equations of eq. (sys).

    PCG itself is compared on the oracle's right-hand side: at equal iteration
    count within 1e-10.  The whole pipeline starts from the library's own
    right-hand side, which agrees with the oracle's to 1e-11; solving with it
    moves u by up to kappa(S-hat) times that (kappa ~ 1e3 here), so the
    pipeline's u is held to 1e-8."""
    P, orc, orj = case(name)
    op = B.Operator(dfn=P)
    q = W.rhs_uniform(P.n_h, 1)
    lo, hi = B.pp_estimate_bounds(op.handle, 20)
    lmin, lmax = O.lanczos_bounds(orj, 20)
    if name in SENSITIVE_MIN:
        # The smallest eigenvalues of S-hat are close (0.0555, 0.0563, 0.0633
        # for f2g48; 0.026, 0.049, 0.070 for f2g56) and 20 steps leave the Ritz
        # value unconverged: it moves in its second or third digit when the
        # operator's rounding changes, so the two Lanczos runs agree only
        # roughly; both must stay above lambda_min (interlacing).
        S = np.column_stack([orj.apply(e) for e in np.eye(P.n_u)])
        ev = np.linalg.eigvalsh((S + S.T) / 2)
        assert ev[0] - 1e-9 * ev[-1] <= lo and abs(lo - lmin) <= SENSITIVE_MIN[name] * lmin
        assert abs(hi - lmax) <= 1e-6 * lmax
    else:
        assert abs(lo - lmin) <= 1e-6 * lmax and abs(hi - lmax) <= 1e-6 * lmax
    k, xi = 8, 1e-3
    B.pp_setup(op.handle, k, lmin, lmax, xi)
    r = torch.empty(P.n_u, dtype=torch.float64, device="cuda")
    B.pp_dfn_rhs(op.handle, dev(q), r)
    r0 = orc.rhs(q)
    u0, st0 = O.pcg(orj, k, lmin, lmax, xi, r0, tol=1e-8, maxit=2000)
    assert st0["status"] == O.OK
    u = torch.zeros(P.n_u, dtype=torch.float64, device="cuda")
    s, it, relres = B.pcg_solve(op.handle, r, u, 1e-8, 2000)
    assert s == B.PP_OK and abs(it - st0["iters"]) <= 2
    # PCG parity on the same right-hand side, equal iteration count
    u.zero_()
    s, it2, _ = B.pcg_solve(op.handle, dev(r0), u, 0.0, st0["iters"])
    assert it2 == st0["iters"]
    assert rel(host(u), u0) <= 1e-10
    # the pipeline: the library's own right-hand side
    u.zero_()
    s, it2, _ = B.pcg_solve(op.handle, r, u, 0.0, st0["iters"])
    assert it2 == st0["iters"]
    ug = host(u)
    assert rel(ug, u0) <= 1e-8
    h = torch.empty(P.n_h, dtype=torch.float64, device="cuda")
    p = torch.empty_like(h)
    B.pp_dfn_recover(op.handle, dev(q), u, h, p)
    hg, pg = host(h), host(p)
    A, C, Bm, Gh, Gu = (m.to_scipy() for m in (P.a, P.c, P.b, P.gh, P.gu))
    a = P.alpha
    sc = np.linalg.norm(q)
    assert np.linalg.norm(A @ hg - C @ ug - q) <= 1e-10 * sc
    assert np.linalg.norm(Gh @ hg - a * (Bm @ ug) + A @ pg) <= 1e-8 * sc
    # the third block equation is the Schur system S_u u = r, solved to the
    # tolerance of the scaled system: held to what the oracle's own pipeline
    # (its u0 and recovery) leaves, not to a fixed multiple of ||q||
    h0, p0 = orc.recover(q, u0)
    res_orc = np.linalg.norm(-a * (Bm.T @ h0) + Gu @ u0 - C.T @ p0)
    assert np.linalg.norm(-a * (Bm.T @ hg) + Gu @ ug - C.T @ pg) <= 2.0 * res_orc + 1e-10 * sc
    op.close()


def _bad(P, **kw):
    import copy

    Q = copy.copy(P)
    for k, v in kw.items():
        setattr(Q, k, v)
    return Q


def _csr(S):
    S = S.tocsr()
    S.sort_indices()
    return W.CSR(S.shape[0], S.shape[1], S.indptr.astype(np.int64), S.indices.astype(np.int32), S.data)


def test_invalid_inputs(B):
    P = W.dfn_su(n_frac=4, G=8, n_traces=6, L_lo=2, L_hi=8, seed=2)
    # entry of A outside the band of its block
    a = P.a.to_scipy().tolil()
    a[0, 63] = a[63, 0] = -1e-3
    # asymmetric G^u
    gu = P.gu.to_scipy().tolil()
    gu[0, 1] += 1.0
    # a column of C in another fracture's block
    c = P.c.to_scipy().tolil()
    j = int(P.u_off[1])  # first unknown of fracture 1
    c[0, j] = 1.0
    b = P.b.to_scipy().tolil()
    b[0, j] = 1.0  # keep B = C + E pattern plausible
    uo = P.u_off.copy()
    uo[-1] -= 1
    for Q, msg in ((_bad(P, a=_csr(a)), "band"), (_bad(P, gu=_csr(gu)), "symmetric"),
                   (_bad(P, c=_csr(c)), "outside the fracture"), (_bad(P, u_off=uo), "u_off")):
        with pytest.raises(B.PPError) as e:
            B.Operator(dfn=Q)
        assert e.value.status == B.PP_ERR_ARG and msg in str(e.value), str(e.value)
    with pytest.raises(B.PPError):
        B.Operator(dfn=P, flags=B.PP_MIXED)
    # S_u indefinite for a large alpha: a non-positive diag(S_u) or a CG breakdown, never a wrong OK
    Q = _bad(P, alpha=50.0)
    try:
        op = B.Operator(dfn=Q)
    except B.PPError as e:
        assert e.status == B.PP_ERR_ARG
    else:
        op.close()


def _with_empty_fracture(P):
    """P plus one more fracture (a copy of block 0 of A and G^h) that owns no
    unknowns and meets no trace."""
    import scipy.sparse as sp

    nf = P.grid ** 2
    Q = _bad(P)
    for nm in ("a", "gh"):
        M = getattr(P, nm).to_scipy()
        blk = M[:nf, :nf]
        setattr(Q, nm, _csr(sp.block_diag([M, blk]).tocsr()))
    for nm in ("c", "b"):
        M = getattr(P, nm).to_scipy()
        setattr(Q, nm, _csr(sp.vstack([M, sp.csr_matrix((nf, P.n_u))]).tocsr()))
    Q.n_frac = P.n_frac + 1
    Q.u_off = np.concatenate([P.u_off, P.u_off[-1:]])
    return Q


@pytest.mark.parametrize("shape", ["empty_fracture", "one_cell"])
def test_degenerate_shapes(B, shape):
    """A fracture with no unknowns (skipped by Algorithm 4's workgroups, a zero
    block in every solve); one-cell fractures (G = 1: G^h = 0, alpha small
    enough for a positive diag(S_u); S_u itself is only semidefinite there)."""
    if shape == "empty_fracture":
        P = _with_empty_fracture(W.dfn_su(n_frac=5, G=7, n_traces=8, L_lo=2, L_hi=7, seed=9))
    else:
        P = W.dfn_su(n_frac=6, G=1, n_traces=9, L_lo=1, L_hi=1, seed=7, alpha=0.01)
    orc = O.DfnOperator(P, jacobi=False)
    assert np.all(orc.diag_raw() > 0)
    op = B.Operator(dfn=P)
    rng = np.random.default_rng(5)
    x = rng.standard_normal(P.n_u)
    y = torch.empty(P.n_u, dtype=torch.float64, device="cuda")
    B.pp_operator_apply(op.handle, dev(x), y)
    assert rel(host(y), orc.apply(x)) <= 1e-11
    q = W.rhs_uniform(P.n_h, 4)
    r = torch.empty(P.n_u, dtype=torch.float64, device="cuda")
    B.pp_dfn_rhs(op.handle, dev(q), r)
    assert rel(host(r), orc.rhs(q)) <= 1e-11
    h = torch.empty(P.n_h, dtype=torch.float64, device="cuda")
    p = torch.empty_like(h)
    B.pp_dfn_recover(op.handle, dev(q), dev(x), h, p)
    h0, p0 = orc.recover(q, x)
    assert rel(host(h), h0) <= 1e-11 and rel(host(p), p0) <= 1e-11
    # D_S from Algorithm 4 on the device: pp_apply at k = 0 is D_S^{-1} r / theta
    B.pp_setup(op.handle, 0, 0.5, 2.0, 0.0)
    z = torch.empty(P.n_u, dtype=torch.float64, device="cuda")
    B.pp_apply(op.handle, dev(x), z)
    theta = (0.5 + 2.0) / 2
    assert rel(host(z), x / orc.diag_raw() / theta) <= 1e-12
    op.close()


def test_gh_wide_rows(B):
    """G^h with rows longer than the entry-slot layout holds (17 entries: the
    whole band of a G = 8 grid), so the fracture kernel reads G^h by CSR rows."""
    import scipy.sparse as sp

    P = W.dfn_su(n_frac=4, G=8, n_traces=6, L_lo=2, L_hi=8, seed=4)
    gh = P.gh.to_scipy().tolil()
    lo, m = 20, 17  # a principal block of fracture 0 inside its band: SPD, so G^h stays SPSD
    for i in range(m):
        for j in range(m):
            d = abs(i - j)
            if d <= P.grid:
                gh[lo + i, lo + j] += 1e-2 * (3.0 if d == 0 else 0.5 ** d)
    Q = _bad(P, gh=_csr(gh))
    assert np.diff(Q.gh.rowptr).max() > 16
    orc = O.DfnOperator(Q, jacobi=False)
    op = B.Operator(dfn=Q)
    rng = np.random.default_rng(3)
    x = rng.standard_normal(Q.n_u)
    y = torch.empty(Q.n_u, dtype=torch.float64, device="cuda")
    B.pp_operator_apply(op.handle, dev(x), y)
    assert rel(host(y), orc.apply(x)) <= 1e-11
    q = W.rhs_uniform(Q.n_h, 2)
    r = torch.empty(Q.n_u, dtype=torch.float64, device="cuda")
    B.pp_dfn_rhs(op.handle, dev(q), r)
    assert rel(host(r), orc.rhs(q)) <= 1e-11
    h = torch.empty(Q.n_h, dtype=torch.float64, device="cuda")
    p = torch.empty_like(h)
    B.pp_dfn_recover(op.handle, dev(q), dev(x), h, p)
    h0, p0 = orc.recover(q, x)
    assert rel(host(h), h0) <= 1e-11 and rel(host(p), p0) <= 1e-11
    op.close()


def test_recover_into_q(B):
    """pp_dfn_recover with h (or p) written over q itself."""
    P, orc, _ = case("f6g8")
    op = B.Operator(dfn=P)
    rng = np.random.default_rng(6)
    q = W.rhs_uniform(P.n_h, 4)
    u = rng.standard_normal(P.n_u)
    h0, p0 = orc.recover(q, u)
    for into in ("h", "p"):
        qd = dev(q)
        other = torch.empty_like(qd)
        h, p = (qd, other) if into == "h" else (other, qd)
        B.pp_dfn_recover(op.handle, qd, dev(u), h, p)
        assert rel(host(h), h0) <= 1e-11 and rel(host(p), p0) <= 1e-11, into
    op.close()
