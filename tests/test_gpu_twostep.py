"""GPU checks of the fused pairs of Chebyshev steps on 3-D 7-point operators.

The pair kernel computes the same terms per row as the one-step kernels, so
p_k(A) r with pairs and without them agree to a few ulps (relative 1e-14
in FP64), and both match the oracle's Algorithm 2 to 1e-12; in the FP32 mixed
mode they agree within FP32 rounding.  Box shapes cover ragged y-tiles (tiles of 8 lines: remainders of
5 and 7), z-ranges that are not whole chunks of 32 planes (37 planes; 33,
so that the last chunk holds one plane), and boxes that are not cubes
(principal blocks of the first z-planes).
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


def first_planes(a, N, nz):
    """Principal block of the first nz z-planes of an N^3 operator: an N x N x nz box."""
    m = N * N * nz
    S = a.to_scipy()[:m, :m].tocsr()
    S.sort_indices()
    return W.CSR(m, m, S.indptr.astype(np.int64), S.indices.astype(np.int32), S.data)


CASES = {
    "poisson32": (lambda: W.poisson3d(32), False),
    "hetero37": (lambda: W.hetero_diffusion(37, 2.0, 3), True),
    "hetero31": (lambda: W.hetero_diffusion(31, 1.0, 4), True),  # x-y tiles of 30 and 1
    "box23x23x9": (lambda: first_planes(W.hetero_diffusion(23, 2.0, 6), 23, 9), True),
    "box40x40x33": (lambda: first_planes(W.hetero_diffusion(40, 2.0, 9), 40, 33), True),
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("k,xi", [(4, 0.0), (5, 0.0), (6, 1e-3), (20, 0.0), (21, 1e-2)])
def test_pairs_match_single_steps_and_oracle(B, name, k, xi):
    build, jac = CASES[name]
    a = build()
    op = B.Operator(a=a, flags=B.PP_JACOBI if jac else 0)
    B.pp_set_option(op.handle, B.PP_OPT_TWO_STEP, 2)  # these boxes are smaller than the automatic rule's
    assert B.pp_get_stats(op.handle)["two_step"] == 1
    orc = O.Operator(a, jacobi=jac)
    lmin, lmax = O.lanczos_bounds(orc, 20)
    B.pp_setup(op.handle, k, lmin, lmax, xi)
    r = W.rhs_uniform(a.n_rows, 7)
    z2 = torch.empty(a.n_rows, dtype=torch.float64, device="cuda")
    z1 = torch.empty_like(z2)
    B.pp_apply(op.handle, dev(r), z2)
    B.pp_set_option(op.handle, B.PP_OPT_TWO_STEP, 0)
    assert B.pp_get_stats(op.handle)["two_step"] == 0
    B.pp_apply(op.handle, dev(r), z1)
    g2, g1 = host(z2), host(z1)
    assert np.linalg.norm(g2 - g1) <= 1e-14 * np.linalg.norm(g1)
    ref = O.cheb_apply(orc, k, lmin, lmax, xi, r)
    assert np.linalg.norm(g2 - ref) <= 1e-12 * np.linalg.norm(ref)
    op.close()


@pytest.mark.parametrize("k", [4, 7, 20])
@pytest.mark.parametrize("name", ["hetero37", "box40x40x33", "poisson32"])
def test_mixed_pairs(B, name, k):
    """Mixed mode runs the pairs in FP32 too; at even k the last pair's second step
    reads r in FP64 for the dot product and writes z in FP64 (odd k: the last step
    runs alone, FP32 in, FP64 out; pp_apply under Jacobi scaling, whose output is
    scaled, ends with a single step too, so the unscaled poisson32 covers the last
    pair in pp_apply).  p_k(A) r with FP32 pairs against the FP32
    single steps and against the oracle within FP32 rounding (the bound of the
    mixed pp_apply test, 1e-4; the two FP32 forms differ only in rounding, 1e-5);
    PCG: FP64 true scaled residual <= 1e-8, iterations within 2 of the FP64 oracle."""
    build, jac = CASES[name]
    a = build()
    op = B.Operator(a=a, flags=(B.PP_JACOBI if jac else 0) | B.PP_MIXED)
    B.pp_set_option(op.handle, B.PP_OPT_TWO_STEP, 2)
    assert B.pp_get_stats(op.handle)["two_step"] == 1
    orc = O.Operator(a, jacobi=jac)
    lmin, lmax = O.lanczos_bounds(orc, 20)
    B.pp_setup(op.handle, k, lmin, lmax, 1e-3)
    r = W.rhs_uniform(a.n_rows, 7)
    z2 = torch.empty(a.n_rows, dtype=torch.float64, device="cuda")
    z1 = torch.empty_like(z2)
    B.pp_apply(op.handle, dev(r), z2)
    B.pp_set_option(op.handle, B.PP_OPT_TWO_STEP, 0)
    B.pp_apply(op.handle, dev(r), z1)
    g2, g1 = host(z2), host(z1)
    ref = O.cheb_apply(orc, k, lmin, lmax, 1e-3, r)
    assert np.linalg.norm(g2 - g1) <= 1e-5 * np.linalg.norm(g1)
    assert np.linalg.norm(g2 - ref) <= 1e-4 * np.linalg.norm(ref)
    B.pp_set_option(op.handle, B.PP_OPT_TWO_STEP, 2)
    b = W.rhs_uniform(a.n_rows, 1)
    xo, sto = O.pcg(orc, k, lmin, lmax, 1e-3, b, tol=1e-8, maxit=2000)
    x = torch.zeros(a.n_rows, dtype=torch.float64, device="cuda")
    s, it, rel = B.pcg_solve(op.handle, dev(b), x, 1e-8, 2000)
    assert s == B.PP_OK and abs(it - sto["iters"]) <= 2, (it, sto["iters"])
    res = orc.apply_raw(host(x)) - b
    bb = b
    if jac:
        res, bb = res * orc.dis, b * orc.dis
    assert np.linalg.norm(res) / np.linalg.norm(bb) <= 1e-8
    op.close()


@pytest.mark.parametrize("k", [4, 7, 12])
@pytest.mark.parametrize("name", ["hetero37", "box23x23x9", "box40x40x33"])
def test_pairs_pcg_parity(B, name, k):
    """Even k: the last pair carries the dot product of the CG step; odd k: the
    last step runs alone; k = 4: the smallest degree that uses pairs."""
    build, jac = CASES[name]
    a = build()
    op = B.Operator(a=a, flags=B.PP_JACOBI)
    B.pp_set_option(op.handle, B.PP_OPT_TWO_STEP, 2)
    assert B.pp_get_stats(op.handle)["two_step"] == 1
    orc = O.Operator(a, jacobi=True)
    lmin, lmax = O.lanczos_bounds(orc, 20)
    xi = 1e-3
    b = W.rhs_uniform(a.n_rows, 1)
    xo, sto = O.pcg(orc, k, lmin, lmax, xi, b, tol=1e-8, maxit=2000)
    B.pp_setup(op.handle, k, lmin, lmax, xi)
    x = torch.zeros(a.n_rows, dtype=torch.float64, device="cuda")
    s, it, rel = B.pcg_solve(op.handle, dev(b), x, 1e-8, 2000)
    assert s == B.PP_OK and abs(it - sto["iters"]) <= 2
    x.zero_()
    s, it2, rel2 = B.pcg_solve(op.handle, dev(b), x, 0.0, sto["iters"])
    assert np.linalg.norm(host(x) - xo) <= 1e-10 * np.linalg.norm(xo)
    op.close()


def test_face_coupling_disables_pairs(B):
    """A coupling across an x-face of the box (row x = N-1 to the next line's x = 0,
    both ways) keeps offset 1 a stored diagonal but rules the pair kernel out."""
    N = 12
    A = W.poisson3d(N).to_scipy().tolil()
    i = N - 1  # (x = N-1, y = 0, z = 0) -> (0, 1, 0)
    A[i, i + 1] = -0.5
    A[i + 1, i] = -0.5
    A = A.tocsr()
    A.sort_indices()
    a = W.CSR(N ** 3, N ** 3, A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data)
    op = B.Operator(a=a)
    st = B.pp_get_stats(op.handle)
    assert st["diagonals"] == 4 and st["two_step"] == 0
    orc = O.Operator(a)
    lmin, lmax = O.lanczos_bounds(orc, 20)
    B.pp_setup(op.handle, 9, lmin, lmax, 0.0)
    r = W.rhs_uniform(a.n_rows, 3)
    z = torch.empty(a.n_rows, dtype=torch.float64, device="cuda")
    B.pp_apply(op.handle, dev(r), z)
    ref = O.cheb_apply(orc, 9, lmin, lmax, 0.0, r)
    assert np.linalg.norm(host(z) - ref) <= 1e-12 * np.linalg.norm(ref)
    op.close()


def test_pair_timing_stats(B):
    """With PP_OPT_TIMING the solve reports the fused-pair launches it timed:
    floor(k / 2) per polynomial application (steps 1 and 2 form the first pair;
    for even k the last pair carries the dot product), one application per iteration."""
    a = W.hetero_diffusion(24, 2.0, 2)
    op = B.Operator(a=a, flags=B.PP_JACOBI)
    B.pp_set_option(op.handle, B.PP_OPT_TWO_STEP, 2)
    orc = O.Operator(a, jacobi=True)
    lmin, lmax = O.lanczos_bounds(orc, 20)
    b = dev(W.rhs_uniform(a.n_rows, 3))
    x = torch.zeros(a.n_rows, dtype=torch.float64, device="cuda")
    for k in (12, 13):
        B.pp_setup(op.handle, k, lmin, lmax, 0.0)
        B.pp_set_option(op.handle, B.PP_OPT_TIMING, 1)
        x.zero_()
        s, it, _ = B.pcg_solve(op.handle, b, x, 1e-8, 500)
        st = B.pp_get_stats(op.handle)
        assert s == B.PP_OK and it > 0
        assert st["pair_launches"] == it * (k // 2)
        assert 0 < st["pair_ms"] < st["cheb_ms"]
        B.pp_set_option(op.handle, B.PP_OPT_TIMING, 0)
        x.zero_()
        B.pcg_solve(op.handle, b, x, 1e-8, 500)
        st = B.pp_get_stats(op.handle)
        assert st["pair_launches"] == 0 and st["pair_ms"] == 0
    op.close()


def test_automatic_rule(B):
    """By default pairs run only when the box gives at least one tile per compute
    unit (a 24^3 box gives three); 2 forces them, 0 turns them off, other values
    are refused."""
    a = W.hetero_diffusion(24, 1.0, 3)
    op = B.Operator(a=a, flags=B.PP_JACOBI)
    assert B.pp_get_stats(op.handle)["two_step"] == 0
    B.pp_set_option(op.handle, B.PP_OPT_TWO_STEP, 2)
    assert B.pp_get_stats(op.handle)["two_step"] == 1
    B.pp_set_option(op.handle, B.PP_OPT_TWO_STEP, 0)
    assert B.pp_get_stats(op.handle)["two_step"] == 0
    with pytest.raises(B.PPError):
        B.pp_set_option(op.handle, B.PP_OPT_TWO_STEP, 3)
    op.close()


def test_unit_diagonal_flag(B):
    """Under Jacobi scaling the stored main diagonal of a CSR operator is exactly 1
    (reported as unit_diagonal, and the pairs do not read it); without scaling,
    and for the Schur shape (whose stored A_ff diagonal is not the operator's), it
    is the stored data.  Operator application stays within the per-row bound."""
    a = W.hetero_diffusion(12, 2.0, 3)
    orc = O.Operator(a, jacobi=True)
    for flags, want in ((B.PP_JACOBI, 1), (0, 0), (B.PP_JACOBI | B.PP_SLICED, 0)):
        op = B.Operator(a=a, flags=flags)
        assert B.pp_get_stats(op.handle)["unit_diagonal"] == want, flags
        op.close()
    s = W.dfn_schur(n_frac=13, G=16, n_traces=30, L_lo=3, L_hi=12, seed=2)
    op = B.Operator(schur=s, flags=B.PP_JACOBI)
    assert B.pp_get_stats(op.handle)["unit_diagonal"] == 0
    op.close()
    op = B.Operator(a=a, flags=B.PP_JACOBI)
    x = W.rhs_uniform(a.n_rows, 4)
    y = torch.empty(a.n_rows, dtype=torch.float64, device="cuda")
    B.pp_operator_apply(op.handle, dev(x), y)
    bound = abs(a.to_scipy()) @ np.abs(x)
    assert np.all(np.abs(host(y) - orc.apply_raw(x)) <= 32 * np.finfo(np.float64).eps * bound)
    op.close()
