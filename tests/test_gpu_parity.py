"""GPU parity: the HIP library (through the C ABI) against the CPU oracle.

Inputs come from the seeded generators; expected values come only from the
oracle.  Tolerances:
  * operator application: per row |y - y_ref| <= 8 eps sum_j |a_ij x_j|
    (different summation order and fused multiply-adds on the GPU);
  * p_k(A) r: relative 2-norm error <= 1e-12 (k steps of a stable three-term
    recurrence, each adding a few ulps);
  * PCG: iteration count within +-2 at tol 1e-8; at equal iteration count
    (maxit = the oracle's count, tol = 0) relative solution error <= 1e-10.
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


def dev(x, dt=None):
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dt is not None:
        t = t.to(dt)
    return t.cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def absdot_bound(a, x):
    """sum_j |a_ij x_j| per row."""
    A = a.to_scipy()
    return abs(A) @ np.abs(x)


def _cases():
    return {
        "poisson32": lambda: (W.poisson3d(32), None),
        "hetero21": lambda: (W.hetero_diffusion(21, 2.0, 5), None),
        "dfn_small": lambda: (None, W.dfn_schur(n_frac=13, G=16, n_traces=30, L_lo=3, L_hi=12, seed=2)),
    }


LAYOUTS = ["diag", "sliced"]


def make_op(B, a, s, flags, layout="diag"):
    """layout "diag": the library's default (symmetric stored diagonals where they pay);
    "sliced": every entry in the sliced ELLPACK layout (PP_SLICED)."""
    return B.Operator(a=a, schur=s, flags=flags | (B.PP_SLICED if layout == "sliced" else 0))


def make_oracle(a, s, jacobi):
    if s is not None:
        return O.Operator(s.a, s.c, s.m, jacobi=jacobi)
    return O.Operator(a, jacobi=jacobi)


# ---------------------------------------------------------------------------
# operator application
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("case", list(_cases()))
@pytest.mark.parametrize("flags", [0, 1])
def test_operator_apply(B, case, flags, layout):
    a, s = _cases()[case]()
    op = make_op(B, a, s, flags, layout)
    orc = make_oracle(a, s, False)
    x = W.rhs_uniform(orc.n, 42)
    y = torch.empty(orc.n, dtype=torch.float64, device="cuda")
    B.pp_operator_apply(op.handle, dev(x), y)
    got = host(y)
    ref = orc.apply_raw(x)
    if s is None:
        bound = absdot_bound(a, x)
    else:
        Cm = s.c.to_scipy()
        bound = absdot_bound(s.a, x) + abs(Cm.T) @ ((abs(Cm) @ np.abs(x)) / s.m)
    tol = (8 if flags == 0 else 32) * EPS * bound + 1e-300
    assert np.all(np.abs(got - ref) <= tol), np.max(np.abs(got - ref) / tol)
    st = B.pp_get_stats(op.handle)
    assert st["n"] == orc.n
    # 7-point stencils keep 4 stored diagonals (0, 1, N, N^2), the fracture blocks 3 (0, 1, G)
    assert st["diagonals"] == (0 if layout == "sliced" else (3 if s is not None else 4))
    op.close()


# ---------------------------------------------------------------------------
# p_k(A) r (Algorithm 2)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("case", list(_cases()))
@pytest.mark.parametrize("jacobi", [False, True])
@pytest.mark.parametrize("k,xi", [(0, 0.0), (1, 0.0), (2, 1e-3), (3, 0.0), (10, 1e-3), (40, 0.0)])
def test_pp_apply(B, case, jacobi, k, xi, layout):
    a, s = _cases()[case]()
    orc = make_oracle(a, s, jacobi)
    lmin, lmax = O.lanczos_bounds(orc, 20)
    op = make_op(B, a, s, B.PP_JACOBI if jacobi else 0, layout)
    B.pp_setup(op.handle, k, lmin, lmax, xi)
    r = W.rhs_uniform(orc.n, 7)
    z = torch.empty(orc.n, dtype=torch.float64, device="cuda")
    B.pp_apply(op.handle, dev(r), z)
    got = host(z)
    ref = O.cheb_apply(orc, k, lmin, lmax, xi, r)
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert err <= 1e-12, err
    op.close()


def test_pp_apply_requires_setup(B):
    a = W.poisson3d(8)
    op = make_op(B, a, None, 0)
    r = torch.zeros(a.n_rows, dtype=torch.float64, device="cuda")
    z = torch.zeros_like(r)
    with pytest.raises(B.PPError) as e:
        B.pp_apply(op.handle, r, z)
    assert e.value.status == B.PP_ERR_STATE
    for args in [(3, 0.0, 1.0, 0.0), (3, 2.0, 1.0, 0.0), (3, 0.1, 1.0, -1.0), (-1, 0.1, 1.0, 0.0),
                 (5000, 0.1, 1.0, 0.0), (3, float("nan"), 1.0, 0.0)]:
        with pytest.raises(B.PPError) as e:
            B.pp_setup(op.handle, *args)
        assert e.value.status == B.PP_ERR_ARG
    op.close()


# ---------------------------------------------------------------------------
# PCG
# ---------------------------------------------------------------------------

PCG_CASES = [
    # name, builder, jacobi, k, xi
    ("poisson32_k10", lambda: (W.poisson3d(32), None), False, 10, 0.0),
    ("poisson32_k10_xi", lambda: (W.poisson3d(32), None), False, 10, 1e-3),
    ("hetero21_k20_jac", lambda: (W.hetero_diffusion(21, 2.0, 5), None), True, 20, 0.0),
    ("hetero21_k3_jac", lambda: (W.hetero_diffusion(21, 2.0, 5), None), True, 3, 1e-3),
    ("hetero21_k0_jac", lambda: (W.hetero_diffusion(21, 2.0, 5), None), True, 0, 0.0),
    ("dfn_small_k8_jac", lambda: (None, W.dfn_schur(n_frac=13, G=16, n_traces=30, L_lo=3, L_hi=12, seed=2)),
     True, 8, 1e-3),
]


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("driver", [0, 1], ids=["stream", "persistent"])
@pytest.mark.parametrize("name,builder,jacobi,k,xi", PCG_CASES, ids=[c[0] for c in PCG_CASES])
def test_pcg_parity(B, name, builder, jacobi, k, xi, driver, layout):
    a, s = builder()
    orc = make_oracle(a, s, jacobi)
    n = orc.n
    b = W.rhs_uniform(n, 1)
    lmin, lmax = O.lanczos_bounds(orc, 20)
    xo, sto = O.pcg(orc, k, lmin, lmax, xi, b, tol=1e-8, maxit=5000)
    assert sto["status"] == O.OK
    op = make_op(B, a, s, B.PP_JACOBI if jacobi else 0, layout)
    B.pp_set_option(op.handle, B.PP_OPT_DRIVER, driver)
    B.pp_setup(op.handle, k, lmin, lmax, xi)
    bd = dev(b)
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    status, it, rel = B.pcg_solve(op.handle, bd, x, 1e-8, 5000)
    assert B.pp_get_stats(op.handle)["driver"] == driver
    assert status == B.PP_OK
    assert abs(it - sto["iters"]) <= 2, (it, sto["iters"])
    assert rel <= 1e-8
    # equal iteration count: run exactly the oracle's iterations
    x.zero_()
    status, it2, rel2 = B.pcg_solve(op.handle, bd, x, 0.0, sto["iters"])
    assert it2 == sto["iters"] and status == B.PP_NOT_CONVERGED
    got = host(x)
    err = np.linalg.norm(got - xo) / np.linalg.norm(xo)
    assert err <= 1e-10, err
    assert abs(rel2 - sto["relres"]) <= 1e-6 * sto["relres"] + 1e-14
    st = B.pp_get_stats(op.handle)
    assert st["iters"] == it2
    op.close()


VARIANTS = {
    # the launch forms the 256^3 benchmark runs, forced at a size the oracle finishes in seconds
    "nt_loads": {"PP_OPT_NT_LOADS": 1, "PP_OPT_TWO_STEP": 0},
    "pairs": {"PP_OPT_NT_LOADS": 0, "PP_OPT_TWO_STEP": 2},
    "pairs_nt_loads": {"PP_OPT_NT_LOADS": 1, "PP_OPT_TWO_STEP": 2},
    "verify": {"PP_OPT_VERIFY": 1},
}


@pytest.mark.parametrize("variant", list(VARIANTS))
@pytest.mark.parametrize("name,builder,jacobi,k,xi", [PCG_CASES[i] for i in (0, 1, 2, 3)],
                         ids=[PCG_CASES[i][0] for i in (0, 1, 2, 3)])
def test_pcg_parity_variants(B, name, builder, jacobi, k, xi, variant):
    """Equal-iteration parity (1e-10) and iteration counts (+-2) with non-temporal
    loads and fused pairs of steps forced on (both switch on by themselves only at
    2^22 rows and on boxes that fill the chip), and with the true-residual check."""
    a, s = builder()
    orc = make_oracle(a, s, jacobi)
    n = orc.n
    b = W.rhs_uniform(n, 1)
    lmin, lmax = O.lanczos_bounds(orc, 20)
    xo, sto = O.pcg(orc, k, lmin, lmax, xi, b, tol=1e-8, maxit=5000)
    op = make_op(B, a, s, B.PP_JACOBI if jacobi else 0)
    for key, val in VARIANTS[variant].items():
        B.pp_set_option(op.handle, getattr(B, key), val)
    B.pp_setup(op.handle, k, lmin, lmax, xi)
    st = B.pp_get_stats(op.handle)
    if variant.startswith("pairs"):
        assert st["two_step"] == 1
    bd = dev(b)
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    status, it, rel = B.pcg_solve(op.handle, bd, x, 1e-8, 5000)
    assert status == B.PP_OK and abs(it - sto["iters"]) <= 2, (it, sto["iters"])
    st = B.pp_get_stats(op.handle)
    if variant == "verify":
        # the returned residual is the true one; check it with the oracle's operator
        got = host(x)
        r = (orc.apply_raw(got) - b) * (orc.dis if jacobi else 1.0)
        bb = b * (orc.dis if jacobi else 1.0)
        true = np.linalg.norm(r) / np.linalg.norm(bb)
        assert st["true_relres"] == pytest.approx(true, rel=1e-6) and true <= 1e-8
        if st["restarts"] == 0:  # the check passed at once: one more operator application
            assert st["op_applies"] == 1 + k * it + it + 1
    x.zero_()
    status, it2, rel2 = B.pcg_solve(op.handle, bd, x, 0.0, sto["iters"])
    assert it2 == sto["iters"] and status == B.PP_NOT_CONVERGED
    err = np.linalg.norm(host(x) - xo) / np.linalg.norm(xo)
    assert err <= 1e-10, err
    op.close()


@pytest.mark.parametrize("driver", [0, 1], ids=["stream", "persistent"])
def test_pcg_edge_cases(B, driver):
    a = W.poisson3d(10)
    orc = O.Operator(a)
    n = orc.n
    op = make_op(B, a, None, 0)
    B.pp_set_option(op.handle, B.PP_OPT_DRIVER, driver)
    B.pp_setup(op.handle, 4, 0.2, 12.0, 0.0)
    # b = 0 -> x = 0, no iteration
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    s, it, rel = B.pcg_solve(op.handle, torch.zeros(n, dtype=torch.float64, device="cuda"), x)
    assert s == B.PP_OK and it == 0 and float(x.abs().max()) == 0.0
    # maxit = 1
    b = W.rhs_uniform(n, 0)
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    s, it, rel = B.pcg_solve(op.handle, dev(b), x, 1e-8, 1)
    assert s == B.PP_NOT_CONVERGED and it == 1
    # maxit = 0
    x.zero_()
    s, it, rel = B.pcg_solve(op.handle, dev(b), x, 1e-8, 0)
    assert s == B.PP_NOT_CONVERGED and it == 0
    # NaN in b -> breakdown
    bb = b.copy()
    bb[5] = np.nan
    x.zero_()
    s, it, rel = B.pcg_solve(op.handle, dev(bb), x, 1e-8, 100)
    assert s == B.PP_BREAKDOWN
    # x0 = solution -> zero iterations
    xs = np.linalg.solve(a.to_scipy().toarray(), b)
    x = dev(xs)
    s, it, rel = B.pcg_solve(op.handle, dev(b), x, 1e-8, 100)
    assert s == B.PP_OK and it == 0
    # warm start from a partial solve converges to the same solution
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    B.pcg_solve(op.handle, dev(b), x, 0.0, 3)
    s, it, rel = B.pcg_solve(op.handle, dev(b), x, 1e-10, 500)
    assert s == B.PP_OK
    assert np.linalg.norm(host(x) - xs) / np.linalg.norm(xs) < 1e-8
    # invalid arguments
    with pytest.raises(B.PPError):
        B.pcg_solve(op.handle, dev(b), x, -1.0, 10)
    with pytest.raises(B.PPError):
        B.pcg_solve(op.handle, dev(b), x, 1e-8, -1)
    op.close()


@pytest.mark.parametrize("driver", [0, 1], ids=["stream", "persistent"])
def test_odd_degree_bad_bounds_breakdown(B, driver):
    """Odd k with lambda_max far too small makes P indefinite (p_k < 0 beyond 2 theta-bar)."""
    a = W.poisson3d(12)
    orc = O.Operator(a)
    b = W.rhs_uniform(orc.n, 3)
    lmin, lmax = 0.05, 2.0  # true lambda_max ~ 11.7 > 2 theta-bar
    xo, sto = O.pcg(orc, 9, lmin, lmax, 0.0, b, tol=1e-8, maxit=300)
    op = make_op(B, a, None, 0)
    B.pp_set_option(op.handle, B.PP_OPT_DRIVER, driver)
    B.pp_setup(op.handle, 9, lmin, lmax, 0.0)
    x = torch.zeros(orc.n, dtype=torch.float64, device="cuda")
    s, it, rel = B.pcg_solve(op.handle, dev(b), x, 1e-8, 300)
    assert sto["status"] == O.BREAKDOWN
    assert s == B.PP_BREAKDOWN
    op.close()


def test_create_rejects_bad_input(B):
    a = W.poisson3d(6)
    bad = a.col.copy()
    bad[3] = a.n_rows + 5
    with pytest.raises(B.PPError) as e:
        B.pp_create_csr(a.n_rows, a.nnz, dev(a.rowptr), dev(bad), dev(a.val))
    assert e.value.status == B.PP_ERR_ARG
    v = a.val.copy()
    v[a.rowptr[2]:a.rowptr[3]] = -1.0  # row 2 diagonal negative
    with pytest.raises(B.PPError) as e:
        B.pp_create_csr(a.n_rows, a.nnz, dev(a.rowptr), dev(a.col), dev(v), B.PP_JACOBI)
    assert e.value.status == B.PP_ERR_ARG


# ---------------------------------------------------------------------------
# Lanczos bounds
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("case", list(_cases()))
@pytest.mark.parametrize("jacobi", [False, True])
def test_lanczos_bounds(B, case, jacobi, layout):
    a, s = _cases()[case]()
    orc = make_oracle(a, s, jacobi)
    lo_r, hi_r = O.lanczos_bounds(orc, 20)
    op = make_op(B, a, s, B.PP_JACOBI if jacobi else 0, layout)
    lo, hi = B.pp_estimate_bounds(op.handle, 20)
    # Ritz values are eigenvalues of T_20; two T_20 built with different
    # rounding orders differ by O(eps ||A||) amplified by the loss of
    # orthogonality of plain Lanczos, and by Weyl's theorem so do their
    # eigenvalues: the tolerance is relative to ||A|| ~ lambda_max, not to
    # an unconverged lambda_min.
    assert abs(lo - lo_r) <= 1e-7 * hi_r
    assert abs(hi - hi_r) <= 1e-7 * hi_r
    op.close()


def test_config0_end_to_end(B):
    """3-D Poisson 32^3, degree 10, bounds from 20-step Lanczos, tol 1e-8: the whole path on the GPU."""
    a, b = W.config_poisson32()
    orc = O.Operator(a)
    lo_r, hi_r = O.lanczos_bounds(orc, 20)
    xo, sto = O.pcg(orc, 10, lo_r, hi_r, 0.0, b, tol=1e-8, maxit=1000)
    op = make_op(B, a, None, 0)
    lo, hi = B.pp_estimate_bounds(op.handle, 20)
    B.pp_setup(op.handle, 10, lo, hi, 0.0)
    assert abs(lo - lo_r) <= 1e-7 * hi_r and abs(hi - hi_r) <= 1e-7 * hi_r
    x = torch.zeros(orc.n, dtype=torch.float64, device="cuda")
    s, it, rel = B.pcg_solve(op.handle, dev(b), x, 1e-8, 1000)
    assert s == B.PP_OK and abs(it - sto["iters"]) <= 2
    got = host(x)
    true_rel = np.linalg.norm(b - a.to_scipy() @ got) / np.linalg.norm(b)
    assert true_rel <= 1.5e-8
    assert np.linalg.norm(got - xo) / np.linalg.norm(xo) <= 1e-6
    op.close()


# ---------------------------------------------------------------------------
# mixed precision (FP32 polynomial, FP64 CG)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("driver", [0, 1], ids=["stream", "persistent"])
@pytest.mark.parametrize("name,builder,jacobi,k,xi", PCG_CASES[:4] + PCG_CASES[5:], ids=[c[0] for c in PCG_CASES[:4] + PCG_CASES[5:]])
def test_mixed_pcg_residual(B, name, builder, jacobi, k, xi, driver, layout):
    a, s = builder()
    orc = make_oracle(a, s, jacobi)
    n = orc.n
    b = W.rhs_uniform(n, 1)
    lmin, lmax = O.lanczos_bounds(orc, 20)
    xo, sto = O.pcg(orc, k, lmin, lmax, xi, b, tol=1e-8, maxit=5000)
    op = make_op(B, a, s, (B.PP_JACOBI if jacobi else 0) | B.PP_MIXED, layout)
    B.pp_set_option(op.handle, B.PP_OPT_DRIVER, driver)
    B.pp_setup(op.handle, k, lmin, lmax, xi)
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    status, it, rel = B.pcg_solve(op.handle, dev(b), x, 1e-8, 5000)
    assert B.pp_get_stats(op.handle)["driver"] == driver
    assert status == B.PP_OK and rel <= 1e-8
    assert abs(it - sto["iters"]) <= 2, (it, sto["iters"])
    got = host(x)
    # FP64 true residual of the scaled system, computed by the oracle operator
    r = orc.apply_raw(got) - b
    if jacobi:
        r = r * orc.dis
        bb = b * orc.dis
    else:
        bb = b
    # the true-residual check (on by default in mixed mode) holds the FP64 true
    # residual to the tolerance, and the library reports that residual
    true = np.linalg.norm(r) / np.linalg.norm(bb)
    st = B.pp_get_stats(op.handle)
    assert true <= 1e-8, true
    assert st["true_relres"] == pytest.approx(true, rel=1e-6)
    # final-solution error against the FP64 oracle, bounded by the condition number
    assert np.linalg.norm(got - xo) / np.linalg.norm(xo) <= 1e-4
    op.close()


@pytest.mark.parametrize("jacobi", [False, True])
def test_mixed_pp_apply_close(B, jacobi):
    a = W.hetero_diffusion(21, 2.0, 5)
    orc = O.Operator(a, jacobi=jacobi)
    lmin, lmax = O.lanczos_bounds(orc, 20)
    op = make_op(B, a, None, (B.PP_JACOBI if jacobi else 0) | B.PP_MIXED)
    for k in (1, 2, 20, 60):
        B.pp_setup(op.handle, k, lmin, lmax, 0.0)
        r = W.rhs_uniform(orc.n, 7)
        z = torch.empty(orc.n, dtype=torch.float64, device="cuda")
        B.pp_apply(op.handle, dev(r), z)
        ref = O.cheb_apply(orc, k, lmin, lmax, 0.0, r)
        err = np.linalg.norm(host(z) - ref) / np.linalg.norm(ref)
        assert err <= 1e-4, (k, err)
    op.close()


def test_drivers_agree_bitwise_iterations(B):
    """Stream-driven and persistent drivers reduce in different partitions, so
    iterates differ in the last bits; iteration counts may differ by one at most."""
    a = W.hetero_diffusion(24, 2.0, 9)
    orc = O.Operator(a, jacobi=True)
    lmin, lmax = O.lanczos_bounds(orc, 20)
    b = W.rhs_uniform(a.n_rows, 2)
    res = []
    for driver in (0, 1):
        op = make_op(B, a, None, B.PP_JACOBI)
        B.pp_set_option(op.handle, B.PP_OPT_DRIVER, driver)
        B.pp_setup(op.handle, 12, lmin, lmax, 1e-3)
        x = torch.zeros(a.n_rows, dtype=torch.float64, device="cuda")
        s, it, rel = B.pcg_solve(op.handle, dev(b), x, 1e-10, 1000)
        assert s == B.PP_OK
        res.append((it, host(x)))
        op.close()
    assert abs(res[0][0] - res[1][0]) <= 1
    assert np.linalg.norm(res[0][1] - res[1][1]) / np.linalg.norm(res[0][1]) < 1e-9
