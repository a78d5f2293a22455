"""GPU parity of the Newton form (Algorithm 1) against the oracle's Algorithm 1.

pp_apply after pp_setup_newton: relative error <= 1e-12 against the oracle's
newton_apply (same recursion, different rounding order).  In exact
arithmetic the Newton form equals the Chebyshev polynomial of degree
2^nlev - 1 (pinned on the CPU), so PCG with it is checked against the
oracle's Chebyshev PCG of that degree: iteration counts within +-2, and the
solutions agree to the tolerance of the solve; and against the oracle's PCG
with Algorithm 1 itself at equal iteration count (1e-10).
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
    "poisson16": (lambda: (W.poisson3d(16), None), False),
    "hetero21_jac": (lambda: (W.hetero_diffusion(21, 2.0, 5), None), True),
    "dfn_small_jac": (lambda: (None, W.dfn_schur(n_frac=13, G=16, n_traces=30, L_lo=3, L_hi=12, seed=2)), True),
}


def make(B, name, flags=0):
    build, jac = CASES[name]
    a, s = build()
    fl = (B.PP_JACOBI if jac else 0) | flags
    if s is not None:
        return B.Operator(schur=s, flags=fl), O.Operator(s.a, s.c, s.m, jacobi=jac)
    return B.Operator(a=a, flags=fl), O.Operator(a, jacobi=jac)


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("nlev,xi", [(0, 0.0), (1, 0.0), (2, 1e-3), (3, 0.0), (4, 1e-2), (6, 1e-3)])
def test_newton_apply(B, name, nlev, xi):
    op, orc = make(B, name)
    lmin, lmax = O.lanczos_bounds(orc, 20)
    B.pp_setup_newton(op.handle, nlev, lmin, lmax, xi)
    r = W.rhs_uniform(orc.n, 7)
    z = torch.empty(orc.n, dtype=torch.float64, device="cuda")
    B.pp_apply(op.handle, dev(r), z)
    if orc.dis is None:
        ref = O.newton_apply_hat(orc, nlev, lmin, lmax, xi, r)
    else:
        ref = orc.dis * O.newton_apply_hat(orc, nlev, lmin, lmax, xi, orc.dis * r)
    assert np.linalg.norm(host(z) - ref) <= 1e-12 * np.linalg.norm(ref)
    op.close()


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("nlev,xi", [(2, 0.0), (4, 1e-3)])
def test_newton_pcg(B, name, nlev, xi):
    op, orc = make(B, name, B.PP_MIXED)  # the Newton form runs in FP64 even under PP_MIXED
    lmin, lmax = O.lanczos_bounds(orc, 20)
    k = 2 ** nlev - 1
    b = W.rhs_uniform(orc.n, 1)
    xo, sto = O.pcg(orc, k, lmin, lmax, xi, b, tol=1e-10, maxit=3000)
    B.pp_setup_newton(op.handle, nlev, lmin, lmax, xi)
    B.pp_set_option(op.handle, B.PP_OPT_DRIVER, 1)  # falls back to the stream driver
    B.pp_set_option(op.handle, B.PP_OPT_VERIFY, 0)  # keep the loop's count identity exact
    x = torch.zeros(orc.n, dtype=torch.float64, device="cuda")
    s, it, rel = B.pcg_solve(op.handle, dev(b), x, 1e-10, 3000)
    st = B.pp_get_stats(op.handle)
    assert s == B.PP_OK and abs(it - sto["iters"]) <= 2 and st["driver"] == 0
    assert st["op_applies"] == 1 + k * it + it
    got = host(x)
    # both stop at ||r_hat|| <= 1e-10 ||b_hat||: the solutions differ by at most ~2 kappa 1e-10
    assert np.linalg.norm(got - xo) <= 1e-6 * np.linalg.norm(xo)
    # back to the three-term form
    B.pp_setup(op.handle, k, lmin, lmax, xi)
    x.zero_()
    s2, it2, _ = B.pcg_solve(op.handle, dev(b), x, 1e-10, 3000)
    assert s2 == B.PP_OK and abs(it2 - sto["iters"]) <= 2
    op.close()


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("nlev,xi", [(0, 0.0), (2, 0.0), (3, 1e-3), (5, 1e-2)])
def test_newton_pcg_equal_iterations(B, name, nlev, xi):
    """PCG with the Newton form against the oracle's PCG with Algorithm 1 (the
    same preconditioner, different rounding order): iterations within 2 at
    tol 1e-8, and the iterate after the oracle's iteration count within 1e-10."""
    op, orc = make(B, name)
    lmin, lmax = O.lanczos_bounds(orc, 20)
    b = W.rhs_uniform(orc.n, 1)
    xo, sto = O.pcg_newton(orc, nlev, lmin, lmax, xi, b, tol=1e-8, maxit=3000)
    assert sto["status"] == O.OK
    B.pp_setup_newton(op.handle, nlev, lmin, lmax, xi)
    x = torch.zeros(orc.n, dtype=torch.float64, device="cuda")
    s, it, _ = B.pcg_solve(op.handle, dev(b), x, 1e-8, 3000)
    assert s == B.PP_OK and abs(it - sto["iters"]) <= 2, (it, sto["iters"])
    x.zero_()
    s, it2, _ = B.pcg_solve(op.handle, dev(b), x, 0.0, sto["iters"])
    assert it2 == sto["iters"] and s == B.PP_NOT_CONVERGED
    err = np.linalg.norm(host(x) - xo) / np.linalg.norm(xo)
    assert err <= 1e-10, err
    op.close()


def test_newton_bad_args(B):
    a = W.poisson3d(6)
    op = B.Operator(a=a)
    for args in [(-1, 0.1, 10.0, 0.0), (13, 0.1, 10.0, 0.0), (3, 0.0, 10.0, 0.0), (3, 1.0, 0.5, 0.0)]:
        with pytest.raises(B.PPError):
            B.pp_setup_newton(op.handle, *args)
    op.close()
