"""Grid barriers of the persistent PCG driver (PP_OPT_BARRIER).

The runtime's cooperative barrier (mode 0), the flat hand-written barrier (1)
and the two-level one (2: per-XCD arrival and one L2 writeback per XCD, then a
global arrival among the XCD leaders) must give the same solve: at the
oracle's iteration count (tol = 0) the iterate within 1e-10 of the oracle's
PCG, and the tol-driven iteration count within 2.  Grids of 5 workgroups
(three XCDs hold none), 8 (one per XCD), 37 (uneven shares) and 128; the
Schur-shaped kernel and mixed precision too.  A spin limit of one poll makes
the hand-written waits give up: the solve returns PP_ERR_TIMEOUT (an error
forced from the host; every workgroup still leaves the kernel), and the
handle then solves normally again.
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


@pytest.fixture(scope="module")
def poisson():
    a = W.poisson3d(32)
    orc = O.Operator(a)
    lmin, lmax = O.lanczos_bounds(orc, 20)
    b = W.rhs_uniform(a.n_rows, 1)
    xo, sto = O.pcg(orc, 10, lmin, lmax, 0.0, b, tol=1e-8, maxit=5000)
    assert sto["status"] == O.OK
    return a, orc, (lmin, lmax), b, xo, sto


def persistent_op(B, flags, mode, grid, a=None, schur=None):
    op = B.Operator(a=a, schur=schur, flags=flags)
    B.pp_set_option(op.handle, B.PP_OPT_DRIVER, 1)
    B.pp_set_option(op.handle, B.PP_OPT_BARRIER, mode)
    B.pp_set_option(op.handle, B.PP_OPT_GRID, grid)
    return op


def solve_and_compare(B, op, b, xo, sto, grid, mode):
    n = b.size
    bd = dev(b)
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    s, it, rel = B.pcg_solve(op.handle, bd, x, 1e-8, 5000)
    st = B.pp_get_stats(op.handle)
    assert (st["driver"], st["grid"], st["barrier"]) == (1, grid, mode), st
    assert s == B.PP_OK and rel <= 1e-8 and abs(it - sto["iters"]) <= 2, (it, sto["iters"])
    x.zero_()
    s, it2, _ = B.pcg_solve(op.handle, bd, x, 0.0, sto["iters"])
    assert s == B.PP_NOT_CONVERGED and it2 == sto["iters"]
    err = np.linalg.norm(host(x) - xo) / np.linalg.norm(xo)
    assert err <= 1e-10, err


@pytest.mark.parametrize("grid", [5, 8, 37, 128])
@pytest.mark.parametrize("mode", [0, 1, 2], ids=["runtime", "flat", "two_level"])
def test_barrier_modes_parity(B, poisson, mode, grid):
    a, orc, (lmin, lmax), b, xo, sto = poisson
    op = persistent_op(B, 0, mode, grid, a=a)
    B.pp_setup(op.handle, 10, lmin, lmax, 0.0)
    solve_and_compare(B, op, b, xo, sto, grid, mode)
    op.close()


@pytest.mark.parametrize("mode", [1, 2], ids=["flat", "two_level"])
def test_barrier_schur_parity(B, mode):
    s = W.dfn_schur(n_frac=13, G=16, n_traces=30, L_lo=3, L_hi=12, seed=2)
    orc = O.Operator(s.a, s.c, s.m, jacobi=True)
    lmin, lmax = O.lanczos_bounds(orc, 20)
    b = W.rhs_uniform(orc.n, 1)
    xo, sto = O.pcg(orc, 8, lmin, lmax, 1e-3, b, tol=1e-8, maxit=5000)
    assert sto["status"] == O.OK
    op = persistent_op(B, B.PP_JACOBI, mode, 13, schur=s)
    B.pp_setup(op.handle, 8, lmin, lmax, 1e-3)
    solve_and_compare(B, op, b, xo, sto, 13, mode)
    op.close()


@pytest.mark.parametrize("mode", [1, 2], ids=["flat", "two_level"])
def test_barrier_mixed_true_residual(B, poisson, mode):
    a, orc, (lmin, lmax), b, xo, sto = poisson
    op = persistent_op(B, B.PP_MIXED, mode, 64, a=a)
    B.pp_setup(op.handle, 10, lmin, lmax, 0.0)
    x = torch.zeros(a.n_rows, dtype=torch.float64, device="cuda")
    s, it, rel = B.pcg_solve(op.handle, dev(b), x, 1e-8, 5000)
    st = B.pp_get_stats(op.handle)
    assert (st["driver"], st["grid"], st["barrier"]) == (1, 64, mode)
    assert s == B.PP_OK and abs(it - sto["iters"]) <= 2
    got = host(x)
    true = np.linalg.norm(orc.apply_raw(got) - b) / np.linalg.norm(b)
    assert true <= 1e-8 and st["true_relres"] == pytest.approx(true, rel=1e-6)
    assert np.linalg.norm(got - xo) / np.linalg.norm(xo) <= 1e-4
    op.close()


@pytest.mark.parametrize("mode", [1, 2], ids=["flat", "two_level"])
def test_barrier_timeout_then_recovers(B, poisson, mode):
    a, orc, (lmin, lmax), b, xo, sto = poisson
    op = persistent_op(B, 0, mode, 32, a=a)
    B.pp_setup(op.handle, 10, lmin, lmax, 0.0)
    B.pp_set_option(op.handle, B.PP_OPT_SPIN_LIMIT, 1)
    x = torch.zeros(a.n_rows, dtype=torch.float64, device="cuda")
    with pytest.raises(B.PPError) as e:
        B.pcg_solve(op.handle, dev(b), x, 1e-8, 5000)
    assert e.value.status == B.PP_ERR_TIMEOUT
    assert B.pp_get_stats(op.handle)["status"] == B.PP_ERR_TIMEOUT
    B.pp_set_option(op.handle, B.PP_OPT_SPIN_LIMIT, 1 << 21)
    solve_and_compare(B, op, b, xo, sto, 32, mode)
    op.close()


def test_barrier_options_validated(B, poisson):
    a = poisson[0]
    op = B.Operator(a=a, flags=0)
    for key, bad in ((B.PP_OPT_BARRIER, 3), (B.PP_OPT_BARRIER, -2), (B.PP_OPT_SPIN_LIMIT, 0),
                     (B.PP_OPT_SPIN_LIMIT, (1 << 31) + 1)):
        with pytest.raises(B.PPError) as e:
            B.pp_set_option(op.handle, key, bad)
        assert e.value.status == B.PP_ERR_ARG
    op.close()
