"""The allocation-free solve (pcg_solve_csr_noalloc) against the library's
handle-based solve (pp_create_csr + pp_setup + pcg_solve) on the same inputs,
through the C ABI: iteration counts within 2 at tol 1e-8, and at equal
iteration counts (tol = 0, maxit = the handle solve's count) the iterates
within 1e-10.  Two calls in a row share the library's scratch array; the
second is smaller than the first, so stale contents of the first call must
not leak into it.
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


def _csr_dev(a):
    return dev(np.asarray(a.rowptr, dtype=np.int64)), dev(np.asarray(a.col, dtype=np.int32)), dev(a.val)


def _compare(B, a, jacobi, k, xi):
    n = a.n_rows
    orc = O.Operator(a, jacobi=jacobi)
    lmin, lmax = O.lanczos_bounds(orc, 20)
    b = W.rhs_uniform(n, 1)
    flags = B.PP_JACOBI if jacobi else 0
    rp, ci, va = _csr_dev(a)
    bd = dev(b)
    # the existing entry points
    op = B.Operator(a=a, flags=flags)
    B.pp_setup(op.handle, k, lmin, lmax, xi)
    x_ref = torch.zeros(n, dtype=torch.float64, device="cuda")
    s_ref, it_ref, rel_ref = B.pcg_solve(op.handle, bd, x_ref, 1e-8, 3000)
    assert s_ref == B.PP_OK
    x_ref.zero_()
    B.pcg_solve(op.handle, bd, x_ref, 0.0, it_ref)
    op.close()
    # the allocation-free one
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    s, it, rel = B.pcg_solve_csr_noalloc(n, len(a.val), rp, ci, va, flags, k, lmin, lmax, xi, bd, x, 1e-8, 3000)
    assert s == B.PP_OK and rel <= 1e-8 and abs(it - it_ref) <= 2, (s, it, it_ref, rel)
    x.fill_(0.0)
    s, it2, _ = B.pcg_solve_csr_noalloc(n, len(a.val), rp, ci, va, flags, k, lmin, lmax, xi, bd, x, 0.0, it_ref)
    assert s == B.PP_NOT_CONVERGED and it2 == it_ref
    xr = host(x_ref)
    err = np.linalg.norm(host(x) - xr) / np.linalg.norm(xr)
    assert err <= 1e-10, err


def test_noalloc_matches_pcg_solve_two_calls(B):
    # first call: 24^3 heterogeneous operator, Jacobi, k = 20; second: a smaller
    # Poisson box without scaling, k = 10 (stale scratch from the first must not matter)
    _compare(B, W.hetero_diffusion(24, 2.0, 0), True, 20, 0.0)
    _compare(B, W.poisson3d(12), False, 10, 1e-3)


def test_noalloc_degree0_and_zero_rhs(B):
    a = W.poisson3d(10)
    n = a.n_rows
    rp, ci, va = _csr_dev(a)
    orc = O.Operator(a)
    lmin, lmax = O.lanczos_bounds(orc, 20)
    b = W.rhs_uniform(n, 3)
    xo, sto = O.pcg(orc, 0, lmin, lmax, 0.0, b, tol=1e-8, maxit=2000)
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    s, it, _ = B.pcg_solve_csr_noalloc(n, len(a.val), rp, ci, va, 0, 0, lmin, lmax, 0.0, dev(b), x, 1e-8, 2000)
    assert s == B.PP_OK and abs(it - sto["iters"]) <= 2
    x.fill_(1.0)
    s, it, rel = B.pcg_solve_csr_noalloc(n, len(a.val), rp, ci, va, 0, 4, lmin, lmax, 0.0,
                                         torch.zeros(n, dtype=torch.float64, device="cuda"), x, 1e-8, 100)
    assert s == B.PP_OK and it == 0 and rel == 0.0 and float(x.abs().max()) == 0.0


def test_noalloc_rejects(B):
    a = W.poisson3d(6)
    n = a.n_rows
    rp, ci, va = _csr_dev(a)
    b = dev(W.rhs_uniform(n, 1))
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    bad = [
        dict(n=(1 << 20) + 1),      # beyond the scratch capacity (checked before any device work)
        dict(flags=2),              # PP_MIXED is not offered
        dict(k=-1), dict(k=1025),
        dict(lmin=0.0), dict(lmax=0.1),
    ]
    for kw in bad:
        args = dict(n=n, flags=0, k=4, lmin=0.5, lmax=12.0)
        args.update(kw)
        with pytest.raises(B.PPError):
            B.pcg_solve_csr_noalloc(args["n"], len(a.val), rp, ci, va, args["flags"], args["k"], args["lmin"],
                                    args["lmax"], 0.0, b, x, 1e-8, 10)
    # a non-positive diagonal under Jacobi: PP_ERR_ARG, x untouched
    va2 = va.clone()
    va2[0] = -6.0 if int(host(ci)[0]) == 0 else va2[0]
    x.fill_(3.0)
    with pytest.raises(B.PPError):
        B.pcg_solve_csr_noalloc(n, len(a.val), rp, ci, va2, B.PP_JACOBI, 4, 0.5, 12.0, 0.0, b, x, 1e-8, 10)
    assert float(x.min()) == 3.0 and float(x.max()) == 3.0
