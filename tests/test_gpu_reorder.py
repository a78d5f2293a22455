"""GPU parity of renumbered operators (reverse Cuthill-McKee at create).

An irregular operator (workloads.irregular_fe: thinned 27-point graph
Laplacian, numbered by random permutations inside windows) is renumbered by
the library; every entry point keeps the caller's numbering.  The oracle sees
the caller's matrix as given.  Bounds as in the other parity tests: operator
application per row within 8 eps sum |a_ij x_j| (times the Jacobi rescaling),
p_k(A) r within 1e-12, Lanczos bounds within 1e-7 lambda_max, PCG iteration
counts within 2 and equal-iteration iterates within 1e-10, features within
1e-9.  PP_NO_REORDER keeps the order and gives the same results.
"""
import numpy as np
import pytest

import oracle as O
from oracle import mlp as M
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


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.fixture(scope="module")
def irr():
    return W.irregular_fe(24, seed=3)


@pytest.mark.parametrize("flags", ["jacobi", "plain", "jacobi_mixed"])
def test_reordered_operator_parity(B, irr, flags):
    a = irr
    jac = flags != "plain"
    fl = (B.PP_JACOBI if jac else 0) | (B.PP_MIXED if flags == "jacobi_mixed" else 0)
    op = B.Operator(a=a, flags=fl)
    st = B.pp_get_stats(op.handle)
    assert st["reordered"] == 1 and st["diagonals"] == 0 and st["gather_spread"] < 0.25
    orc = O.Operator(a, jacobi=jac)
    n = a.n_rows
    # operator application, in the caller's numbering
    x = W.rhs_uniform(n, 4)
    y = torch.empty(n, dtype=torch.float64, device="cuda")
    B.pp_operator_apply(op.handle, dev(x), y)
    bound = abs(a.to_scipy()) @ np.abs(x)
    assert np.all(np.abs(host(y) - orc.apply_raw(x)) <= (32 if jac else 8) * EPS * bound)
    # bounds from the caller's start vector
    lmin, lmax = O.lanczos_bounds(orc, 20)
    lo, hi = B.pp_estimate_bounds(op.handle, 20)
    assert abs(lo - lmin) <= 1e-7 * lmax and abs(hi - lmax) <= 1e-7 * lmax
    k, xi = 12, 1e-3
    B.pp_setup(op.handle, k, lmin, lmax, xi)
    r = W.rhs_uniform(n, 7)
    z = torch.empty(n, dtype=torch.float64, device="cuda")
    B.pp_apply(op.handle, dev(r), z)
    ref = O.cheb_apply(orc, k, lmin, lmax, xi, r)
    err = np.linalg.norm(host(z) - ref) / np.linalg.norm(ref)
    assert err <= (1e-5 if flags == "jacobi_mixed" else 1e-12), err
    # PCG
    b = W.rhs_uniform(n, 1)
    xo, sto = O.pcg(orc, k, lmin, lmax, xi, b, tol=1e-8, maxit=3000)
    xs = torch.zeros(n, dtype=torch.float64, device="cuda")
    s, it, rel = B.pcg_solve(op.handle, dev(b), xs, 1e-8, 3000)
    assert s == B.PP_OK and abs(it - sto["iters"]) <= 2, (it, sto["iters"])
    if flags == "jacobi_mixed":
        res = (orc.apply_raw(host(xs)) - b) * orc.dis
        assert np.linalg.norm(res) / np.linalg.norm(b * orc.dis) <= 1e-8
    else:
        xs.zero_()
        s, it2, _ = B.pcg_solve(op.handle, dev(b), xs, 0.0, sto["iters"])
        assert it2 == sto["iters"]
        err = np.linalg.norm(host(xs) - xo) / np.linalg.norm(xo)
        assert err <= 1e-10, err
    op.close()


def test_reorder_off_gives_the_same(B, irr):
    a = irr
    n = a.n_rows
    ops = [B.Operator(a=a, flags=B.PP_JACOBI), B.Operator(a=a, flags=B.PP_JACOBI | B.PP_NO_REORDER)]
    assert [B.pp_get_stats(o.handle)["reordered"] for o in ops] == [1, 0]
    orc = O.Operator(a, jacobi=True)
    lmin, lmax = O.lanczos_bounds(orc, 20)
    b = W.rhs_uniform(n, 2)
    outs = []
    for o in ops:
        B.pp_setup(o.handle, 20, lmin, lmax, 0.0)
        x = torch.zeros(n, dtype=torch.float64, device="cuda")
        s, it, _ = B.pcg_solve(o.handle, dev(b), x, 0.0, 15)
        outs.append(host(x))
        o.close()
    assert np.linalg.norm(outs[0] - outs[1]) <= 1e-10 * np.linalg.norm(outs[1])


def test_reordered_lowrank_and_features(B, irr):
    a = irr
    n = a.n_rows
    op = B.Operator(a=a, flags=B.PP_JACOBI)
    orc = O.Operator(a, jacobi=True)
    # V round trip through the library's numbering
    V = np.random.default_rng(0).normal(size=(2, n))
    B.pp_lowrank_set(op.handle, 2, dev(V))
    Vd = torch.empty(2, n, dtype=torch.float64, device="cuda")
    B.pp_lowrank_get(op.handle, Vd)
    assert np.array_equal(host(Vd), V)
    # the correction applies V as given
    lmin, lmax = O.lanczos_bounds(orc, 20)
    B.pp_setup(op.handle, 8, lmin, lmax, 0.0)
    hinv = O.lowrank_setup(orc, V.T)
    r = W.rhs_uniform(n, 5)
    z = torch.empty(n, dtype=torch.float64, device="cuda")
    B.pp_apply(op.handle, dev(r), z)
    ref = orc.dis * O.lowrank_apply_hat(orc, 8, lmin, lmax, 0.0, V.T, hinv, orc.dis * r)
    assert np.linalg.norm(host(z) - ref) <= 1e-11 * np.linalg.norm(ref)
    B.pp_lowrank_set(op.handle, 0)
    # Ritz values of the library's own Lanczos (caller's start vector)
    th = B.pp_lowrank_ritz(op.handle, 30, 2)
    th_o, _ = O.ritz_vectors(orc, 30, 2)
    assert np.all(np.abs(th - th_o) <= 1e-7 * lmax), (th, th_o)
    op.close()
    # features (permutation invariant; power steps from the caller's start vector)
    op = B.Operator(a=a, flags=B.PP_JACOBI)
    got = B.pp_features(op.handle, 8)
    ref = M.features(orc, a, power_steps=8)
    op.close()
    assert np.allclose(got, ref, rtol=1e-9, atol=1e-12), np.max(np.abs(got - ref) / (np.abs(ref) + 1e-12))
