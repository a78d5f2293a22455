"""GPU parity of the persistent batched driver (PP_BOPT_DRIVER = 1).

The whole batched solve runs in one cooperative launch that sweeps the same
workgroup map as the host-driven chunks, so with every member running the
same number of iterations (no redistribution of workgroups on the host
side) its iterates equal the host-driven ones bit for bit; after tol-driven
solves, where the host side redistributes, that still holds (the map is
restored).  Against the
oracle, as for the other batch tests: every system's iterate after m
iterations within 1e-10 of its own oracle solve; tol-driven iteration
counts within 2; mixed precision to an FP64 true residual <= 1e-8.  Eight
members of the 256-system benchmark batch (sides 22..126) run with many
more map entries than resident workgroups, so every workgroup sweeps
several entries.  A spin limit of one poll forces PP_ERR_TIMEOUT from the
host; blocks of right-hand sides fall back to the host-driven chunks.
"""
import numpy as np
import pytest

import oracle as O
from paper_2208_01339_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SIZES = [6, 9, 11, 14, 5, 17]


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
def small():
    systems = [W.hetero_diffusion(N, 2.0, 100 + i) for i, N in enumerate(SIZES)]
    ops, lo, hi = [], [], []
    for a in systems:
        o = O.Operator(a, jacobi=True)
        l, h = O.lanczos_bounds(o, 20)
        ops.append(o)
        lo.append(l)
        hi.append(h)
    return systems, ops, np.array(lo), np.array(hi)


def solve(B, bo, nsys, nrhs, b, tol, maxit, driver):
    B.pp_batch_set_option(bo.handle, B.PP_BOPT_DRIVER, driver)
    X = torch.zeros(bo.n, nrhs, dtype=torch.float64, device="cuda")
    s, it, rel, stt = B.pcg_solve_batch(bo.handle, nsys, nrhs, dev(b), X, tol, maxit)
    return s, it, rel, stt, host(X), B.pp_batch_get_stats(bo.handle)


@pytest.mark.parametrize("layout", ["diag", "sliced"])
def test_persistent_batch_equal_iterations(B, small, layout):
    systems, ops, lo, hi = small
    k, xi, m = 7, 1e-3, 9
    flags = B.PP_JACOBI | (B.PP_SLICED if layout == "sliced" else 0)
    bo = B.BatchOperator(systems, nrhs=1, flags=flags)
    B.pp_batch_setup(bo.handle, k, lo, hi, xi)
    b = W.block_rhs(int(bo.sys_ptr[-1]), 1, 40)
    s, it, rel, stt, Xp, st = solve(B, bo, len(systems), 1, b, 0.0, m, 1)
    assert st["driver"] == 1
    assert np.all(it == m) and np.all(stt == B.PP_NOT_CONVERGED)
    for i, o in enumerate(ops):
        r0, r1 = bo.sys_ptr[i], bo.sys_ptr[i + 1]
        xo, sto = O.pcg(o, k, lo[i], hi[i], xi, b[r0:r1, 0], tol=0.0, maxit=m)
        err = np.linalg.norm(Xp[r0:r1, 0] - xo) / np.linalg.norm(xo)
        assert err <= 1e-10, (i, err)
        assert abs(rel[i, 0] - sto["relres"]) <= 1e-6 * sto["relres"]
    # the host-driven chunks on the same map give the same bits
    s0, it0, rel0, _, Xg, st0 = solve(B, bo, len(systems), 1, b, 0.0, m, 0)
    assert st0["driver"] == 0
    assert np.array_equal(it0, it) and np.array_equal(Xg, Xp) and np.array_equal(rel0, rel)
    bo.close()


def test_persistent_batch_tol_driven(B, small):
    """Members converge at different iterations (the host-driven solve then moves the
    workgroups of finished systems to the others; the persistent launch keeps its map):
    both within one iteration of each other, and a later equal-iteration solve on both
    drivers still gives the same bits."""
    systems, ops, lo, hi = small
    k = 10
    bo = B.BatchOperator(systems, nrhs=1, flags=B.PP_JACOBI)
    B.pp_batch_setup(bo.handle, k, lo, hi, 0.0)
    b = W.block_rhs(int(bo.sys_ptr[-1]), 1, 7)
    s, it, rel, stt, Xp, st = solve(B, bo, len(systems), 1, b, 1e-9, 500, 1)
    assert st["driver"] == 1 and s == B.PP_OK and np.all(stt == B.PP_OK) and np.all(rel <= 1e-9)
    assert len(set(int(v) for v in it[:, 0])) > 1
    for i, o in enumerate(ops):
        r0, r1 = bo.sys_ptr[i], bo.sys_ptr[i + 1]
        xo, sto = O.pcg(o, k, lo[i], hi[i], 0.0, b[r0:r1, 0], tol=1e-9, maxit=500)
        assert abs(int(it[i, 0]) - sto["iters"]) <= 2
        assert np.linalg.norm(Xp[r0:r1, 0] - xo) / np.linalg.norm(xo) <= 1e-6
    # the same tol-driven solve host-driven: the same iteration counts within one
    s0, it0, rel0, stt0, Xg, st0 = solve(B, bo, len(systems), 1, b, 1e-9, 500, 0)
    assert st0["driver"] == 0 and np.all(np.abs(it0 - it) <= 1) and np.all(rel0 <= 1e-9)
    # map restored: equal-iteration solves agree bit for bit again
    m = 6
    _, itp, _, _, Xpm, _ = solve(B, bo, len(systems), 1, b, 0.0, m, 1)
    _, itg, _, _, Xgm, _ = solve(B, bo, len(systems), 1, b, 0.0, m, 0)
    assert np.all(itp == m) and np.array_equal(itp, itg) and np.array_equal(Xpm, Xgm)
    bo.close()


@pytest.mark.parametrize("layout", ["diag", "sliced"])
def test_persistent_batch_mixed_residual(B, small, layout):
    systems, ops, lo, hi = small
    k = 12
    flags = B.PP_JACOBI | B.PP_MIXED | (B.PP_SLICED if layout == "sliced" else 0)
    bo = B.BatchOperator(systems, nrhs=1, flags=flags)
    B.pp_batch_setup(bo.handle, k, lo, hi, 0.0)
    b = W.block_rhs(int(bo.sys_ptr[-1]), 1, 3)
    s, it, rel, stt, Xp, st = solve(B, bo, len(systems), 1, b, 1e-8, 500, 1)
    assert st["driver"] == 1 and s == B.PP_OK and st["verified"] == 1
    for i, o in enumerate(ops):
        r0, r1 = bo.sys_ptr[i], bo.sys_ptr[i + 1]
        bi = b[r0:r1, 0]
        res = (o.apply_raw(Xp[r0:r1, 0]) - bi) * o.dis
        true = np.linalg.norm(res) / np.linalg.norm(bi * o.dis)
        assert true <= 1e-8, (i, true)
        assert rel[i, 0] == pytest.approx(true, rel=1e-6)
        xo, sto = O.pcg(o, k, lo[i], hi[i], 0.0, bi, tol=1e-8, maxit=500)
        assert abs(int(it[i, 0]) - sto["iters"]) <= 2
    bo.close()


def test_persistent_batch_degree0_and_zero_rhs(B, small):
    """k = 0 (the scaled identity) and a system whose right-hand side is zero."""
    systems, ops, lo, hi = small
    bo = B.BatchOperator(systems, nrhs=1, flags=B.PP_JACOBI)
    B.pp_batch_setup(bo.handle, 0, lo, hi, 0.0)
    b = W.block_rhs(int(bo.sys_ptr[-1]), 1, 9)
    b[bo.sys_ptr[2]:bo.sys_ptr[3], 0] = 0.0
    s, it, rel, stt, Xp, st = solve(B, bo, len(systems), 1, b, 1e-9, 2000, 1)
    assert st["driver"] == 1 and s == B.PP_OK
    assert it[2, 0] == 0 and np.all(Xp[bo.sys_ptr[2]:bo.sys_ptr[3], 0] == 0.0)
    for i, o in enumerate(ops):
        if i == 2:
            continue
        r0, r1 = bo.sys_ptr[i], bo.sys_ptr[i + 1]
        xo, sto = O.pcg(o, 0, lo[i], hi[i], 0.0, b[r0:r1, 0], tol=1e-9, maxit=2000)
        assert abs(int(it[i, 0]) - sto["iters"]) <= 2
    bo.close()


def test_persistent_batch_timeout_then_recovers(B, small):
    systems, ops, lo, hi = small
    k, m = 7, 9
    bo = B.BatchOperator(systems, nrhs=1, flags=B.PP_JACOBI)
    B.pp_batch_setup(bo.handle, k, lo, hi, 0.0)
    b = W.block_rhs(int(bo.sys_ptr[-1]), 1, 40)
    B.pp_batch_set_option(bo.handle, B.PP_OPT_SPIN_LIMIT, 1)
    with pytest.raises(B.PPError) as e:
        solve(B, bo, len(systems), 1, b, 0.0, m, 1)
    assert e.value.status == B.PP_ERR_TIMEOUT
    B.pp_batch_set_option(bo.handle, B.PP_OPT_SPIN_LIMIT, 1 << 21)
    s, it, rel, stt, Xp, st = solve(B, bo, len(systems), 1, b, 0.0, m, 1)
    assert st["driver"] == 1 and np.all(it == m)
    s0, it0, _, _, Xg, _ = solve(B, bo, len(systems), 1, b, 0.0, m, 0)
    assert np.array_equal(Xg, Xp)
    for key, bad in ((B.PP_BOPT_DRIVER, 2), (B.PP_OPT_BARRIER, 3), (B.PP_OPT_SPIN_LIMIT, 0)):
        with pytest.raises(B.PPError) as e:
            B.pp_batch_set_option(bo.handle, key, bad)
        assert e.value.status == B.PP_ERR_ARG
    bo.close()


def test_persistent_batch_block_rhs_falls_back(B, small):
    systems, ops, lo, hi = small
    k, m, nrhs = 7, 9, 3
    bo = B.BatchOperator(systems, nrhs=nrhs, flags=B.PP_JACOBI)
    B.pp_batch_setup(bo.handle, k, lo, hi, 0.0)
    b = W.block_rhs(int(bo.sys_ptr[-1]), nrhs, 41)
    s, it, rel, stt, Xp, st = solve(B, bo, len(systems), nrhs, b, 0.0, m, 1)
    assert st["driver"] == 0 and np.all(it == m)
    i = 3
    r0, r1 = bo.sys_ptr[i], bo.sys_ptr[i + 1]
    xo, _ = O.pcg(ops[i], k, lo[i], hi[i], 0.0, b[r0:r1, 1], tol=0.0, maxit=m)
    assert np.linalg.norm(Xp[r0:r1, 1] - xo) / np.linalg.norm(xo) <= 1e-10
    bo.close()


def test_persistent_batch_benchmark_subset(B):
    """Eight members of the 256-system benchmark batch (sides 22..126): the map has many
    more entries than resident workgroups.  Iterates after m iterations against each
    system's oracle solve (1e-10) and, bit for bit, against the host-driven chunks."""
    sides = W.batch_sizes()
    order = np.argsort(sides, kind="stable")
    pick = sorted(set(int(order[int(round(q * (len(order) - 1)))]) for q in np.linspace(0.0, 1.0, 8)))
    systems, rhs = [], []
    for i in pick:
        a_i, b_i = W.batch_system(i, int(sides[i]))
        systems.append(a_i)
        rhs.append(b_i)
    ops, lo, hi = [], [], []
    for a in systems:
        o = O.Operator(a, jacobi=True)
        l, h = O.lanczos_bounds(o, 20)
        ops.append(o)
        lo.append(l)
        hi.append(h)
    lo, hi = np.array(lo), np.array(hi)
    k, m = 60, 3
    bo = B.BatchOperator(systems, nrhs=1, flags=B.PP_JACOBI)
    B.pp_batch_setup(bo.handle, k, lo, hi, 0.0)
    bvec = np.concatenate(rhs).reshape(-1, 1)
    s, it, rel, stt, Xp, st = solve(B, bo, len(systems), 1, bvec, 0.0, m, 1)
    assert st["driver"] == 1 and np.all(it == m)
    for j, o in enumerate(ops):
        r0, r1 = bo.sys_ptr[j], bo.sys_ptr[j + 1]
        xo, _ = O.pcg(o, k, lo[j], hi[j], 0.0, rhs[j], tol=0.0, maxit=m)
        err = np.linalg.norm(Xp[r0:r1, 0] - xo) / np.linalg.norm(xo)
        assert err <= 1e-10, (pick[j], err)
    s0, it0, _, _, Xg, st0 = solve(B, bo, len(systems), 1, bvec, 0.0, m, 0)
    assert st0["driver"] == 0 and st0["grid"] > st["grid"]  # several map entries per workgroup
    assert np.array_equal(Xg, Xp)
    bo.close()
    # mixed, tol-driven, as in the benchmark: members finish at different iterations
    bm = B.BatchOperator(systems, nrhs=1, flags=B.PP_JACOBI | B.PP_MIXED)
    B.pp_batch_setup(bm.handle, k, lo, hi, 0.0)
    s, it, rel, stt, Xp, st = solve(B, bm, len(systems), 1, bvec, 1e-8, 500, 1)
    assert st["driver"] == 1 and s == B.PP_OK and st["verified"] == 1
    assert len(set(int(v) for v in it[:, 0])) > 1
    for j, o in enumerate(ops):
        r0, r1 = bm.sys_ptr[j], bm.sys_ptr[j + 1]
        res = (o.apply_raw(Xp[r0:r1, 0]) - rhs[j]) * o.dis
        true = np.linalg.norm(res) / np.linalg.norm(rhs[j] * o.dis)
        assert true <= 1e-8, (pick[j], true)
    s0, it0, _, _, _, _ = solve(B, bm, len(systems), 1, bvec, 1e-8, 500, 0)
    assert np.all(np.abs(it0 - it) <= 1)
    bm.close()
