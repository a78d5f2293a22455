"""GPU parity of the batched path: many systems and/or a block of right-hand sides.

Every (system, column) is compared with its own single-system oracle solve
on the same inputs; the bounds passed to both come from the oracle.
FP64: equal iteration count (every member runs exactly m iterations, tol 0)
-> relative solution error <= 1e-10; tol-driven iteration counts within +-2.
FP32 polynomial (mixed): the scaled FP64 true residual <= 1e-8 (the library
checks it at exit) and iteration counts within +-2 of the FP64 oracle (no
iterate-level pin).  A subset of the 256-system benchmark batch (eight
members, sides 22 to 126) checks per-system storage and the redistribution
of workgroups at the benchmark's sizes.
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


SIZES = [6, 9, 11, 14, 5, 17]


def members():
    return [W.hetero_diffusion(N, 2.0, 100 + i) for i, N in enumerate(SIZES)]


def oracle_bounds(systems):
    lo, hi = [], []
    ops = []
    for a in systems:
        o = O.Operator(a, jacobi=True)
        l, h = O.lanczos_bounds(o, 20)
        lo.append(l)
        hi.append(h)
        ops.append(o)
    return ops, np.array(lo), np.array(hi)


def block_rhs(sys_ptr, nrhs, seed0):
    n = int(sys_ptr[-1])
    return W.block_rhs(n, nrhs, seed0)


LAYOUTS = ["diag", "sliced"]


def lay(B, layout):
    """Storage flag: "diag" = the default per-system choice, "sliced" = PP_SLICED."""
    return B.PP_SLICED if layout == "sliced" else 0


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("nrhs", [1, 3, 8])
def test_batch_bounds_match_oracle(B, nrhs, layout):
    systems = members()
    ops, lo, hi = oracle_bounds(systems)
    bo = B.BatchOperator(systems, nrhs=nrhs, flags=B.PP_JACOBI | lay(B, layout))
    assert B.pp_batch_get_stats(bo.handle)["diag_systems"] == (len(systems) if layout == "diag" else 0)
    glo, ghi = B.pp_batch_estimate_bounds(bo.handle, len(systems), 20)
    assert np.all(np.abs(glo - lo) <= 1e-7 * hi)
    assert np.all(np.abs(ghi - hi) <= 1e-7 * hi)
    bo.close()


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("nrhs,w", [(1, 1), (3, 8), (3, 4), (3, 2), (3, 1), (8, 8), (8, 2), (8, 1), (20, 32),
                                    (20, 16), (20, 8), (20, 4)])
def test_batch_fp64_equal_iterations(B, nrhs, w, layout):
    systems = members()
    ops, lo, hi = oracle_bounds(systems)
    k, xi, m = 7, 1e-3, 9
    bo = B.BatchOperator(systems, nrhs=nrhs, flags=B.PP_JACOBI | lay(B, layout))
    B.pp_batch_set_layout(bo.handle, w)
    B.pp_batch_setup(bo.handle, k, lo, hi, xi)
    Bm = block_rhs(bo.sys_ptr, nrhs, 40)
    X = torch.zeros(bo.n, nrhs, dtype=torch.float64, device="cuda")
    s, it, rel, stt = B.pcg_solve_batch(bo.handle, len(systems), nrhs, dev(Bm), X, 0.0, m)
    assert np.all(it == m) and np.all(stt == B.PP_NOT_CONVERGED)
    Xg = host(X)
    for i, o in enumerate(ops):
        r0, r1 = bo.sys_ptr[i], bo.sys_ptr[i + 1]
        for c in range(nrhs):
            xo, sto = O.pcg(o, k, lo[i], hi[i], xi, Bm[r0:r1, c], tol=0.0, maxit=m)
            err = np.linalg.norm(Xg[r0:r1, c] - xo) / np.linalg.norm(xo)
            assert err <= 1e-10, (i, c, err)
            assert abs(rel[i, c] - sto["relres"]) <= 1e-6 * sto["relres"]
    bo.close()


@pytest.mark.parametrize("nrhs", [1, 4])
def test_batch_fp64_tol_driven(B, nrhs):
    systems = members()
    ops, lo, hi = oracle_bounds(systems)
    k = 10
    bo = B.BatchOperator(systems, nrhs=nrhs, flags=B.PP_JACOBI)
    B.pp_batch_setup(bo.handle, k, lo, hi, 0.0)
    Bm = block_rhs(bo.sys_ptr, nrhs, 7)
    X = torch.zeros(bo.n, nrhs, dtype=torch.float64, device="cuda")
    s, it, rel, stt = B.pcg_solve_batch(bo.handle, len(systems), nrhs, dev(Bm), X, 1e-9, 500)
    assert s == B.PP_OK and np.all(stt == B.PP_OK) and np.all(rel <= 1e-9)
    Xg = host(X)
    for i, o in enumerate(ops):
        r0, r1 = bo.sys_ptr[i], bo.sys_ptr[i + 1]
        for c in range(nrhs):
            xo, sto = O.pcg(o, k, lo[i], hi[i], 0.0, Bm[r0:r1, c], tol=1e-9, maxit=500)
            assert abs(int(it[i, c]) - sto["iters"]) <= 2
            assert np.linalg.norm(Xg[r0:r1, c] - xo) / np.linalg.norm(xo) <= 1e-6
    bo.close()


def random_spd(n, seed):
    """Random symmetric sparsity (too many distinct offsets for stored diagonals), diagonally dominant."""
    rng = np.random.default_rng(seed)
    i = rng.integers(0, n, 3 * n)
    j = rng.integers(0, n, 3 * n)
    keep = i != j
    i, j = i[keep], j[keep]
    w = -rng.uniform(0.1, 1.0, len(i))
    import scipy.sparse as sp

    A = sp.coo_matrix((np.concatenate([w, w]), (np.concatenate([i, j]), np.concatenate([j, i]))), shape=(n, n)).tocsr()
    A = A + sp.diags(np.asarray(abs(A).sum(axis=1)).ravel() + 1.0)
    A = A.tocsr()
    A.sum_duplicates()
    A.sort_indices()
    return W.CSR(n, n, A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data.astype(np.float64))


def test_batch_mixed_storage(B):
    """Systems with different storages in one batch: 7-point (4 stored diagonals),
    fracture blocks (3), and a random pattern (slice layout only)."""
    systems = [W.hetero_diffusion(8, 2.0, 5), W.dfn_schur(n_frac=3, G=12, n_traces=4, L_lo=2, L_hi=6, seed=1).a,
               random_spd(700, 3), W.hetero_diffusion(5, 1.0, 6)]
    ops, lo, hi = oracle_bounds(systems)
    k, xi, m = 6, 0.0, 8
    for nrhs in (1, 4):
        bo = B.BatchOperator(systems, nrhs=nrhs, flags=B.PP_JACOBI)
        assert B.pp_batch_get_stats(bo.handle)["diag_systems"] == 3
        B.pp_batch_setup(bo.handle, k, lo, hi, xi)
        Bm = block_rhs(bo.sys_ptr, nrhs, 90)
        X = torch.zeros(bo.n, nrhs, dtype=torch.float64, device="cuda")
        s, it, rel, stt = B.pcg_solve_batch(bo.handle, len(systems), nrhs, dev(Bm), X, 0.0, m)
        assert np.all(it == m)
        Xg = host(X)
        for i, o in enumerate(ops):
            r0, r1 = bo.sys_ptr[i], bo.sys_ptr[i + 1]
            for c in range(nrhs):
                xo, sto = O.pcg(o, k, lo[i], hi[i], xi, Bm[r0:r1, c], tol=0.0, maxit=m)
                err = np.linalg.norm(Xg[r0:r1, c] - xo) / np.linalg.norm(xo)
                assert err <= 1e-10, (i, c, err)
        bo.close()


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("nrhs", [1, 8])
def test_batch_mixed_residual(B, nrhs, layout):
    systems = members()
    ops, lo, hi = oracle_bounds(systems)
    k = 12
    bo = B.BatchOperator(systems, nrhs=nrhs, flags=B.PP_JACOBI | B.PP_MIXED | lay(B, layout))
    B.pp_batch_setup(bo.handle, k, lo, hi, 0.0)
    Bm = block_rhs(bo.sys_ptr, nrhs, 3)
    X = torch.zeros(bo.n, nrhs, dtype=torch.float64, device="cuda")
    s, it, rel, stt = B.pcg_solve_batch(bo.handle, len(systems), nrhs, dev(Bm), X, 1e-8, 500)
    assert s == B.PP_OK and np.all(rel <= 1e-8)
    assert B.pp_batch_get_stats(bo.handle)["verified"] == 1
    Xg = host(X)
    for i, o in enumerate(ops):
        r0, r1 = bo.sys_ptr[i], bo.sys_ptr[i + 1]
        for c in range(nrhs):
            b = Bm[r0:r1, c]
            x = Xg[r0:r1, c]
            res = (o.apply_raw(x) - b) * o.dis
            # the true-residual check (default in mixed mode) holds the FP64 true residual to tol
            true = np.linalg.norm(res) / np.linalg.norm(b * o.dis)
            assert true <= 1e-8, (i, c, true)
            assert rel[i, c] == pytest.approx(true, rel=1e-6)
            xo, sto = O.pcg(o, k, lo[i], hi[i], 0.0, b, tol=1e-8, maxit=500)
            assert abs(int(it[i, c]) - sto["iters"]) <= 2
    bo.close()


def test_batch_apply_matches_oracle(B):
    systems = members()
    ops, lo, hi = oracle_bounds(systems)
    nrhs, k = 3, 9
    bo = B.BatchOperator(systems, nrhs=nrhs, flags=B.PP_JACOBI)
    B.pp_batch_setup(bo.handle, k, lo, hi, 2e-3)
    R = block_rhs(bo.sys_ptr, nrhs, 11)
    Z = torch.empty(bo.n, nrhs, dtype=torch.float64, device="cuda")
    B.pp_batch_apply(bo.handle, dev(R), Z)
    Zg = host(Z)
    for i, o in enumerate(ops):
        r0, r1 = bo.sys_ptr[i], bo.sys_ptr[i + 1]
        for c in range(nrhs):
            ref = O.cheb_apply(o, k, lo[i], hi[i], 2e-3, R[r0:r1, c])
            assert np.linalg.norm(Zg[r0:r1, c] - ref) / np.linalg.norm(ref) <= 1e-12
    bo.close()


def test_batch_graph_replays_match_eager(B):
    """Captured iteration chunks replayed many times give the same iterates as eager launches,
    with eager work and synchronisations between the replays."""
    systems = members()
    ops, lo, hi = oracle_bounds(systems)
    nrhs = 8
    bo = B.BatchOperator(systems, nrhs=nrhs, flags=B.PP_JACOBI)
    B.pp_batch_setup(bo.handle, 6, lo, hi, 0.0)
    B.pp_batch_set_option(bo.handle, B.PP_OPT_CHUNK, 3)
    Bm = dev(block_rhs(bo.sys_ptr, nrhs, 21))
    results = []
    for graph in (0, 1, 1, 0, 1):
        B.pp_batch_set_option(bo.handle, B.PP_BOPT_GRAPH, graph)
        X = torch.zeros(bo.n, nrhs, dtype=torch.float64, device="cuda")
        s, it, rel, stt = B.pcg_solve_batch(bo.handle, len(systems), nrhs, Bm, X, 1e-10, 400)
        assert s == B.PP_OK
        results.append((it.copy(), host(X)))
        # unrelated eager work in between
        y = torch.randn(1000, device="cuda").sum()
        torch.cuda.synchronize()
    for it, x in results[1:]:
        assert np.array_equal(it, results[0][0])
        assert np.array_equal(x, results[0][1])
    bo.close()


def test_batch_autotune_and_zero_rhs(B, tmp_path, monkeypatch):
    from paper_2208_01339_amd import autotune

    monkeypatch.setenv("PP_AUTOTUNE_CACHE", str(tmp_path / "cache.json"))
    systems = members()
    ops, lo, hi = oracle_bounds(systems)
    nrhs = 20
    bo = B.BatchOperator(systems, nrhs=nrhs, flags=B.PP_JACOBI | B.PP_MIXED)
    B.pp_batch_setup(bo.handle, 8, lo, hi, 0.0)
    r1 = autotune.tune(bo.handle, mixed=True)
    assert r1["w"] in (32, 16, 8, 4) and not r1["cached"]
    r2 = autotune.tune(bo.handle, mixed=True)
    assert r2["cached"] and r2["w"] == r1["w"]
    Bm = block_rhs(bo.sys_ptr, nrhs, 5)
    Bm[:, 3] = 0.0  # a zero right-hand side column: x = 0, zero iterations
    X = torch.ones(bo.n, nrhs, dtype=torch.float64, device="cuda")
    s, it, rel, stt = B.pcg_solve_batch(bo.handle, len(systems), nrhs, dev(Bm), X, 1e-8, 500)
    assert s == B.PP_OK
    Xg = host(X)
    assert np.all(Xg[:, 3] == 0.0) and np.all(it[:, 3] == 0)
    assert np.all(rel[:, [0, 1, 2, 4]] <= 1e-8)
    bo.close()


def test_batch_rejects_bad_input(B):
    a = W.hetero_diffusion(5, 1.0, 0)
    b2 = W.hetero_diffusion(4, 1.0, 1)
    full, sp = W.block_diag([a, b2])
    # couple the two systems
    col = full.col.copy()
    col[0] = int(sp[1]) + 1
    with pytest.raises(B.PPError) as e:
        B.pp_create_batch(2, sp, full.nnz, dev(full.rowptr), dev(col), dev(full.val), 1, B.PP_JACOBI)
    assert e.value.status == B.PP_ERR_ARG
    for nrhs in (0, 33):
        with pytest.raises(B.PPError):
            B.pp_create_batch(2, sp, full.nnz, dev(full.rowptr), dev(full.col), dev(full.val), nrhs)
    h = B.pp_create_batch(2, sp, full.nnz, dev(full.rowptr), dev(full.col), dev(full.val), 2, B.PP_JACOBI)
    X = torch.zeros(full.n_rows, 2, dtype=torch.float64, device="cuda")
    with pytest.raises(B.PPError) as e:
        B.pcg_solve_batch(h, 2, 2, X.clone(), X, 1e-8, 10)
    assert e.value.status == B.PP_ERR_STATE
    B.pp_destroy_batch(h)


def _bench_subset():
    """Eight members of the 256-system benchmark batch: the smallest, the largest and six
    between them in size order (sides 22..126)."""
    sides = W.batch_sizes()
    order = np.argsort(sides, kind="stable")
    pick = sorted(set(int(order[int(round(q * (len(order) - 1)))]) for q in np.linspace(0.0, 1.0, 8)))
    return [(i, int(sides[i])) for i in pick]


def test_batch_benchmark_subset(B):
    """FP64 batch of eight benchmark members (up to 2M rows each): every system's iterate
    after m iterations equals its own oracle solve to 1e-10; then the mixed batch to
    tol 1e-8 as the benchmark runs it: every FP64 true residual <= 1e-8, and iteration
    counts within 2 of the plain FP64 solve of each system on the GPU.  Members finish
    at different iterations, so workgroups of finished systems are redistributed."""
    picked = _bench_subset()
    sides_all = W.batch_sizes()
    assert len(picked) == 8 and {N for _, N in picked} >= {int(sides_all.min()), int(sides_all.max())}
    systems, rhs = [], []
    for i, N in picked:
        a_i, b_i = W.batch_system(i, N)
        systems.append(a_i)
        rhs.append(b_i)
    ops, lo, hi = oracle_bounds(systems)
    k, m = 60, 3
    bo = B.BatchOperator(systems, nrhs=1, flags=B.PP_JACOBI)
    assert B.pp_batch_get_stats(bo.handle)["diag_systems"] == len(systems)
    B.pp_batch_setup(bo.handle, k, lo, hi, 0.0)
    bvec = np.concatenate(rhs).reshape(-1, 1)
    X = torch.zeros(bo.n, 1, dtype=torch.float64, device="cuda")
    s, it, rel, stt = B.pcg_solve_batch(bo.handle, len(systems), 1, dev(bvec), X, 0.0, m)
    assert np.all(it == m)
    Xg = host(X)
    for j, o in enumerate(ops):
        r0, r1 = bo.sys_ptr[j], bo.sys_ptr[j + 1]
        xo, _ = O.pcg(o, k, lo[j], hi[j], 0.0, rhs[j], tol=0.0, maxit=m)
        err = np.linalg.norm(Xg[r0:r1, 0] - xo) / np.linalg.norm(xo)
        assert err <= 1e-10, (picked[j], err)
    bo.close()
    # mixed, tol-driven, as in the benchmark
    bm = B.BatchOperator(systems, nrhs=1, flags=B.PP_JACOBI | B.PP_MIXED)
    B.pp_batch_setup(bm.handle, k, lo, hi, 0.0)
    X.zero_()
    s, it, rel, stt = B.pcg_solve_batch(bm.handle, len(systems), 1, dev(bvec), X, 1e-8, 500)
    assert s == B.PP_OK and B.pp_batch_get_stats(bm.handle)["verified"] == 1
    assert len(set(int(v) for v in it[:, 0])) > 1  # members finish at different iterations
    Xg = host(X)
    for j, o in enumerate(ops):
        r0, r1 = bm.sys_ptr[j], bm.sys_ptr[j + 1]
        res = (o.apply_raw(Xg[r0:r1, 0]) - rhs[j]) * o.dis
        assert np.linalg.norm(res) / np.linalg.norm(rhs[j] * o.dis) <= 1e-8, picked[j]
        op = B.Operator(a=systems[j], flags=B.PP_JACOBI)
        B.pp_setup(op.handle, k, lo[j], hi[j], 0.0)
        x1 = torch.zeros(r1 - r0, dtype=torch.float64, device="cuda")
        s1, it1, _ = B.pcg_solve(op.handle, dev(rhs[j]), x1, 1e-8, 500)
        assert s1 == B.PP_OK and abs(int(it[j, 0]) - it1) <= 2, (picked[j], int(it[j, 0]), it1)
        op.close()
    bm.close()
