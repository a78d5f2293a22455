#!/usr/bin/env python3
"""Benchmark: polynomial-preconditioned CG time-to-1e-8 on one MI355X.

Workload (default): 7-point heterogeneous diffusion on a 256^3 grid
(n = 16,777,216, nnz = 117,047,296), lognormal(0, sigma = 2) cell
permeability with harmonic-mean faces, rhs U[-1,1] (seed 1), Jacobi scaling,
bounds from 20 Lanczos steps, degree k in {20, 60, 120}, tol 1e-8, FP64.

One "step" is one full pcg_solve from x0 = 0 until the residual of the
Jacobi-scaled system meets ||b_hat - A_hat x_hat|| <= 1e-8 ||b_hat|| (the
paper's criterion on the scaled system, section 4.3): the recursive residual
ends the iteration and the true residual of the returned iterate is then
checked in FP64 (PP_OPT_VERIFY; one more operator application).  Every
operator application, polynomial step, reduction and the device-side
convergence logic is inside the step.  Operator creation (Jacobi scaling,
storage layout) and the Lanczos bounds are timed separately and reported, as
the paper excludes the eigenvalue estimation from its solve times.

The JSON line also carries:
  roofline      the dominant kernel: on 3-D 7-point operators the fused pair
                of Chebyshev steps (k_cheb2_stencil, two steps per launch),
                else the fused step (k_cheb).  achieved = the bytes the
                kernel must move in the storage the library holds (stored
                diagonals read once per launch, the vectors each step reads
                and writes) over its mean launch time, measured with HIP
                events on the library's stream inside the timed solves;
                frac = achieved / 8 TB/s; traffic = HBM bytes per launch from
                a committed counter summary of the same sources (null when
                the sources changed since).  csr_equiv_gbs states the same
                launch time against the bytes a plain CSR pass per step would
                move (k B_A + 8n(4k-3)) / k, B_A = 12 nnz + 4(n+1): a rate of
                the method's work, not of HBM;
  general       the sliced (general sparse) path: the same 256^3 operator held
                entirely in the 64-row-slice layout (PP_SLICED), and an
                irregular SPD operator of 4.1M rows (workloads.irregular_fe,
                no shared column offsets) that the stored-diagonal layout
                rejects; solve times and a roofline record for k_cheb;
  poisson32     the 32^3 Poisson case at k = 10: a cache-resident working set
                (about 4 MB), so its rate is "effective GB/s", not HBM;
  cpu_baseline  the CPU oracle (its OpenMP build, all host threads) on the
                headline solve at k = 20: the whole solve when a probe of two
                iterations projects it under a minute, else a stated bounded
                sample scaled per operator application;
  mixed         the same solve with the polynomial in FP32 (PP_MIXED), its
                FP64 true residual (checked by the library) and its distance
                to the FP64 solution;
  batch256      256 uneven heterogeneous systems (sides 22..126) solved as one
                batch (FP32 polynomial, FP64 CG) against the same systems
                solved one by one in plain FP64;
  learned       the bounds MLP: features + forward time against 20 Lanczos
                steps, mean PCG iterations at k = 40 with the predicted
                (lambda_min, lambda_max, xi) against Lanczos bounds with
                xi = 0 on held-out operators, the fallback rate, and the
                training time of the library's kernels on a small labelled
                set made in the run;
  newton        the same solve with the Newton form of Algorithm 1 at degrees
                15 and 63 against the three-term form at the same degrees;
  dfn_su        the DFN Schur complement S_u of section 4.2 (Algorithms 3 and 4;
                400 fractures of 48 x 48, n_u = 55,132): iterations, time and
                S_u applications at the degrees of Table tab11 (xi = 1e-3),
                the rank-one correction at degree 31, and the recovery of h, p;
  lowrank       the same solve, the DFN one and the Poisson 32^3 one (k = 10)
                with the spectral low-rank correction of section 3.1 from
                Ritz vectors of 64 Lanczos steps, ranks 1 and 4 (3 for
                Poisson), xi in {0, 1e-2}, against no correction.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "PCG time-to-1e-8 residual (s) + p_k(A)v HBM GB/s; mixed/batched vs plain FP64"
HBM_PEAK_GBS = 8000.0
TRAFFIC_SUMMARY = "k_cheb2_stencil_fp64_hetero256_k20_hbm_counters.txt"
SLICED_TRAFFIC = {1: "k_cheb_lt_fp64_sliced256_k20_hbm_counters.txt",
                  0: "k_cheb_fp64_sliced256_plain_k20_hbm_counters.txt"}
IRREGULAR_TRAFFIC = "k_cheb_fp64_irregular160_k20_hbm_counters.txt"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def csr_diagonal(a):
    """diag(A) of a CSR matrix (for reporting the scaled true residual)."""
    rows = np.repeat(np.arange(a.n_rows, dtype=np.int64), np.diff(a.rowptr))
    m = a.col == rows
    return np.bincount(rows[m], weights=a.val[m], minlength=a.n_rows)


def cheb_bytes_per_step(n, nnz, k, fp32=False):
    """Algorithmic HBM bytes of one fused Chebyshev step, averaged over the k steps of p_k(A) r."""
    if fp32:
        ba = 8 * nnz + 4 * (n + 1)
        vec = 4
    else:
        ba = 12 * nnz + 4 * (n + 1)
        vec = 8
    if k <= 0:
        return 0.0
    # step 1 reads r and writes s_1; step 2 reads s_1, r; steps >= 3 read s_{j-1}, r, s_{j-2}
    total = k * ba + vec * n * (4 * k - 3) if k >= 2 else ba + 2 * vec * n
    return total / k


def stored_bytes_per_step(n, stats, k, fp32=False):
    """Bytes one fused step reads and writes in the storage the library chose.

    Symmetric stored diagonals (d arrays of n padded to whole 64-row slices),
    the sliced remainder (value + int32 column per stored entry, one int64
    offset per slice), and the vector traffic of the step.
    """
    vb = 4 if fp32 else 8
    npad = -(-n // 64) * 64
    mat = vb * stats["diagonals"] * npad
    if stats["nnz_stored"] > 0:
        mat += (vb + 4) * stats["nnz_stored"] + 8 * (npad // 64 + 1)
    total = k * mat + vb * n * (4 * k - 3) if k >= 2 else mat + 2 * vb * n
    return total / k


def schur_bytes_per_step(n, nnz_a, nt, nnz_c, k):
    """Algorithmic bytes of one fused step with the never-assembled S = A_ff + C^T M^-1 C (FP64).

    A_ff in CSR (12 nnz + 4(n+1)), C read twice (trace phase and transpose
    scatter, 12 nnz_c each, one row structure 4(nt+1)), the trace vector w
    written and read and M read (24 nt), plus the vector traffic of the
    Chebyshev step (as for a CSR operator).
    """
    bop = 12 * nnz_a + 4 * (n + 1) + 24 * nnz_c + 4 * (nt + 1) + 24 * nt
    total = k * bop + 8 * n * (4 * k - 3) if k >= 2 else bop + 16 * n
    return total / k


def run_dfn(args, B, W, torch, dev):
    """DFN-shaped Schur operator (2000 fractures of 64 x 64 cells, 5000 traces), degree dfn_k."""
    t0 = time.perf_counter()
    s, b = W.config_dfn()
    n, nt = s.n, s.nt
    up = lambda x: torch.from_numpy(x).to(dev)
    h = B.pp_create_schur(n, s.a.nnz, up(s.a.rowptr), up(s.a.col), up(s.a.val), nt, s.c.nnz,
                          up(s.c.rowptr), up(s.c.col), up(s.c.val), up(s.m), B.PP_JACOBI)
    t_create = time.perf_counter() - t0
    lmin, lmax = B.pp_estimate_bounds(h, 20)
    B.pp_set_option(h, B.PP_OPT_TIMING, 1)
    k = args.dfn_k
    B.pp_setup(h, k, lmin, lmax, args.xi)
    bd = up(b)
    x = torch.zeros(n, dtype=torch.float64, device=dev)
    for _ in range(args.warmup):
        x.zero_()
        B.pcg_solve(h, bd, x, args.tol, args.maxit)
    torch.cuda.synchronize()
    cms, csteps = 0.0, 0
    tt0 = time.perf_counter()
    for _ in range(args.steps):
        x.zero_()
        status, it, rel = B.pcg_solve(h, bd, x, args.tol, args.maxit)
        st = B.pp_get_stats(h)
        cms += st["cheb_ms"]
        csteps += st["cheb_steps"]
    torch.cuda.synchronize()
    tsolve = (time.perf_counter() - tt0) / max(1, args.steps)
    step_us = 1000.0 * cms / max(1, csteps)
    bps = schur_bytes_per_step(n, s.a.nnz, nt, s.c.nnz, k)
    # stored: diagonals + sliced trace columns, plus the trace phase (C read, w written and read)
    sbps = stored_bytes_per_step(n, st, k) + 12 * s.c.nnz + 8 * (nt + 1) + 16 * nt
    out = dict(workload="dfn_schur_2000x64x64_5000traces_jacobi", n=n, nt=nt, nnz_a=s.a.nnz, nnz_c=s.c.nnz,
               k=k, s_per_solve=tsolve, iters=it, relres=rel, status=B.pp_status_str(status),
               bounds=[lmin, lmax], step_us=step_us, step_csr_equiv_gbs=bps / (step_us * 1e-6) / 1e9,
               create_s=t_create, nnz_stored=st["nnz_stored"], diagonals=st["diagonals"],
               stored_bytes_per_step=int(sbps), stored_gbs=sbps / (step_us * 1e-6) / 1e9,
               step_frac_hbm=sbps / (step_us * 1e-6) / 1e9 / HBM_PEAK_GBS)
    log("dfn k=%d: %.3f s/solve, iters %d, step %.1f us (%.0f GB/s stored)"
        % (k, tsolve, it, step_us, out["stored_gbs"]))
    if not args.no_lowrank:
        out["lowrank"] = lowrank_leg(B, torch, h, bd, x, k, lmin, lmax, args.tol, args.maxit)
    B.pp_destroy(h)
    return out


def run_dfn_su(args, B, W, torch, dev):
    """The DFN Schur complement S_u of section 4.2 (400 fractures of 48 x 48 cells,
    1100 traces: n_h = 921,600, n_u = 55,132, the sizes of the paper's DFN test
    case #1): reduced right-hand side, PCG on D_S^{-1/2} S_u D_S^{-1/2} at the
    degrees of Table tab11 (xi = 1e-3), recovery of h and p.  The time of one
    S_u application (Algorithm 3) is the solve time over the operator
    applications."""
    t0 = time.perf_counter()
    P = W.dfn_su()
    t_gen = time.perf_counter() - t0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    op = B.Operator(dfn=P)
    torch.cuda.synchronize()
    t_create = time.perf_counter() - t0
    h = op.handle
    t0 = time.perf_counter()
    lmin, lmax = B.pp_estimate_bounds(h, 20)
    t_bounds = time.perf_counter() - t0
    q = torch.from_numpy(W.rhs_uniform(P.n_h, 1)).to(dev)
    r = torch.empty(P.n_u, dtype=torch.float64, device=dev)
    B.pp_dfn_rhs(h, q, r)
    u = torch.zeros(P.n_u, dtype=torch.float64, device=dev)
    xi = 1e-3
    rows = []
    for k in args.dfn_su_ks:
        B.pp_setup(h, k, lmin, lmax, xi)
        u.zero_()
        B.pcg_solve(h, r, u, args.tol, args.maxit)
        u.zero_()
        torch.cuda.synchronize()
        s0 = time.perf_counter()
        status, it, rel = B.pcg_solve(h, r, u, args.tol, args.maxit)
        torch.cuda.synchronize()
        ts = time.perf_counter() - s0
        st = B.pp_get_stats(h)
        rows.append(dict(k=k, iters=it, s_per_solve=ts, op_applies=st["op_applies"], dots=st["dots"],
                         us_per_su_apply=1e6 * ts / max(1, st["op_applies"]), relres=rel,
                         status=B.pp_status_str(status)))
        log("dfn S_u k=%d: %d iters, %.3f s, %d S_u applications (%.0f us each), %d dots"
            % (k, it, ts, st["op_applies"], rows[-1]["us_per_su_apply"], st["dots"]))
    best = min(rows, key=lambda x: x["s_per_solve"])
    B.pp_setup(h, best["k"], lmin, lmax, xi)
    u.zero_()
    B.pcg_solve(h, r, u, args.tol, args.maxit)
    hh = torch.empty(P.n_h, dtype=torch.float64, device=dev)
    pp = torch.empty_like(hh)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B.pp_dfn_recover(h, q, u, hh, pp)
    t_rec = time.perf_counter() - t0
    # residual of the mass balance A h - C u = q (sparse product on the device)
    a = P.a.to_scipy().tocsr()
    c = P.c.to_scipy().tocsr()
    mb = a @ hh.cpu().numpy() - c @ u.cpu().numpy() - q.cpu().numpy()
    mb_rel = float(np.linalg.norm(mb) / np.linalg.norm(q.cpu().numpy()))
    lowrank = None
    if not args.no_lowrank:
        # the leftmost eigenvector from 64 Lanczos steps on the degree-31 preconditioner
        B.pp_setup(h, 31, lmin, lmax, xi)
        B.pp_set_option(h, B.PP_OPT_RITZ, 1)
        th = B.pp_lowrank_ritz(h, 64, 1)
        _, res = B.pp_lowrank_info(h)
        u.zero_()
        torch.cuda.synchronize()
        s0 = time.perf_counter()
        status, it, rel = B.pcg_solve(h, r, u, args.tol, args.maxit)
        torch.cuda.synchronize()
        st = B.pp_get_stats(h)
        lowrank = dict(k=31, rank=1, iters=it, s_per_solve=time.perf_counter() - s0, op_applies=st["op_applies"],
                       dots=st["dots"], ritz_value=float(th[0]), ritz_residual=float(res[0]),
                       ritz="64 Lanczos steps on p_31(S-hat)", status=B.pp_status_str(status))
        log("dfn S_u k=31 rank-one correction: %d iters, %d S_u applications, %d dots (Ritz residual %.1e)"
            % (it, st["op_applies"], st["dots"], res[0]))
        B.pp_lowrank_set(h, 0)
        B.pp_set_option(h, B.PP_OPT_RITZ, 0)
    # factor bytes per application: two solves, each a forward and a backward sweep over the
    # step-ordered coefficients (G doubles per row) plus 1/L(i,i)^2 in the forward sweep
    fbytes = 4 * P.n_h * P.grid * 8 + 2 * P.n_h * 8
    out = dict(workload="dfn_su_400x48x48_1100traces_alpha1", n_h=P.n_h, n_u=P.n_u, n_frac=P.n_frac, grid=P.grid,
               nnz=dict(a=P.a.nnz, gh=P.gh.nnz, c=P.c.nnz, b=P.b.nnz, gu=P.gu.nnz), xi=xi,
               bounds=[lmin, lmax], gen_s=t_gen, create_s=t_create, bounds_s=t_bounds, per_k=rows,
               best_k=best["k"], s_per_solve=best["s_per_solve"], recover_s=t_rec, mass_balance_relres=mb_rel,
               lowrank=lowrank, factor_bytes_per_apply=fbytes,
               factor_gbs=fbytes / (best["us_per_su_apply"] * 1e-6) / 1e9)
    op.close()
    return out


def run_block(args, B, W, torch, dev, a, lmin, lmax, fp64_single):
    """32 right-hand sides on the 256^3 operator: FP32 block polynomial, FP64 CG per column."""
    from paper_2208_01339_amd import autotune

    n, nnz = a.n_rows, a.nnz
    nrhs, k = args.block_rhs, args.block_k
    sp = np.array([0, n], dtype=np.int64)
    h = B.pp_create_batch(1, sp, nnz, torch.from_numpy(a.rowptr).to(dev), torch.from_numpy(a.col).to(dev),
                          torch.from_numpy(a.val).to(dev), nrhs, B.PP_JACOBI | B.PP_MIXED)
    B.pp_batch_setup(h, k, np.array([lmin]), np.array([lmax]), args.xi)
    tune = autotune.tune(h, mixed=True)
    Bm = torch.from_numpy(W.block_rhs(n, nrhs, 3000)).to(dev)
    X = torch.zeros(n, nrhs, dtype=torch.float64, device=dev)
    B.pcg_solve_batch(h, 1, nrhs, Bm, X, args.tol, args.maxit)  # warm-up (captures the graph)
    torch.cuda.synchronize()
    times = []
    for _ in range(max(1, min(args.steps, 3))):
        X.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s, it, rel, stt = B.pcg_solve_batch(h, 1, nrhs, Bm, X, args.tol, args.maxit)
        times.append(time.perf_counter() - t0)
    tb = float(np.median(times))
    st = B.pp_batch_get_stats(h)
    B.pp_destroy_batch(h)
    single = fp64_single(k)
    out = dict(workload="hetero_diffusion_256^3_%drhs_jacobi" % nrhs, nrhs=nrhs, k=k, dtype="f32 polynomial, f64 CG",
               s_per_solve=tb, s_per_rhs=tb / nrhs, iters_max=int(it.max()), iters_min=int(it.min()),
               relres_max=float(rel.max()), verified=st["verified"], restarts=st["restarts"],
               status=B.pp_status_str(s), layout_w=st["w"], autotune=tune, runs=len(times),
               fp64_single_s=single, fp64_sequential_s=single * nrhs,
               speedup_vs_fp64_sequential=single * nrhs / tb)
    log("block %d rhs k=%d: %.3f s (%.4f s per rhs), iters %d..%d, vs %d sequential FP64 solves %.2fx"
        % (nrhs, k, tb, tb / nrhs, it.min(), it.max(), nrhs, out["speedup_vs_fp64_sequential"]))
    return out


def run_batch256(args, B, W, torch, dev):
    """256 uneven heterogeneous systems (n ~ U[1e4, 2e6]) in one batched solve vs one-at-a-time FP64."""
    t0 = time.perf_counter()
    sides = W.batch_sizes()
    systems, rhs = [], []
    for i, N in enumerate(sides):
        a_i, b_i = W.batch_system(i, int(N))
        systems.append(a_i)
        rhs.append(b_i)
    full, sp = W.block_diag(systems)
    bvec = np.concatenate(rhs)
    log("batch256: generated n=%d nnz=%d in %.0fs" % (full.n_rows, full.nnz, time.perf_counter() - t0))
    k = args.block_k
    h = B.pp_create_batch(len(systems), sp, full.nnz, torch.from_numpy(full.rowptr).to(dev),
                          torch.from_numpy(full.col).to(dev), torch.from_numpy(full.val).to(dev), 1,
                          B.PP_JACOBI | B.PP_MIXED)
    del full
    lo, hi = B.pp_batch_estimate_bounds(h, len(systems), 20)
    B.pp_batch_setup(h, k, lo, hi, args.xi)
    bd = torch.from_numpy(bvec).to(dev).reshape(-1, 1)
    X = torch.zeros_like(bd)
    B.pcg_solve_batch(h, len(systems), 1, bd, X, args.tol, args.maxit)
    times = []
    for _ in range(max(1, min(args.steps, 3))):
        X.zero_()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        s, it, rel, stt = B.pcg_solve_batch(h, len(systems), 1, bd, X, args.tol, args.maxit)
        times.append(time.perf_counter() - t1)
    tb = float(np.median(times))
    bst = B.pp_batch_get_stats(h)
    # the same solve as one persistent launch (no host round trip, workgroup map fixed)
    B.pp_batch_set_option(h, B.PP_BOPT_DRIVER, 1)
    B.pcg_solve_batch(h, len(systems), 1, bd, X, args.tol, args.maxit)
    ptimes = []
    for _ in range(max(1, min(args.steps, 3))):
        X.zero_()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        sp_, itp, relp, _ = B.pcg_solve_batch(h, len(systems), 1, bd, X, args.tol, args.maxit)
        ptimes.append(time.perf_counter() - t1)
    pst = B.pp_batch_get_stats(h)
    persistent = dict(s_per_solve=float(np.median(ptimes)), iters_max=int(itp.max()), relres_max=float(relp.max()),
                      verified=pst["verified"], status=B.pp_status_str(sp_), grid=pst["grid"],
                      map_entries=bst["grid"])
    B.pp_destroy_batch(h)
    # plain FP64, one system at a time, same bounds and degree
    tseq = 0.0
    for i, a_i in enumerate(systems):
        op = B.Operator(a=a_i, flags=B.PP_JACOBI)
        B.pp_setup(op.handle, k, lo[i], hi[i], args.xi)
        bi = torch.from_numpy(rhs[i]).to(dev)
        xi = torch.zeros_like(bi)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        B.pcg_solve(op.handle, bi, xi, args.tol, args.maxit)
        tseq += time.perf_counter() - t2
        op.close()
    out = dict(workload="batch256_hetero_uneven_sides%d-%d" % (int(sides.min()), int(sides.max())),
               nsys=len(systems), n=int(sp[-1]), k=k, dtype="f32 polynomial, f64 CG", s_per_solve=tb,
               runs=len(times), iters_max=int(it.max()), iters_min=int(it.min()),
               relres_max=float(rel.max()), verified=bst["verified"], restarts=bst["restarts"],
               graph=bst["graph"], status=B.pp_status_str(s), fp64_sequential_s=tseq,
               speedup_vs_fp64_sequential=tseq / tb,
               driver="chunks of CG iterations captured once as a hipGraph and replayed; the host polls the "
                      "done counter one chunk behind and redistributes workgroups of finished systems",
               persistent=persistent)
    log("batch256: %.2f s batched vs %.2f s sequential FP64 (%.2fx); one persistent launch %.2f s (%d workgroups "
        "over %d map entries)" % (tb, tseq, tseq / tb, persistent["s_per_solve"], persistent["grid"],
                                  persistent["map_entries"]))
    out["small_systems"] = run_batch_small(args, B, W, torch, dev)
    return out


def run_batch_small(args, B, W, torch, dev):
    """Batches of 256 small heterogeneous systems (the uneven batch's generator), sides 4..8
    (68 k rows: every phase a few microseconds of work) and 8..24 (1.3 M rows: bandwidth
    bound again); host-driven chunks against one persistent launch, FP64, k = 20."""
    return [batch_small_case(args, B, W, torch, dev, lo, hi, seed) for lo, hi, seed in ((4, 8, 7), (8, 24, 5))]


def batch_small_case(args, B, W, torch, dev, smin, smax, seed):
    sides = np.random.default_rng(seed).integers(smin, smax + 1, 256)
    systems, rhs = [], []
    for i, N in enumerate(sides):
        a_i, b_i = W.batch_system(i, int(N))
        systems.append(a_i)
        rhs.append(b_i)
    full, sp = W.block_diag(systems)
    h = B.pp_create_batch(len(systems), sp, full.nnz, torch.from_numpy(full.rowptr).to(dev),
                          torch.from_numpy(full.col).to(dev), torch.from_numpy(full.val).to(dev), 1, B.PP_JACOBI)
    lo, hi = B.pp_batch_estimate_bounds(h, len(systems), 20)
    k = 20
    B.pp_batch_setup(h, k, lo, hi, 0.0)
    bd = torch.from_numpy(np.concatenate(rhs)).to(dev).reshape(-1, 1)
    X = torch.zeros_like(bd)
    rec = {}
    for name, drv in (("chunks", 0), ("persistent", 1)):
        B.pp_batch_set_option(h, B.PP_BOPT_DRIVER, drv)
        B.pcg_solve_batch(h, len(systems), 1, bd, X, args.tol, args.maxit)
        ts = []
        for _ in range(5):
            X.zero_()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            s, it, rel, _ = B.pcg_solve_batch(h, len(systems), 1, bd, X, args.tol, args.maxit)
            ts.append(time.perf_counter() - t1)
        st = B.pp_batch_get_stats(h)
        rec[name] = dict(s_per_solve=float(np.median(ts)), iters_max=int(it.max()), status=B.pp_status_str(s),
                         grid=st["grid"])
    B.pp_destroy_batch(h)
    out = dict(workload="batch256_hetero_sides%d-%d" % (smin, smax), nsys=len(systems), n=int(sp[-1]), k=k,
               dtype="f64", **rec)
    log("batch256 sides %d..%d (n=%d): chunks %.2f ms, one persistent launch %.2f ms (%d workgroups), %d iterations "
        "at most" % (smin, smax, int(sp[-1]), 1e3 * rec["chunks"]["s_per_solve"], 1e3 * rec["persistent"]["s_per_solve"],
                     rec["persistent"]["grid"], rec["persistent"]["iters_max"]))
    return out


def stream_probes(torch, dev, nbytes=1 << 30, reps=5):
    """Achievable HBM rates on this GPU, measured in this run with plain PyTorch
    kernels on 1 GiB arrays (best of reps): a device copy (one read, one write)
    and addcmul (three reads, one write, the read/write mix of the fused pair)."""
    n = nbytes // 8
    a = torch.empty(n, dtype=torch.float64, device=dev).fill_(1.0)
    b = torch.empty_like(a).fill_(2.0)
    c = torch.empty_like(a).fill_(3.0)
    d = torch.empty_like(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def best(fn, moved):
        t = []
        for _ in range(reps):
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            t.append(e0.elapsed_time(e1) * 1e-3)
        return round(moved / min(t) / 1e9, 1)

    out = {"copy_gbs": best(lambda: d.copy_(a), 2 * 8 * n),
           "read3_write1_gbs": best(lambda: torch.addcmul(a, b, c, out=d), 4 * 8 * n),
           "note": "plain PyTorch kernels on 1 GiB FP64 arrays, best of %d: the streaming rates a kernel reaches "
                   "on this part, against the 8 TB/s peak" % reps}
    del a, b, c, d
    torch.cuda.synchronize()
    return out


def timed_solves(B, torch, h, bd, x, tol, maxit, warmup, runs):
    """warmup + runs solves from x0 = 0; returns (median s, status, iters, relres, stats of the last)."""
    for _ in range(warmup):
        x.zero_()
        B.pcg_solve(h, bd, x, tol, maxit)
    times, cms, csteps = [], 0.0, 0
    for _ in range(runs):
        x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        status, it, rel = B.pcg_solve(h, bd, x, tol, maxit)
        times.append(time.perf_counter() - t0)
        st = B.pp_get_stats(h)
        cms += st["cheb_ms"]
        csteps += st["cheb_steps"]
    st["step_us"] = 1000.0 * cms / max(1, csteps)
    return float(np.median(times)), status, it, rel, st


def sliced_roofline(n, nnz, st, k, what, lds_tiles=0):
    """Roofline record of the one-step kernel on an operator held in the slice layout: k_cheb_lt
    (x staged in LDS per tile, 8-byte value + 2-byte staging index per slot, x read once per
    tile) or k_cheb (8-byte value + 4-byte column per slot)."""
    if lds_tiles:
        npad = -(-n // 64) * 64
        sb = 10 * st["nnz_stored"] + 8 * (npad // 64 + 1) + 8 * n * (4 * k - 3) / k
        kern = "k_cheb_lt (fused SpMV + Chebyshev step, 64-row slices, x staged in LDS per tile, FP64): "
    else:
        sb = stored_bytes_per_step(n, st, k)
        kern = "k_cheb (fused SpMV + Chebyshev step, 64-row slices, FP64): "
    us = st["step_us"]
    ach = sb / (us * 1e-6) / 1e9
    return {"bound": "hbm", "kernel": kern + what,
            "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
            "bytes_per_launch": int(sb), "mean_launch_us": round(us, 2),
            "csr_equiv_gbs": round(cheb_bytes_per_step(n, nnz, k) / (us * 1e-6) / 1e9, 1),
            "storage": "%d stored diagonals + %d sliced entries" % (st["diagonals"], st["nnz_stored"])}


def run_general(args, B, W, torch, dev, a, bd, lmin, lmax):
    """The sliced (general sparse) path: the 256^3 operator under PP_SLICED, and an
    irregular operator the stored-diagonal layout rejects; k = 20, tol 1e-8."""
    out = {}
    k, runs = 20, max(1, min(args.steps, 3))
    n, nnz = a.n_rows, a.nnz
    up = lambda v: torch.from_numpy(v).to(dev)
    h = B.pp_create_csr(n, nnz, up(a.rowptr), up(a.col), up(a.val), B.PP_JACOBI | B.PP_SLICED)
    B.pp_set_option(h, B.PP_OPT_TIMING, 1)
    B.pp_setup(h, k, lmin, lmax, args.xi)
    x = torch.zeros(n, dtype=torch.float64, device=dev)
    ts, status, it, rel, st = timed_solves(B, torch, h, bd, x, args.tol, args.maxit, 1, runs)
    out["hetero256_sliced"] = dict(k=k, s_per_solve=ts, iters=it, relres=rel, status=B.pp_status_str(status),
                                   lds_tiles=st["lds_tiles"],
                                   roofline=with_traffic(
                                       sliced_roofline(n, nnz, st, k, "256^3 operator, every entry sliced",
                                                       st["lds_tiles"]),
                                       committed_traffic(args, n, k, SLICED_TRAFFIC[st["lds_tiles"]])))
    if st["lds_tiles"]:
        B.pp_set_option(h, B.PP_OPT_LDS_TILES, 0)
        ts0, _, _, _, st0_ = timed_solves(B, torch, h, bd, x, args.tol, args.maxit, 1, runs)
        out["hetero256_sliced"]["without_lds_tiles"] = dict(s_per_solve=ts0, step_us=st0_["step_us"])
    log("general: 256^3 sliced k=%d: %.3f s/solve, %d iters, step %.1f us (%.0f GB/s stored)"
        % (k, ts, it, st["step_us"], out["hetero256_sliced"]["roofline"]["achieved"]))
    B.pp_destroy(h)
    del x
    t0 = time.perf_counter()
    g = W.irregular_fe(args.general_N)
    t_gen = time.perf_counter() - t0
    b = W.rhs_uniform(g.n_rows, 1)
    t0 = time.perf_counter()
    h = B.pp_create_csr(g.n_rows, g.nnz, up(g.rowptr), up(g.col), up(g.val), B.PP_JACOBI)
    torch.cuda.synchronize()
    t_create = time.perf_counter() - t0
    st0 = B.pp_get_stats(h)
    lo, hi = B.pp_estimate_bounds(h, 20)
    B.pp_set_option(h, B.PP_OPT_TIMING, 1)
    B.pp_setup(h, k, lo, hi, args.xi)
    bg = up(b)
    x = torch.zeros(g.n_rows, dtype=torch.float64, device=dev)
    ts, status, it, rel, st = timed_solves(B, torch, h, bg, x, args.tol, args.maxit, 1, runs)
    no_lt = None
    if st["lds_tiles"]:
        B.pp_set_option(h, B.PP_OPT_LDS_TILES, 0)
        ts0, _, _, _, st0_ = timed_solves(B, torch, h, bg, x, args.tol, args.maxit, 1, runs)
        no_lt = dict(s_per_solve=ts0, step_us=st0_["step_us"])
        B.pp_set_option(h, B.PP_OPT_LDS_TILES, 1)
    row_len = np.diff(g.rowptr)
    out["irregular"] = dict(workload="irregular_fe_%d^3_27pt_thinned0.8_window4096_jacobi" % args.general_N,
                            n=g.n_rows, nnz=g.nnz, row_len_min=int(row_len.min()), row_len_max=int(row_len.max()),
                            diagonals=st0["diagonals"], gen_s=round(t_gen, 1), create_s=round(t_create, 3),
                            bounds=[lo, hi], k=k, s_per_solve=ts, iters=it, relres=rel,
                            status=B.pp_status_str(status), reordered=st0["reordered"],
                            gather_spread=st0["gather_spread"], lds_tiles=st["lds_tiles"],
                            without_lds_tiles=no_lt,
                            roofline=with_traffic(
                                sliced_roofline(g.n_rows, g.nnz, st, k, "irregular operator, %.1fM rows"
                                                % (g.n_rows / 1e6), st["lds_tiles"]),
                                None if st["lds_tiles"] else committed_traffic(args, g.n_rows, k,
                                                                               IRREGULAR_TRAFFIC)))
    log("general: irregular n=%d nnz=%d (%d stored diagonals) k=%d: %.3f s/solve, %d iters, step %.1f us "
        "(%.0f GB/s stored)" % (g.n_rows, g.nnz, st0["diagonals"], k, ts, it, st["step_us"],
                                out["irregular"]["roofline"]["achieved"]))
    B.pp_destroy(h)
    return out


def run_poisson32(args, B, W, torch, dev):
    """The 32^3 Poisson case (k = 10, Jacobi off): its working set (about 4 MB) stays in the
    caches, so the step rate is an effective, cache-resident one."""
    a, b = W.config_poisson32()
    up = lambda v: torch.from_numpy(v).to(dev)
    h = B.pp_create_csr(a.n_rows, a.nnz, up(a.rowptr), up(a.col), up(a.val), 0)
    lo, hi = B.pp_estimate_bounds(h, 20)
    B.pp_set_option(h, B.PP_OPT_TIMING, 1)
    B.pp_setup(h, 10, lo, hi, 0.0)
    x = torch.zeros(a.n_rows, dtype=torch.float64, device=dev)
    # the default driver (persistent at this size) and the stream-driven kernels (with step events)
    ts, status, it, rel, st = timed_solves(B, torch, h, up(b), x, args.tol, args.maxit, 5, 20)
    B.pp_set_option(h, B.PP_OPT_DRIVER, 0)
    ts0, _, it0, _, st0 = timed_solves(B, torch, h, up(b), x, args.tol, args.maxit, 5, 20)
    B.pp_destroy(h)
    eff = cheb_bytes_per_step(a.n_rows, a.nnz, 10) / (st0["step_us"] * 1e-6) / 1e9
    out = dict(workload="poisson3d_32^3_k10", n=a.n_rows, nnz=a.nnz, bounds=[lo, hi], k=10, s_per_solve=ts,
               iters=it, relres=rel, status=B.pp_status_str(status),
               driver="persistent" if st["driver"] == 1 else "stream", grid=st["grid"],
               barrier={0: "runtime", 1: "flat", 2: "two-level"}.get(st["barrier"], None),
               stream_driver=dict(s_per_solve=ts0, iters=it0, step_us=st0["step_us"],
                                  effective_gbs_cache_resident=eff))
    log("poisson32 k=10: %.2f ms/solve (%s driver, %d workgroups, %s barrier), %d iters; stream-driven %.2f ms, "
        "step %.1f us (%.0f GB/s effective, cache-resident)" % (1000 * ts, out["driver"], st["grid"], out["barrier"],
                                                              it, 1000 * ts0, st0["step_us"], eff))
    # 64^3: past the default driver's size limit; both drivers, same bounds recipe
    a6 = W.poisson3d(64)
    b6 = W.rhs_uniform(a6.n_rows, 0)
    h = B.pp_create_csr(a6.n_rows, a6.nnz, up(a6.rowptr), up(a6.col), up(a6.val), 0)
    lo6, hi6 = B.pp_estimate_bounds(h, 20)
    B.pp_setup(h, 10, lo6, hi6, 0.0)
    x6 = torch.zeros(a6.n_rows, dtype=torch.float64, device=dev)
    rec = {}
    for name, drv in (("stream", 0), ("persistent", 1)):
        B.pp_set_option(h, B.PP_OPT_DRIVER, drv)
        t6, s6, it6, _, st6 = timed_solves(B, torch, h, up(b6), x6, args.tol, args.maxit, 3, 10)
        rec[name] = dict(s_per_solve=t6, iters=it6, status=B.pp_status_str(s6), grid=st6["grid"])
    B.pp_destroy(h)
    out["poisson64"] = dict(workload="poisson3d_64^3_k10", n=a6.n_rows, **rec)
    log("poisson64 k=10: stream-driven %.2f ms/solve, persistent %.2f ms (%d workgroups), %d iters"
        % (1000 * rec["stream"]["s_per_solve"], 1000 * rec["persistent"]["s_per_solve"], rec["persistent"]["grid"],
           rec["stream"]["iters"]))
    return out


def run_learned(args, B, W, torch, dev):
    """The bounds MLP (committed weights, trained on 5000 operators) on held-out operators of
    the evaluation set, and the training time of the library's kernels on operators labelled
    in this run."""
    from paper_2208_01339_amd import learned as L

    m = L.Model.load()
    seed = 1 + 7919  # the held-out set (learned.py evaluate)
    rows = []
    for i in range(args.learned_eval):
        d = L.sample_operator(i, seed)
        op = B.Operator(a=d["a"], schur=d["schur"], flags=B.PP_JACOBI)
        bv = torch.from_numpy(W.rhs_uniform(d["n"], 30_000 + i + seed)).to(dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lo_p, hi_p, xi_p, fb = B.pp_predict_bounds(op.handle, m.h, L.POWER_STEPS)
        t_pred = time.perf_counter() - t0
        t0 = time.perf_counter()
        lo_l, hi_l = B.pp_estimate_bounds(op.handle, 20)
        t_lz = time.perf_counter() - t0
        it_p = L._solve_iters(torch, op, bv, L.K_LABEL, lo_p, hi_p, xi_p)
        it_l = L._solve_iters(torch, op, bv, L.K_LABEL, lo_l, hi_l, 0.0)
        op.close()
        rows.append((d["kind"], it_p, it_l, fb, t_pred, t_lz))
    m.close()
    it_p = np.array([r[1] for r in rows], dtype=float)
    it_l = np.array([r[2] for r in rows], dtype=float)
    t0 = time.perf_counter()
    data = L.build_dataset(args.learned_label, 1, log=lambda *_: None)
    t_label = time.perf_counter() - t0
    epochs = 400
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    m2, hist = L.train(data, epochs=epochs, log=lambda *_: None)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    m2.close()
    kinds = np.array([r[0] for r in rows])
    out = dict(held_out=len(rows), held_out_set="learned.sample_operator(i, seed=7920), i < %d" % len(rows),
               k=L.K_LABEL, mean_iters_pred=float(it_p.mean()), mean_iters_lanczos_xi0=float(it_l.mean()),
               mean_iters_pred_7pt=float(it_p[kinds == "7pt"].mean()),
               mean_iters_lanczos_7pt=float(it_l[kinds == "7pt"].mean()),
               mean_iters_pred_dfn=float(it_p[kinds == "dfn"].mean()),
               mean_iters_lanczos_dfn=float(it_l[kinds == "dfn"].mean()),
               fallback_rate=float(np.mean([r[3] for r in rows])),
               mean_setup_s_features_forward=float(np.mean([r[4] for r in rows])),
               mean_setup_s_lanczos20=float(np.mean([r[5] for r in rows])),
               train=dict(operators_labelled=args.learned_label, label_s=round(t_label, 2), epochs=epochs,
                          batch=128, train_s=round(t_train, 3), final_loss=float(hist[-1]),
                          note="a model trained here from scratch, for the timing; the evaluated weights were "
                               "trained the same way on 5000 operators"))
    log("learned: %d held-out operators, k=%d: %.2f iterations with predicted bounds/xi vs %.2f with Lanczos "
        "and xi=0, fallback %.0f%%; %d epochs over %d operators in %.2f s"
        % (len(rows), L.K_LABEL, out["mean_iters_pred"], out["mean_iters_lanczos_xi0"],
           100 * out["fallback_rate"], epochs, args.learned_label, t_train))
    return out


def cpu_info():
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    threads = None
    try:
        import ctypes

        threads = int(ctypes.CDLL("libgomp.so.1").omp_get_max_threads())
    except OSError:
        pass
    return model, os.cpu_count(), len(os.sched_getaffinity(0)), threads


def run_cpu_baseline(args, a, b, lmin, lmax, kc, gpu_applies):
    """The oracle's OpenMP build on the headline system: the whole solve when a probe of two
    iterations projects it under a minute, else a bounded sample scaled per operator application."""
    import oracle as O

    orc = O.Operator(a, jacobi=True)
    _, pr = O.pcg(orc, kc, lmin, lmax, args.xi, b, tol=args.tol, maxit=2, omp=True)
    per_apply = pr["seconds"] / max(1, pr["n_apply"])
    model, ncpu, naff, threads = cpu_info()
    proj = per_apply * gpu_applies
    if proj <= 60.0:
        _, sto = O.pcg(orc, kc, lmin, lmax, args.xi, b, tol=args.tol, maxit=args.maxit, omp=True)
        value = sto["seconds"]
        sample = ("the whole PCG solve at k=%d (%d iterations, %d operator applications, tol %g on the scaled "
                  "system) of the same 256^3 FP64 system" % (kc, sto["iters"], sto["n_apply"], args.tol))
    else:
        its = max(2, int(30.0 / max(1e-9, per_apply * (kc + 1))))
        _, sto = O.pcg(orc, kc, lmin, lmax, args.xi, b, tol=0.0, maxit=its, omp=True)
        value = sto["seconds"] / sto["n_apply"] * gpu_applies
        sample = ("%d PCG iterations at k=%d (%d operator applications, %.1f s) of the same system, scaled per "
                  "operator application to the %d applications of the GPU's solve"
                  % (its, kc, sto["n_apply"], sto["seconds"], gpu_applies))
    cpu = {"value": round(value, 3), "unit": "s", "cores": threads or naff, "kind": "oracle-omp",
           "sample": sample, "cpu_model": model, "nproc": ncpu, "affinity_cpus": naff,
           "build": "oracle/ppcg_oracle.c, gcc -O2 -fopenmp -ffp-contract=off, static schedule"}
    log("cpu oracle (%s threads, %s): %.2f s per solve" % (cpu["cores"], model, value))
    return cpu


def bounds_leg(B, torch, h, bd, x, ks, tol, maxit, runs):
    """The headline solves with other spectral bounds than the 20 Lanczos steps: 64 Lanczos
    steps (a closer estimate of the same two numbers, which the paper takes from an
    eigensolver, section 6.1) and the learned model's (lambda_min, lambda_max, xi) for this
    operator (trained on operators of 1e4 to 1e6 rows; this one has 1.7e7).  Bounds setup
    is timed apart, as for the headline."""
    from paper_2208_01339_amd import learned as L

    out = {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    l64, h64 = B.pp_estimate_bounds(h, 64)
    t64 = time.perf_counter() - t0
    m = L.Model.load()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lp, hp, xp, fb = B.pp_predict_bounds(h, m.h, L.POWER_STEPS)
    tp = time.perf_counter() - t0
    m.close()
    for name, lo, hi, xi, ts, extra in (("lanczos64", l64, h64, 0.0, t64, {}),
                                        ("learned", lp, hp, xp, tp, {"fallback": fb})):
        rows = []
        for k in ks:
            B.pp_setup(h, k, lo, hi, xi)
            x.zero_()
            B.pcg_solve(h, bd, x, tol, maxit)
            times = []
            for _ in range(runs):
                x.zero_()
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                st, it, rel = B.pcg_solve(h, bd, x, tol, maxit)
                torch.cuda.synchronize()
                times.append(time.perf_counter() - t1)
            rows.append(dict(k=k, iters=it, s_per_solve=round(float(np.median(times)), 4), relres=rel,
                             status=B.pp_status_str(st)))
        out[name] = dict(bounds=[lo, hi], xi=xi, setup_s=round(ts, 4), per_k=rows, **extra)
        log("bounds %s [%.4g, %.4g] xi %.2g (setup %.3f s): %s" % (
            name, lo, hi, xi, ts, ", ".join("k=%d %d iters %.3f s" % (r["k"], r["iters"], r["s_per_solve"])
                                            for r in rows)))
    return out


def lowrank_leg(B, torch, h, bd, x, k, lmin, lmax, tol, maxit, ranks=(1, 4), xis=(0.0, 1e-3), steps=None,
                ritz="poly"):
    """PCG with the spectral low-rank correction (section 3.1) against the same solve without
    it; one timed solve each.  Ritz vectors: ritz="poly" from 64 Lanczos steps on the
    preconditioner p_k(A-hat) with full reorthogonalisation (PP_OPT_RITZ = 1), "lanczos"
    from 64 plain Lanczos steps on A-hat; their relative residuals and the time to compute
    them (paid once per operator and degree) are reported."""
    if steps is None:
        steps = 64
    B.pp_set_option(h, B.PP_OPT_RITZ, 1 if ritz == "poly" else 0)
    def solve():
        x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, it, rel = B.pcg_solve(h, bd, x, tol, maxit)
        return time.perf_counter() - t0, it, B.pp_status_str(st)

    rows = []
    for xi in xis:
        B.pp_lowrank_set(h, 0)
        B.pp_setup(h, k, lmin, lmax, xi)
        solve()
        t0, it0, s0 = solve()
        for p in ranks:
            torch.cuda.synchronize()
            tr = time.perf_counter()
            th = B.pp_lowrank_ritz(h, steps, p)
            tr = time.perf_counter() - tr
            _, res = B.pp_lowrank_info(h)
            solve()
            t1, it1, s1 = solve()
            rows.append(dict(xi=xi, rank=p, ritz=ritz, ritz_steps=steps, ritz_s=round(tr, 4),
                             ritz_values=[float(v) for v in th], ritz_residuals=[float(v) for v in res],
                             iters=it1, s_per_solve=round(t1, 4), status=s1, iters_without=it0,
                             s_without=round(t0, 4)))
            log("lowrank (%s) k=%d xi=%g rank %d: %d iters %.3f s (without: %d iters %.3f s), Ritz %.3f s, "
                "residuals %s" % (ritz, k, xi, p, it1, t1, it0, t0, tr, " ".join("%.1e" % v for v in res)))
    B.pp_lowrank_set(h, 0)
    B.pp_set_option(h, B.PP_OPT_RITZ, 0)
    return rows


def committed_traffic(args, n, k, summary=TRAFFIC_SUMMARY):
    """HBM bytes per launch (per step for one-step kernels) from a committed
    rocprofv3 counter summary under profiles/.

    Null unless the summary was taken on this workload and degree from the
    kernel sources that are built now (same source digest), with the default
    launch options.
    """
    from paper_2208_01339_amd import profsum

    summ = profsum.read_summary(os.path.join(ROOT, "profiles", summary))
    try:
        ok = (summ.get("source_digest") == profsum.source_digest() and int(summ.get("n", -1)) == n
              and int(summ.get("k", -1)) == k and args.grid == 0 and args.nt_loads < 0 and args.xi == 0.0)
        return float(summ["traffic_bytes_per_launch"]) if ok else None
    except (KeyError, ValueError):
        return None


def with_traffic(roof, traffic):
    """Adds the counter-measured HBM bytes per launch (or null) to a roofline record."""
    us = roof["mean_launch_us"]
    roof["traffic"] = round(traffic) if traffic else None
    roof["traffic_gbs"] = round(traffic / (us * 1e-6) / 1e9, 1) if traffic else None
    return roof


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--N", type=int, default=256, help="grid side (n = N^3)")
    ap.add_argument("--ks", default="20,60,120")
    ap.add_argument("--xi", type=float, default=0.0)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--maxit", type=int, default=5000)
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-unscaled", action="store_true", help="skip the solve to a true unscaled 1e-8")
    ap.add_argument("--no-general", action="store_true", help="skip the sliced-layout and irregular-operator legs")
    ap.add_argument("--no-poisson32", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-bounds", action="store_true", help="skip the headline solves with other spectral bounds")
    ap.add_argument("--learned-eval", type=int, default=40, help="held-out operators of the learned leg")
    ap.add_argument("--learned-label", type=int, default=100, help="operators labelled in the run for training")
    ap.add_argument("--general-N", type=int, default=160, help="side of the irregular operator (n = N^3)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-dfn", action="store_true", help="skip the DFN-shaped Schur leg")
    ap.add_argument("--dfn-k", type=int, default=40)
    ap.add_argument("--no-block", action="store_true", help="skip the 32-RHS block leg")
    ap.add_argument("--no-lowrank", action="store_true", help="skip the low-rank correction legs")
    ap.add_argument("--no-newton", action="store_true", help="skip the Newton-form leg")
    ap.add_argument("--no-dfn-su", action="store_true", help="skip the DFN S_u leg (section 4.2)")
    ap.add_argument("--dfn-su-ks", default="0,7,15,31,63")
    ap.add_argument("--no-two-step", action="store_true",
                    help="one pass per Chebyshev step (no fused pairs) in the main leg")
    ap.add_argument("--block-rhs", type=int, default=32)
    ap.add_argument("--block-k", type=int, default=60)
    ap.add_argument("--no-batch256", action="store_true",
                    help="skip the 256-system uneven batch (about 60 GB on the device, 25 s to generate)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one plain 1 GiB device copy first (HBM counter calibration)")
    ap.add_argument("--grid", type=int, default=0, help="workgroups per launch (0 = library default)")
    ap.add_argument("--nt-loads", type=int, default=-1, help="1/0: non-temporal matrix loads (-1 = default)")
    ap.add_argument("--cpu-sample-k", type=int, default=0, help="degree of the CPU sample iteration (0 = 20)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(row-stripe sharding is described in the design notes, not built)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2208_01339_amd import binding as B
    from paper_2208_01339_amd import build as hipbuild
    from paper_2208_01339_amd import workloads as W

    if not os.path.exists(hipbuild.OUT):
        hipbuild.build(verbose=False)
    B.lib()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    ks = [int(v) for v in args.ks.split(",") if v]

    t0 = time.perf_counter()
    a, b = W.config_hetero(args.N, 2.0)
    n, nnz = a.n_rows, a.nnz
    log("generated n=%d nnz=%d in %.1fs" % (n, nnz, time.perf_counter() - t0))

    dev = torch.device("cuda:0")
    rp = torch.from_numpy(a.rowptr).to(dev)
    ci = torch.from_numpy(a.col).to(dev)
    va = torch.from_numpy(a.val).to(dev)
    bd = torch.from_numpy(b).to(dev)
    torch.cuda.synchronize()

    if args.calib_copy:
        src = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    t0 = time.perf_counter()
    h = B.pp_create_csr(n, nnz, rp, ci, va, B.PP_JACOBI)
    torch.cuda.synchronize()
    t_create = time.perf_counter() - t0
    t0 = time.perf_counter()
    lmin, lmax = B.pp_estimate_bounds(h, 20)
    t_bounds = time.perf_counter() - t0
    log("create %.2fs, Lanczos bounds [%.6g, %.6g] in %.3fs" % (t_create, lmin, lmax, t_bounds))
    st0 = B.pp_get_stats(h)
    B.pp_set_option(h, B.PP_OPT_TIMING, 1)
    B.pp_set_option(h, B.PP_OPT_VERIFY, 1)  # true residual of the scaled system checked at exit
    dis = torch.from_numpy(1.0 / np.sqrt(csr_diagonal(a))).to(dev)
    bhat_norm = float(torch.linalg.norm(bd * dis))
    if args.grid:
        B.pp_set_option(h, B.PP_OPT_GRID, args.grid)
    if args.nt_loads >= 0:
        B.pp_set_option(h, B.PP_OPT_NT_LOADS, args.nt_loads)
    if args.no_two_step:
        B.pp_set_option(h, B.PP_OPT_TWO_STEP, 0)

    x = torch.zeros(n, dtype=torch.float64, device=dev)
    per_k = []
    for k in ks:
        B.pp_setup(h, k, lmin, lmax, args.xi)
        for _ in range(args.warmup):
            x.zero_()
            B.pcg_solve(h, bd, x, args.tol, args.maxit)
        torch.cuda.synchronize()
        times, iters, rels, cheb_ms, cheb_steps, pair_ms, pairs = [], [], [], 0.0, 0, 0.0, 0
        tt0 = time.perf_counter()
        for _ in range(args.steps):
            x.zero_()
            s0 = time.perf_counter()
            status, it, rel = B.pcg_solve(h, bd, x, args.tol, args.maxit)
            times.append(time.perf_counter() - s0)
            st = B.pp_get_stats(h)
            iters.append(it)
            rels.append(rel)
            cheb_ms += st["cheb_ms"]
            cheb_steps += st["cheb_steps"]
            pair_ms += st["pair_ms"]
            pairs += st["pair_launches"]
            if status != B.PP_OK:
                log("k=%d solve status %s" % (k, B.pp_status_str(status)))
        torch.cuda.synchronize()
        wall = (time.perf_counter() - tt0) / max(1, args.steps)
        # true residuals of the last solve, with the library's unscaled operator:
        # of the scaled system (what tol refers to) and of the original one
        y = torch.empty_like(x)
        B.pp_operator_apply(h, x, y)
        torch.cuda.synchronize()
        true_rel = float(torch.linalg.norm(bd - y) / torch.linalg.norm(bd))
        true_scaled = float(torch.linalg.norm((bd - y) * dis) / bhat_norm)
        step_us = 1000.0 * cheb_ms / max(1, cheb_steps)
        bps = cheb_bytes_per_step(n, nnz, k)
        pair_us = 1000.0 * pair_ms / pairs if pairs else None
        single_us = (1000.0 * (cheb_ms - pair_ms) / (cheb_steps - 2 * pairs)
                     if cheb_steps > 2 * pairs else None)
        rec = dict(k=k, s_per_solve=wall, s_median=float(np.median(times)), iters=iters[-1], relres=rels[-1],
                   true_relres_scaled=true_scaled, true_relres_scaled_lib=st["true_relres"],
                   true_relres=true_rel, restarts=st["restarts"],
                   op_applies=st["op_applies"], cheb_step_us=step_us,
                   cheb_step_csr_equiv_gbs=bps / (step_us * 1e-6) / 1e9 if step_us > 0 else None,
                   pair_launch_us=pair_us, pair_launches=pairs // max(1, args.steps),
                   single_step_us=single_us, status=B.pp_status_str(status))
        per_k.append(rec)
        log("k=%d: %.3f s/solve, iters %d, step %.1f us, pair launch %s us, true relres scaled %.2e unscaled %.2e"
            % (k, wall, iters[-1], step_us, "%.1f" % pair_us if pair_us else "-", true_scaled, true_rel))

    best = min(per_k, key=lambda r: r["s_per_solve"])
    kh = best["k"]
    bounds = None
    if not args.no_bounds:
        bounds = bounds_leg(B, torch, h, bd, x, ks, args.tol, args.maxit, max(1, min(args.steps, 3)))
    B.pp_setup(h, kh, lmin, lmax, args.xi)

    # pp_apply alone at the headline degree (events on the library's stream = torch's current)
    r = torch.from_numpy(W.rhs_uniform(n, 7)).to(dev)
    z = torch.empty_like(r)
    B.pp_apply(h, r, z)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 3
    e0.record()
    for _ in range(reps):
        B.pp_apply(h, r, z)
    e1.record()
    torch.cuda.synchronize()
    apply_ms = e0.elapsed_time(e1) / reps
    apply_bytes = kh * (12 * nnz + 4 * (n + 1)) + 8 * n * (4 * kh - 3)
    apply_gbs = apply_bytes / (apply_ms * 1e-3) / 1e9

    # the original (unscaled) system to 1e-8 as well: tol tightened by the ratio
    # of the two true residuals measured at tol 1e-8
    unscaled = None
    if not args.no_unscaled:
        rb = best
        tol_u = args.tol * min(1.0, rb["true_relres_scaled"] / max(rb["true_relres"], 1e-300))
        for _ in range(3):
            x.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            su, itu, _ = B.pcg_solve(h, bd, x, tol_u, args.maxit)
            tu = time.perf_counter() - t0
            y = torch.empty_like(x)
            B.pp_operator_apply(h, x, y)
            tru = float(torch.linalg.norm(bd - y) / torch.linalg.norm(bd))
            if tru <= args.tol:
                break
            tol_u *= 0.7 * args.tol / tru
        unscaled = dict(k=kh, tol_scaled_used=tol_u, iters=itu, s_per_solve=tu, true_relres=tru,
                        status=B.pp_status_str(su))
        log("unscaled 1e-8: tol %.2e on the scaled system, %d iters, %.3f s, true relres %.2e"
            % (tol_u, itu, tu, tru))

    bps = cheb_bytes_per_step(n, nnz, kh)
    storage = "%d symmetric stored diagonals%s + %d sliced entries" % (
        st0["diagonals"], " (the main one exactly 1 after Jacobi scaling, not read by the pairs)"
        if st0["unit_diagonal"] else "", st0["nnz_stored"])
    if best["pair_launch_us"]:
        # two steps per launch; the operator (stored diagonals) is read once for both
        launch_us = best["pair_launch_us"]
        lb = 2 * bps
        npad = -(-n // 64) * 64
        # the stored diagonals once (a unit main diagonal is not read), r, s_{j-1}, s_{j-2}
        # read, s_j and s_{j+1} written
        sb = 8 * (st0["diagonals"] - st0["unit_diagonal"]) * npad + 5 * 8 * n
        kern = "k_cheb2_stencil (two fused Chebyshev steps per launch, FP64, symmetric stored diagonals)"
        traffic = committed_traffic(args, n, kh)
    else:
        launch_us = best["cheb_step_us"]
        lb = bps
        sb = stored_bytes_per_step(n, st0, kh)
        kern = "k_cheb (fused SpMV + Chebyshev three-term step, FP64)"
        traffic = None
    achieved = sb / (launch_us * 1e-6) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": kern, "steps_per_launch": 2 if best["pair_launch_us"] else 1,
                "bytes_per_launch": int(sb), "mean_launch_us": round(launch_us, 2),
                "traffic_gbs": round(traffic / (launch_us * 1e-6) / 1e9, 1) if traffic else None,
                "traffic_frac": round(traffic / (launch_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4) if traffic else None,
                "storage": storage,
                "csr_equiv_bytes_per_launch": int(lb),
                "csr_equiv_gbs": round(lb / (launch_us * 1e-6) / 1e9, 1),
                "single_step_us": round(best["single_step_us"], 2) if best["single_step_us"] else None,
                "note": ("bytes_per_launch: what the kernel must move in the storage held (operator once per "
                         "launch, the step vectors); csr_equiv_*: the same launch time against one plain CSR "
                         "pass per step, a rate of the method's work that can pass the HBM peak")}
    probes = stream_probes(torch, dev)
    roofline["probes"] = probes
    roofline["frac_of_copy"] = round(achieved / probes["copy_gbs"], 4)
    roofline["frac_of_read3_write1"] = round(achieved / probes["read3_write1_gbs"], 4)
    log("roofline: %.0f GB/s stored bytes (frac %.3f of 8 TB/s); this GPU streams copy %.0f GB/s, "
        "3 reads + 1 write %.0f GB/s" % (achieved, achieved / HBM_PEAK_GBS, probes["copy_gbs"],
                                          probes["read3_write1_gbs"]))

    mixed = None
    if not args.no_mixed:
        hm = B.pp_create_csr(n, nnz, rp, ci, va, B.PP_JACOBI | B.PP_MIXED)
        B.pp_set_option(hm, B.PP_OPT_TIMING, 1)
        if args.grid:
            B.pp_set_option(hm, B.PP_OPT_GRID, args.grid)
        if args.nt_loads >= 0:
            B.pp_set_option(hm, B.PP_OPT_NT_LOADS, args.nt_loads)
        B.pp_setup(hm, kh, lmin, lmax, args.xi)
        x.zero_()
        B.pcg_solve(hm, bd, x, args.tol, args.maxit)
        torch.cuda.synchronize()
        tt0 = time.perf_counter()
        cms, csteps, pms, npairs = 0.0, 0, 0.0, 0
        for _ in range(args.steps):
            x.zero_()
            status_m, it_m, rel_m = B.pcg_solve(hm, bd, x, args.tol, args.maxit)
            stm = B.pp_get_stats(hm)
            cms += stm["cheb_ms"]
            csteps += stm["cheb_steps"]
            pms += stm["pair_ms"]
            npairs += stm["pair_launches"]
        torch.cuda.synchronize()
        tm = (time.perf_counter() - tt0) / max(1, args.steps)
        y = torch.empty_like(x)
        B.pp_operator_apply(hm, x, y)
        torch.cuda.synchronize()
        tr = float(torch.linalg.norm(bd - y) / torch.linalg.norm(bd))
        trs = float(torch.linalg.norm((bd - y) * dis) / bhat_norm)
        # the FP64 solution of the same system (the solve pinned to the oracle at full size)
        B.pp_setup(h, kh, lmin, lmax, args.xi)
        x64 = torch.zeros_like(x)
        B.pcg_solve(h, bd, x64, args.tol, args.maxit)
        err64 = float(torch.linalg.norm(x - x64) / torch.linalg.norm(x64))
        us32 = 1000.0 * cms / max(1, csteps)
        mixed = dict(k=kh, s_per_solve=tm, iters=it_m, relres=rel_m, true_relres_scaled=trs,
                     true_relres_scaled_lib=stm["true_relres"], restarts=stm["restarts"], true_relres=tr,
                     err_vs_fp64=err64, status=B.pp_status_str(status_m), speedup_vs_fp64=best["s_per_solve"] / tm,
                     cheb_step_us=us32,
                     cheb_step_csr_equiv_gbs=cheb_bytes_per_step(n, nnz, kh, fp32=True) / (us32 * 1e-6) / 1e9)
        if npairs:
            # FP32 pairs: the stored diagonals once (a unit main one not read), r, s_{j-1}, s_{j-2}
            # read and s_j, s_{j+1} written, per launch
            pus = 1000.0 * pms / npairs
            pb = 4 * (stm["diagonals"] - stm["unit_diagonal"]) * (-(-n // 64) * 64) + 5 * 4 * n
            mixed.update(pair_launch_us=pus, pair_launches=npairs // max(1, args.steps), pair_bytes=pb,
                         pair_stored_gbs=pb / (pus * 1e-6) / 1e9)
        else:
            mixed["cheb_step_stored_gbs"] = stored_bytes_per_step(n, stm, kh, fp32=True) / (us32 * 1e-6) / 1e9
        log("mixed k=%d: %.3f s/solve, iters %d, FP64 true relres scaled %.2e (unscaled %.2e), "
            "x vs FP64 solve %.1e, speedup %.2fx" % (kh, tm, it_m, trs, tr, err64, mixed["speedup_vs_fp64"]))
        del x64
        B.pp_destroy(hm)

    newton = None
    if not args.no_newton:
        # Algorithm 1 (Newton form) against the three-term form at the same degree 2^nlev - 1
        newton = []
        for nlev in (4, 6):
            kk = 2 ** nlev - 1
            row = dict(nlev=nlev, k=kk)
            for form in ("chebyshev", "newton"):
                if form == "newton":
                    B.pp_setup_newton(h, nlev, lmin, lmax, args.xi)
                else:
                    B.pp_setup(h, kk, lmin, lmax, args.xi)
                x.zero_()
                B.pcg_solve(h, bd, x, args.tol, args.maxit)
                x.zero_()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                stn, itn, reln = B.pcg_solve(h, bd, x, args.tol, args.maxit)
                row[form] = dict(s_per_solve=round(time.perf_counter() - t0, 4), iters=itn,
                                 status=B.pp_status_str(stn))
            newton.append(row)
            log("degree %d: chebyshev %.3f s (%d iters), newton %.3f s (%d iters)"
                % (kk, row["chebyshev"]["s_per_solve"], row["chebyshev"]["iters"], row["newton"]["s_per_solve"],
                   row["newton"]["iters"]))
        B.pp_setup(h, kh, lmin, lmax, args.xi)

    lowrank = None
    if not args.no_lowrank:
        lowrank = {"hetero256": lowrank_leg(B, torch, h, bd, x, kh, lmin, lmax, args.tol, args.maxit),
                   "hetero256_lanczos64": lowrank_leg(B, torch, h, bd, x, kh, lmin, lmax, args.tol, args.maxit,
                                                      ranks=(1,), xis=(0.0,), ritz="lanczos")}
        B.pp_setup(h, kh, lmin, lmax, args.xi)
        # Poisson 32^3 (degree 10): 20 Lanczos steps overestimate its well separated lambda_1
        ap, bp = W.config_poisson32()
        hp = B.pp_create_csr(ap.n_rows, ap.nnz, torch.from_numpy(ap.rowptr).to(dev),
                             torch.from_numpy(ap.col).to(dev), torch.from_numpy(ap.val).to(dev), 0)
        lp, up = B.pp_estimate_bounds(hp, 20)
        xp = torch.zeros(ap.n_rows, dtype=torch.float64, device=dev)
        lowrank["poisson32"] = lowrank_leg(B, torch, hp, torch.from_numpy(bp).to(dev), xp, 10, lp, up, args.tol,
                                           args.maxit, ranks=(1, 3))
        B.pp_destroy(hp)

    dfn = None if args.no_dfn else run_dfn(args, B, W, torch, dev)
    args.dfn_su_ks = [int(v) for v in args.dfn_su_ks.split(",")]
    dfn_su = None if args.no_dfn_su else run_dfn_su(args, B, W, torch, dev)

    def fp64_single(k):
        """Time of one plain FP64 solve (first block column) at degree k on the same operator."""
        rec = next((r for r in per_k if r["k"] == k), None)
        if rec is not None:
            return rec["s_per_solve"]
        B.pp_setup(h, k, lmin, lmax, args.xi)
        b0 = torch.from_numpy(W.rhs_uniform(n, 3000)).to(dev)
        x.zero_()
        B.pcg_solve(h, b0, x, args.tol, args.maxit)
        x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        B.pcg_solve(h, b0, x, args.tol, args.maxit)
        return time.perf_counter() - t0

    block = None if args.no_block else run_block(args, B, W, torch, dev, a, lmin, lmax, fp64_single)
    batch256 = None if args.no_batch256 else run_batch256(args, B, W, torch, dev)

    general = None if args.no_general else run_general(args, B, W, torch, dev, a, bd, lmin, lmax)
    poisson32 = None if args.no_poisson32 else run_poisson32(args, B, W, torch, dev)
    learned = None if args.no_learned else run_learned(args, B, W, torch, dev)

    cpu = None
    if not args.no_cpu_baseline:
        kc = args.cpu_sample_k or 20
        rec = next((r for r in per_k if r["k"] == kc), best)
        cpu = run_cpu_baseline(args, a, b, lmin, lmax, kc, rec["op_applies"])

    out = {
        "metric": METRIC,
        "value": round(best["s_per_solve"], 5),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1000 * best["s_per_solve"], 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "hetero_diffusion_%d^3_7pt_lognormal_sigma2_jacobi" % args.N, "n": n,
                   "nnz": nnz, "k": kh, "ks": ks, "xi": args.xi, "tol": args.tol,
                   "residual": "||b_hat - A_hat x_hat|| / ||b_hat|| of the Jacobi-scaled system (section 4.3): "
                               "the recursive residual ends CG, the true one is checked in FP64 at exit; "
                               "unscaled_1e8 solves the original system to a true 1e-8",
                   "bounds": [lmin, lmax], "bounds_method": "20 Lanczos steps (the bounds record: 64 steps, learned)",
                   "parallelism": "single_gpu"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "pp_apply": {"k": kh, "ms": round(apply_ms, 3), "csr_equiv_gbs": round(apply_gbs, 1)},
        "per_k": per_k,
        "mixed": mixed,
        "newton": newton,
        "bounds": bounds,
        "lowrank": lowrank,
        "dfn": dfn,
        "dfn_su": dfn_su,
        "block": block,
        "batch256": batch256,
        "general": general,
        "poisson32": poisson32,
        "learned": learned,
        "unscaled_1e8": unscaled,
        "setup": {"create_s": round(t_create, 3), "lanczos_s": round(t_bounds, 4),
                  "nnz_stored": st0["nnz_stored"]},
    }
    B.pp_destroy(h)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
