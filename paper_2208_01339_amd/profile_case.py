"""One workload's solves through the C-ABI, for profiler runs.

    python -m paper_2208_01339_amd.profile_case CASE [--solves S] [--calib-copy]

Each case builds its operator, estimates the spectral bounds, sets up the
polynomial and runs S solves of one right-hand side (FP64, Jacobi scaled,
tol 1e-8), so that a rocprofv3 kernel trace or counter run of the command
holds only the kernels of that workload:

  sliced256        heterogeneous diffusion 256^3 (sigma 2), every entry in
                   64-row slices, x staged in LDS tiles, k = 20
  sliced256_plain  the same with the tiles off (plain slice kernel)
  irregular160     thinned 27-point operator on 160^3 numbered by scattered
                   windows (renumbered at create), k = 20
  dfn              DFN-shaped Schur complement (2000 fractures of 64 x 64
                   cells, 5000 traces), k = 40
  dfn_su           DFN Schur complement S_u (400 fractures of 48 x 48 cells,
                   1100 traces), k = 31, scaling 1e-3
  batch256         256 uneven heterogeneous systems in one batched solve
                   (FP32 polynomial, FP64 CG), k = 60
  batch256_persistent  the same batch, the whole solve in one persistent
                   launch (PP_BOPT_DRIVER = 1)
  poisson32        Poisson 32^3, no scaling, k = 10, the default driver (one
                   persistent launch per solve at this size)

--calib-copy first runs one plain device copy of 1 GiB (the reference of the
HBM byte counters).  Prints one line per solve (iterations, seconds).
"""
from __future__ import annotations

import argparse
import sys
import time

import numpy as np

CASES = ("sliced256", "sliced256_plain", "irregular160", "dfn", "dfn_su", "batch256", "batch256_persistent",
         "poisson32")


def _log(*a):
    print(*a, flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("case", choices=CASES)
    ap.add_argument("--solves", type=int, default=2)
    ap.add_argument("--calib-copy", action="store_true")
    args = ap.parse_args(argv)

    import torch

    from . import binding as B
    from . import workloads as W

    B.lib()
    if not torch.cuda.is_available():
        raise SystemExit("profile_case needs a GPU")
    dev = torch.device("cuda:0")
    up = lambda v: torch.from_numpy(np.ascontiguousarray(v)).to(dev)
    if args.calib_copy:
        src = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    if args.case in ("batch256", "batch256_persistent"):
        sides = W.batch_sizes()
        systems, rhs = zip(*(W.batch_system(i, int(N)) for i, N in enumerate(sides)))
        full, sp = W.block_diag(list(systems))
        nsys = len(systems)
        h = B.pp_create_batch(nsys, sp, full.nnz, up(full.rowptr), up(full.col), up(full.val), 1,
                              B.PP_JACOBI | B.PP_MIXED)
        del full
        lo, hi = B.pp_batch_estimate_bounds(h, nsys, 20)
        B.pp_batch_setup(h, 60, lo, hi, 0.0)
        if args.case == "batch256_persistent":
            B.pp_batch_set_option(h, B.PP_BOPT_DRIVER, 1)
        bd = up(np.concatenate(rhs)).reshape(-1, 1)
        X = torch.zeros_like(bd)
        for i in range(args.solves):
            X.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s, it, _, _ = B.pcg_solve_batch(h, nsys, 1, bd, X, 1e-8, 5000)
            _log("solve %d: status %s, iterations %d..%d, %.3f s, driver %d" % (
                i, B.pp_status_str(s), it.min(), it.max(), time.perf_counter() - t0,
                B.pp_batch_get_stats(h)["driver"]))
        B.pp_destroy_batch(h)
        return 0

    xi, k = 0.0, 20
    if args.case in ("sliced256", "sliced256_plain"):
        a, b = W.config_hetero(256, 2.0)
        op = B.Operator(a=a, flags=B.PP_JACOBI | B.PP_SLICED)
        B.pp_set_option(op.handle, B.PP_OPT_LDS_TILES, 1 if args.case == "sliced256" else 0)
    elif args.case == "irregular160":
        a = W.irregular_fe(160)
        b = W.rhs_uniform(a.n_rows, 1)
        op = B.Operator(a=a, flags=B.PP_JACOBI)
    elif args.case == "poisson32":
        a, b = W.config_poisson32()
        op = B.Operator(a=a, flags=0)
        k = 10
    elif args.case == "dfn":
        s, b = W.config_dfn()
        op = B.Operator(schur=s, flags=B.PP_JACOBI)
        k = 40
    else:
        P = W.dfn_su()
        op = B.Operator(dfn=P)
        q = up(W.rhs_uniform(P.n_h, 1))
        r = torch.empty(P.n_u, dtype=torch.float64, device=dev)
        B.pp_dfn_rhs(op.handle, q, r)
        b = r.cpu().numpy()
        k, xi = 31, 1e-3
    h = op.handle
    lmin, lmax = B.pp_estimate_bounds(h, 20)
    B.pp_setup(h, k, lmin, lmax, xi)
    bd = up(b)
    x = torch.zeros_like(bd)
    for i in range(args.solves):
        x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s, it, rel = B.pcg_solve(h, bd, x, 1e-8, 5000)
        _log("solve %d: status %s, %d iterations, relres %.2e, %.3f s" % (i, B.pp_status_str(s), it, rel,
                                                                         time.perf_counter() - t0))
    st = B.pp_get_stats(h)
    _log("stats: %s" % {key: st[key] for key in ("diagonals", "nnz_stored", "lds_tiles", "reordered",
                                                  "gather_spread", "driver")})
    op.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
