"""Learned spectral bounds and scaling parameter.

Pipeline (all numerical work in the library's HIP kernels):
  1. dataset: seeded 7-point and DFN-shaped operators; for each, the 16
     features (pp_features), the 20-step Lanczos bounds (pp_estimate_bounds)
     and PCG iteration counts at degree 40, all produced by this library on
     the GPU.  Twenty Lanczos steps overestimate lambda_min of ill-conditioned
     operators (the smallest Ritz value has not converged), so the label
     lambda_min is the iteration-optimal s* lambda_min(Lanczos) over
     s in {1, 1/2, 1/4, 1/8} (ties: the larger s), and the label xi* the
     iteration-optimal grid value at that lambda_min (ties: the smaller xi);
  2. training: the 16 -> 128 -> 128 -> 128 -> 3 MLP with the library's
     forward/backward/Adam kernels on normalised features and targets
     (log lambda_min*, log lambda_max(Lanczos), log10(xi* + 1e-5));
  3. evaluation on held-out operators: iterations and setup time of
     (predicted bounds, predicted xi) against (Lanczos bounds, xi = 0), the
     fallback rate, and the bound errors.

    python -m paper_2208_01339_amd.learned dataset --ntrain 5000 --ntest 500 --out DIR
    python -m paper_2208_01339_amd.learned train --data DIR --weights WDIR
    python -m paper_2208_01339_amd.learned evaluate --data DIR --weights WDIR
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

from . import binding as B
from . import workloads as W

XI_GRID = (0.0, 1e-4, 1e-3, 1e-2)
LMIN_SHRINK = (1.0, 0.5, 0.25, 0.125)
K_LABEL = 40
TOL = 1e-8
POWER_STEPS = 8
WEIGHTS_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights")


def sample_operator(i: int, seed: int):
    """Operator i of a dataset: even i -> 7-point, odd i -> DFN-shaped; n log-uniform in [1e4, 1e6]."""
    rng = np.random.default_rng(seed * 1_000_003 + i)
    sigma = float(rng.uniform(0.5, 3.0))
    if i % 2 == 0:
        n = math.exp(rng.uniform(math.log(1e4), math.log(1e6)))
        N = int(min(100, max(22, round(n ** (1.0 / 3.0)))))
        a = W.hetero_diffusion(N, sigma, 10_000 + 7 * i + seed)
        return dict(kind="7pt", a=a, schur=None, n=a.n_rows, sigma=sigma, size=N)
    nf = int(round(math.exp(rng.uniform(math.log(3), math.log(244)))))
    nt = max(nf - 1, int(round(2.5 * nf)))
    s = W.dfn_schur(nf, 64, nt, 10, 60, sigma, 20_000 + 7 * i + seed)
    return dict(kind="dfn", a=None, schur=s, n=s.n, sigma=sigma, size=nf)


def _solve_iters(torch, op, b, k, lmin, lmax, xi, maxit=4000):
    B.pp_setup(op.handle, k, lmin, lmax, xi)
    x = torch.zeros_like(b)
    s, it, rel = B.pcg_solve(op.handle, b, x, TOL, maxit)
    return it if s == B.PP_OK else maxit


def build_dataset(count: int, seed: int, log=print):
    """Features, Lanczos bounds and xi-scan iteration counts for `count` operators."""
    import torch

    feats, bounds, iters, meta = [], [], [], []
    t_start = time.perf_counter()
    for i in range(count):
        d = sample_operator(i, seed)
        op = B.Operator(a=d["a"], schur=d["schur"], flags=B.PP_JACOBI)
        b = torch.from_numpy(W.rhs_uniform(d["n"], 30_000 + i + seed)).cuda()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        f = B.pp_features(op.handle, POWER_STEPS)
        t_feat = time.perf_counter() - t0
        t0 = time.perf_counter()
        lo, hi = B.pp_estimate_bounds(op.handle, 20)
        t_lz = time.perf_counter() - t0
        its_s = [_solve_iters(torch, op, b, K_LABEL, lo * sh, hi, 0.0) for sh in LMIN_SHRINK]
        best_s = LMIN_SHRINK[int(np.flatnonzero(np.array(its_s) == min(its_s))[0])]
        its_x = [its_s[LMIN_SHRINK.index(best_s)]] + [
            _solve_iters(torch, op, b, K_LABEL, lo * best_s, hi, xi) for xi in XI_GRID[1:]]
        op.close()
        feats.append(f)
        bounds.append((lo, hi, best_s))
        iters.append(its_s + its_x)
        meta.append((0 if d["kind"] == "7pt" else 1, d["n"], d["sigma"], d["size"], t_feat, t_lz))
        if (i + 1) % 100 == 0 or i + 1 == count:
            log("dataset %d/%d (%.0fs)" % (i + 1, count, time.perf_counter() - t_start))
    return dict(features=np.array(feats), bounds=np.array(bounds), iters=np.array(iters, dtype=np.int32),
                meta=np.array(meta), xi_grid=np.array(XI_GRID), lmin_shrink=np.array(LMIN_SHRINK))


def targets(data):
    """(log lambda_min*, log lambda_max, log10(xi* + 1e-5)) and the index of xi*."""
    ns = len(data["lmin_shrink"])
    itx = data["iters"][:, ns:]
    best = np.array([int(np.flatnonzero(r == r.min())[0]) for r in itx])  # ties -> smaller xi
    xi = np.asarray(data["xi_grid"])[best]
    lo, hi, sh = data["bounds"][:, 0], data["bounds"][:, 1], data["bounds"][:, 2]
    return np.stack([np.log(lo * sh), np.log(hi), np.log10(xi + 1e-5)], axis=1), best


class Model:
    """The bounds MLP living in the library, with its normalisation."""

    def __init__(self, seed=0):
        import torch

        self.torch = torch
        self.h = B.pp_mlp_create(16, 128, 3, 3, seed)
        self.nparam = B.pp_mlp_num_params(self.h)
        self.norm = None

    def set_norm(self, in_mean, in_std, out_mean, out_std):
        self.norm = [np.asarray(v, dtype=np.float64) for v in (in_mean, in_std, out_mean, out_std)]
        B.pp_mlp_set_normalization(self.h, *self.norm)

    def params(self):
        t = self.torch.empty(self.nparam, dtype=self.torch.float32, device="cuda")
        B.pp_mlp_get_params(self.h, t)
        self.torch.cuda.synchronize()
        return t.cpu().numpy()

    def load_params(self, p):
        B.pp_mlp_set_params(self.h, self.torch.from_numpy(np.ascontiguousarray(p, dtype=np.float32)).cuda())
        self.torch.cuda.synchronize()

    def save(self, wdir):
        os.makedirs(wdir, exist_ok=True)
        np.save(os.path.join(wdir, "bounds_mlp.npy"), self.params(), allow_pickle=False)
        with open(os.path.join(wdir, "bounds_mlp.json"), "w") as f:
            json.dump({"layers": [16, 128, 128, 128, 3], "power_steps": POWER_STEPS, "k_label": K_LABEL,
                       "xi_grid": list(XI_GRID), "in_mean": self.norm[0].tolist(), "in_std": self.norm[1].tolist(),
                       "out_mean": self.norm[2].tolist(), "out_std": self.norm[3].tolist()}, f, indent=1)

    @classmethod
    def load(cls, wdir=WEIGHTS_DIR):
        with open(os.path.join(wdir, "bounds_mlp.json")) as f:
            meta = json.load(f)
        m = cls()
        m.load_params(np.load(os.path.join(wdir, "bounds_mlp.npy"), allow_pickle=False))
        m.set_norm(meta["in_mean"], meta["in_std"], meta["out_mean"], meta["out_std"])
        return m

    def close(self):
        if self.h:
            B.pp_mlp_destroy(self.h)
            self.h = None


def train(data, epochs=400, batch=128, lr=1e-3, seed=0, log=print):
    torch = __import__("torch")
    X = np.asarray(data["features"], dtype=np.float64)
    Y, _ = targets(data)
    in_mean, in_std = X.mean(0), np.maximum(X.std(0), 1e-6)
    out_mean, out_std = Y.mean(0), np.maximum(Y.std(0), 1e-6)
    Xn = ((X - in_mean) / in_std).astype(np.float32)
    Yn = ((Y - out_mean) / out_std).astype(np.float32)
    m = Model(seed)
    m.set_norm(in_mean, in_std, out_mean, out_std)
    Xd = torch.from_numpy(Xn).cuda()
    Yd = torch.from_numpy(Yn).cuda()
    rng = np.random.default_rng(seed)
    n = Xn.shape[0]
    hist = []
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(n)).cuda()
        tot = 0.0
        steps = 0
        for s0 in range(0, n, batch):
            idx = perm[s0:s0 + batch]
            xb = Xd.index_select(0, idx).contiguous()
            yb = Yd.index_select(0, idx).contiguous()
            step_lr = lr * (0.1 if ep >= int(0.8 * epochs) else 1.0)
            tot += B.pp_mlp_train_step(m.h, xb, yb, step_lr)
            steps += 1
        hist.append(tot / steps)
        if (ep + 1) % 50 == 0:
            log("epoch %d loss %.4f" % (ep + 1, hist[-1]))
    return m, hist


def evaluate(model, count: int, seed: int, log=print):
    """Held-out operators: predicted bounds/xi vs Lanczos bounds with xi = 0 (and the best grid xi)."""
    import torch

    rows = []
    for i in range(count):
        d = sample_operator(i, seed)
        op = B.Operator(a=d["a"], schur=d["schur"], flags=B.PP_JACOBI)
        b = torch.from_numpy(W.rhs_uniform(d["n"], 30_000 + i + seed)).cuda()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lo_p, hi_p, xi_p, fb = B.pp_predict_bounds(op.handle, model.h, POWER_STEPS)
        t_pred = time.perf_counter() - t0
        t0 = time.perf_counter()
        lo_l, hi_l = B.pp_estimate_bounds(op.handle, 20)
        t_lz = time.perf_counter() - t0
        it_pred = _solve_iters(torch, op, b, K_LABEL, lo_p, hi_p, xi_p)
        it_lz0 = _solve_iters(torch, op, b, K_LABEL, lo_l, hi_l, 0.0)
        it_grid = min(_solve_iters(torch, op, b, K_LABEL, lo_l * sh, hi_l, xi)
                      for sh in LMIN_SHRINK for xi in XI_GRID)
        op.close()
        rows.append(dict(kind=d["kind"], n=d["n"], it_pred=it_pred, it_lanczos_xi0=it_lz0, it_best_grid=it_grid,
                         fallback=fb, t_pred=t_pred, t_lanczos=t_lz, err_lmin_vs_lanczos=math.log(lo_p / lo_l),
                         err_lmax_vs_lanczos=math.log(hi_p / hi_l), xi_pred=xi_p))
    r = rows
    summ = dict(
        count=count,
        mean_iters_pred=float(np.mean([x["it_pred"] for x in r])),
        mean_iters_lanczos_xi0=float(np.mean([x["it_lanczos_xi0"] for x in r])),
        mean_iters_best_grid=float(np.mean([x["it_best_grid"] for x in r])),
        fallback_rate=float(np.mean([x["fallback"] for x in r])),
        mean_setup_s_pred=float(np.mean([x["t_pred"] for x in r])),
        mean_setup_s_lanczos=float(np.mean([x["t_lanczos"] for x in r])),
        median_log_lmin_over_lanczos=float(np.median([x["err_lmin_vs_lanczos"] for x in r])),
        median_abs_log_err_lmax=float(np.median([abs(x["err_lmax_vs_lanczos"]) for x in r])),
    )
    return summ, rows


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("cmd", choices=["dataset", "train", "evaluate", "all"])
    ap.add_argument("--ntrain", type=int, default=5000)
    ap.add_argument("--ntest", type=int, default=500)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--data", default="gpurun_out/learned")
    ap.add_argument("--weights", default=WEIGHTS_DIR)
    ap.add_argument("--epochs", type=int, default=400)
    args = ap.parse_args(argv)

    def log(msg):
        print("[learned] " + msg, flush=True)

    os.makedirs(args.data, exist_ok=True)
    if args.cmd in ("dataset", "all"):
        tr = build_dataset(args.ntrain, args.seed, log)
        np.savez(os.path.join(args.data, "train.npz"), **tr)
    if args.cmd in ("train", "all"):
        data = dict(np.load(os.path.join(args.data, "train.npz"), allow_pickle=False))
        t0 = time.perf_counter()
        m, hist = train(data, epochs=args.epochs, log=log)
        log("trained in %.1fs, final loss %.4f" % (time.perf_counter() - t0, hist[-1]))
        m.save(args.weights)
        with open(os.path.join(args.data, "train_loss.json"), "w") as f:
            json.dump(hist, f)
        m.close()
    if args.cmd in ("evaluate", "all"):
        m = Model.load(args.weights)
        summ, rows = evaluate(m, args.ntest, args.seed + 7919, log)
        m.close()
        log(json.dumps(summ))
        with open(os.path.join(args.data, "evaluate.json"), "w") as f:
            json.dump({"summary": summ, "rows": rows}, f)
    return 0


if __name__ == "__main__":
    sys.exit(main())
