"""CPU FP64 reference for the bounds MLP and the operator features (test infrastructure only).

MLP: ReLU hidden layers, linear output, loss = mean squared error; parameter
layout per layer: W [fan_in][fan_out] row-major, then b [fan_out].  The
backward pass here is pinned by central finite differences in the CPU tests.

Features: the 16 quantities documented for pp_features, computed from their
definitions with the oracle's operator application in FP64.
"""
from __future__ import annotations

import numpy as np

from .oracle import Operator, fmix32_start


def layer_shapes(n_in=16, hidden=128, depth=3, n_out=3):
    fi = [n_in] + [hidden] * depth
    fo = [hidden] * depth + [n_out]
    return list(zip(fi, fo))


def unpack(params, shapes):
    out, o = [], 0
    for fi, fo in shapes:
        W = params[o:o + fi * fo].reshape(fi, fo)
        o += fi * fo
        b = params[o:o + fo]
        o += fo
        out.append((W, b))
    return out


def forward(params, shapes, X):
    """Returns (Y, cache)."""
    h = np.asarray(X, dtype=np.float64)
    cache = [h]
    layers = unpack(np.asarray(params, dtype=np.float64), shapes)
    for li, (W, b) in enumerate(layers):
        z = h @ W + b
        if li < len(layers) - 1:
            cache.append(z)
            h = np.maximum(z, 0.0)
            cache.append(h)
        else:
            h = z
    return h, cache


def loss(params, shapes, X, T):
    Y, _ = forward(params, shapes, X)
    return float(np.mean((Y - T) ** 2))


def loss_grad(params, shapes, X, T):
    """Mean squared error and its gradient (same flat layout as params)."""
    params = np.asarray(params, dtype=np.float64)
    layers = unpack(params, shapes)
    Y, cache = forward(params, shapes, X)
    M, N = Y.shape
    dz = 2.0 * (Y - T) / (M * N)
    grads = []
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        hin = cache[0] if li == 0 else cache[2 * li]
        grads.append((hin.T @ dz, dz.sum(axis=0)))
        if li > 0:
            zprev = cache[2 * li - 1]
            dz = (dz @ W.T) * (zprev > 0)
    g = np.concatenate([np.concatenate([gw.ravel(), gb]) for gw, gb in reversed(grads)])
    return float(np.mean((Y - T) ** 2)), g


def adam(params, grad, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    p = params - lr * (m / (1 - b1 ** t)) / (np.sqrt(v / (1 - b2 ** t)) + eps)
    return p, m, v


def features(op: Operator, a, c=None, m=None, power_steps: int = 8) -> np.ndarray:
    """The 16 operator features, FP64, from their definitions.

    ``a`` (and for the Schur shape ``c``, ``m``) are the CSR parts that built
    ``op``; ``op.jacobi`` selects the scaled operator.
    """
    n = op.n
    rp, col, val = np.asarray(a.rowptr), np.asarray(a.col), np.asarray(a.val)
    dis = op.dis if op.jacobi else np.ones(n)
    rows = np.repeat(np.arange(n), np.diff(rp))
    ahat = val * dis[rows] * dis[col]
    diag_mask = col == rows
    aii = np.bincount(rows[diag_mask], weights=ahat[diag_mask], minlength=n)
    offa = np.bincount(rows[~diag_mask], weights=np.abs(ahat[~diag_mask]), minlength=n)
    length = np.bincount(rows[val != 0], minlength=n).astype(np.float64)
    tr = np.zeros(n)
    if c is not None:
        crp, ccol, cval = np.asarray(c.rowptr), np.asarray(c.col), np.asarray(c.val)
        trow = np.repeat(np.arange(len(crp) - 1), np.diff(crp))
        cm = cval * dis[ccol] / np.asarray(m)[trow]
        ts = np.bincount(trow, weights=np.abs(cm), minlength=len(crp) - 1)
        chat = cval * dis[ccol]
        tr = np.bincount(ccol, weights=np.abs(chat) * ts[trow], minlength=n)
        length += np.bincount(ccol[cval != 0], minlength=n)
    # unscaled diagonal: of the whole operator under Jacobi, of the A part otherwise
    d = op.diag_raw() if op.jacobi else aii
    ld = np.log10(d)
    rowabs = np.abs(aii) + offa + tr
    gup = rowabs.max()

    def power(shifted):
        v = fmix32_start(n)
        rq = []
        for _ in range(power_steps):
            y = op.apply(v)
            w = gup * v - y if shifted else y
            rq.append(float(v @ w) / float(v @ v))
            v = w
        return rq

    rq = power(False)
    rqs = power(True)
    P = power_steps
    q = [max(1, P // 4), max(1, P // 2), max(1, 3 * P // 4), P]
    lmin_est = gup - rqs[-1]
    f = np.zeros(16)
    f[0] = np.log10(n)
    f[1] = len(val) / n
    f[2] = ld.mean()
    f[3] = np.sqrt(max(0.0, (ld * ld).mean() - ld.mean() ** 2))
    f[4] = ld.min()
    f[5] = ld.max()
    f[6] = gup
    f[7] = (rowabs - aii).mean()
    f[8] = (aii - offa).min()
    f[9:13] = [rq[i - 1] for i in q]
    f[13] = lmin_est
    f[14] = length.max()
    f[15] = np.log10(max(rq[-1], 1e-300) / max(abs(lmin_est), 1e-12))
    return f
