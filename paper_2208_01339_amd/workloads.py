"""Seeded synthetic inputs for the polynomial-preconditioned CG path.

This module only builds operators and right-hand sides.  It holds none of the
method's arithmetic (no polynomial, no CG, no scaling): both the CPU oracle
under ``oracle/`` and the GPU path receive exactly the arrays produced here.

All matrices are returned in CSR form with int64 row pointers, int32 column
indices (ascending inside each row) and float64 values.  Every generator is
deterministic for a given seed (numpy ``default_rng``, PCG64).

Workloads (stand-ins for the paper's matrices, which are not public here):

* ``poisson3d(N)`` -- 7-point Dirichlet Laplacian on an N^3 grid, diagonal 6,
  -1 per interior neighbour, row index ``i + N*(j + N*k)``.
* ``hetero_diffusion(N, sigma, seed)`` -- 7-point finite-volume diffusion with
  cell permeability ``exp(sigma * z)``, ``z`` standard normal; the coefficient
  of an interior face is the harmonic mean ``2 Ka Kb / (Ka + Kb)``, a Dirichlet
  boundary face contributes ``K_cell`` to the diagonal only.  With ``sigma=0``
  this is exactly ``poisson3d(N)``.  Stands in for the large 3-D SPD problems
  of the paper's section 3 experiments.
* ``dfn_schur(...)`` -- the parts of a discrete-fracture-network shaped Schur
  complement ``S = A_ff + C^T M^{-1} C`` (section 4: a block-diagonal,
  fracture-local SPD block plus a trace-coupling term).  ``A_ff`` is block
  diagonal with one ``G x G`` 5-point Dirichlet Laplacian per fracture scaled by
  a lognormal transmissivity; ``C`` has one row per trace cell pair with +1 on
  the cell of one fracture and -1 on the matching cell of the other; ``M`` is a
  positive diagonal.  ``S`` itself is never formed.
* ``dfn_su(...)`` -- the blocks of the paper's DFN system (section 4.1,
  eq. (sys)): A block diagonal, one G x G 5-point finite-volume block per
  fracture with lognormal cell permeability (harmonic faces, Dirichlet
  boundary faces); G^h = gamma times the Neumann graph Laplacian of each
  fracture grid (SPSD, fracture-local); traces between pairs of fractures
  carry L flux unknowns on each side, ordered by the fracture that owns them;
  C (fracture-local) has 1 at the owner's trace cell, B = C + E with E = -1 at
  the matching cell of the other fracture; G^u = g_u [[1, 1], [1, 1]] on the
  two unknowns of every trace cell pair (SPSD, global).  The Schur complement
  S_u = G^u - a B^T A^-1 C - a C^T A^-1 B + C^T A^-1 G^h A^-1 C is never formed.
* ``irregular_fe(N, ...)`` -- an irregular SPD operator: the weighted graph
  Laplacian of a randomly thinned 27-point neighbourhood with a Dirichlet
  boundary, renumbered by random permutations inside windows of consecutive
  nodes (no column offset shared by most rows).  Stands in for unstructured
  3-D finite-element matrices such as the paper's Cube_5317k (section 3.2).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass
class CSR:
    n_rows: int
    n_cols: int
    rowptr: np.ndarray  # int64, n_rows + 1
    col: np.ndarray  # int32, nnz
    val: np.ndarray  # float64, nnz

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def to_scipy(self):
        import scipy.sparse as sp

        return sp.csr_matrix((self.val, self.col, self.rowptr), shape=(self.n_rows, self.n_cols))


@dataclass
class SchurParts:
    """Operator S = A_ff + C^T diag(m)^{-1} C, stored as its parts."""

    a: CSR  # n x n, block diagonal
    c: CSR  # nt x n, two entries per row (+1, -1)
    m: np.ndarray  # float64, nt, positive
    n_frac: int
    grid: int

    @property
    def n(self) -> int:
        return self.a.n_rows

    @property
    def nt(self) -> int:
        return self.c.n_rows


# ---------------------------------------------------------------------------
# 3-D seven-point operators
# ---------------------------------------------------------------------------

def _stencil7(N: int, kcell: np.ndarray | None) -> CSR:
    """Assemble the 7-point operator on an N^3 grid.

    ``kcell`` is the per-cell permeability (shape (N,N,N) indexed [k,j,i]) or
    None for the constant-coefficient Laplacian.  Columns come out ascending:
    -N^2, -N, -1, 0, +1, +N, +N^2.
    """
    n = N * N * N
    if kcell is None:
        kcell = np.ones((N, N, N), dtype=np.float64)
    K = kcell
    # harmonic means on interior faces, per direction (axis 0 = k, 1 = j, 2 = i)
    def harm(a, b):
        return 2.0 * a * b / (a + b)

    hk = harm(K[:-1, :, :], K[1:, :, :])  # face between k and k+1
    hj = harm(K[:, :-1, :], K[:, 1:, :])
    hi = harm(K[:, :, :-1], K[:, :, 1:])

    # face coefficients seen from each cell, per neighbour slot
    # slot order: k-1, j-1, i-1, (diag), i+1, j+1, k+1
    coef = np.zeros((7, N, N, N), dtype=np.float64)
    valid = np.zeros((7, N, N, N), dtype=bool)
    # k-1
    coef[0, 1:, :, :] = hk
    valid[0, 1:, :, :] = True
    coef[1, :, 1:, :] = hj
    valid[1, :, 1:, :] = True
    coef[2, :, :, 1:] = hi
    valid[2, :, :, 1:] = True
    coef[4, :, :, :-1] = hi
    valid[4, :, :, :-1] = True
    coef[5, :, :-1, :] = hj
    valid[5, :, :-1, :] = True
    coef[6, :-1, :, :] = hk
    valid[6, :-1, :, :] = True
    # diagonal: interior faces + boundary faces (coefficient K_cell)
    diag = coef[0] + coef[1] + coef[2] + coef[4] + coef[5] + coef[6]
    nb = 6 - (valid[0].astype(np.int64) + valid[1] + valid[2] + valid[4] + valid[5] + valid[6])
    diag = diag + nb * K
    offs = np.array([-N * N, -N, -1, 0, 1, N, N * N], dtype=np.int64)

    vals7 = np.empty((n, 7), dtype=np.float64)
    mask7 = np.empty((n, 7), dtype=bool)
    for s in range(7):
        if s == 3:
            vals7[:, 3] = diag.reshape(n)
            mask7[:, 3] = True
        else:
            vals7[:, s] = -coef[s].reshape(n)
            mask7[:, s] = valid[s].reshape(n)
    del coef, valid, diag
    rows = np.arange(n, dtype=np.int64)
    cols7 = (rows[:, None] + offs[None, :])
    cols7 = np.where(mask7, cols7, 0).astype(np.int32)
    counts = mask7.sum(axis=1, dtype=np.int64)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    flat = mask7.reshape(-1)
    val = vals7.reshape(-1)[flat]
    col = cols7.reshape(-1)[flat]
    return CSR(n, n, rowptr, np.ascontiguousarray(col), np.ascontiguousarray(val))


def poisson3d(N: int) -> CSR:
    """7-point Dirichlet Laplacian on N^3 (diagonal 6, -1 per interior neighbour)."""
    return _stencil7(N, None)


def permeability(N: int, sigma: float, seed: int) -> np.ndarray:
    """Lognormal cell permeability exp(sigma * z), z ~ N(0,1), shape (N,N,N) [k,j,i]."""
    z = np.random.default_rng(seed).standard_normal(N * N * N)
    return np.exp(sigma * z).reshape(N, N, N)


def hetero_diffusion(N: int, sigma: float = 2.0, seed: int = 0) -> CSR:
    """7-point diffusion with harmonic-mean face coefficients of a lognormal field."""
    return _stencil7(N, permeability(N, sigma, seed))


def rhs_uniform(n: int, seed: int) -> np.ndarray:
    """Right-hand side with entries uniform in [-1, 1)."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, n)


# ---------------------------------------------------------------------------
# DFN-shaped Schur operator
# ---------------------------------------------------------------------------

@dataclass
class DfnSuParts:
    """Blocks of the DFN saddle-point system in the unknowns (h, u, p)."""

    a: CSR  # n_h x n_h, block diagonal SPD (one G x G grid per fracture)
    gh: CSR  # n_h x n_h, block diagonal SPSD
    c: CSR  # n_h x n_u, fracture-local
    b: CSR  # n_h x n_u, C + E
    gu: CSR  # n_u x n_u, SPSD
    alpha: float
    n_frac: int
    grid: int
    u_off: np.ndarray  # int64, n_frac + 1: unknowns owned by fracture f are u_off[f] .. u_off[f+1]-1

    @property
    def n_h(self) -> int:
        return self.a.n_rows

    @property
    def n_u(self) -> int:
        return self.gu.n_rows


def _csr_from_coo(n_rows: int, n_cols: int, r, c, v) -> CSR:
    import scipy.sparse as sp

    m = sp.coo_matrix((v, (r, c)), shape=(n_rows, n_cols)).tocsr()
    m.sum_duplicates()
    m.sort_indices()
    return CSR(n_rows, n_cols, m.indptr.astype(np.int64), m.indices.astype(np.int32), m.data.astype(np.float64))


def _grid_faces(n_frac: int, G: int):
    """Interior faces of every fracture grid: (cell_a, cell_b) global indices, x- then y-faces."""
    m = G * G
    f = np.arange(n_frac, dtype=np.int64)[:, None, None]
    ii, jj = np.meshgrid(np.arange(G, dtype=np.int64), np.arange(G, dtype=np.int64), indexing="ij")
    base = f * m
    xa = (base + ii[:, :-1] * G + jj[:, :-1]).reshape(-1)
    ya = (base + ii[:-1, :] * G + jj[:-1, :]).reshape(-1)
    return np.concatenate([xa, ya]), np.concatenate([xa + 1, ya + G])


def dfn_su(n_frac: int = 400, G: int = 48, n_traces: int = 1100, L_lo: int = 10, L_hi: int = 40,
           sigma: float = 1.0, gamma: float = 100.0, g_u: float = 10.0, alpha: float = 1.0,
           seed: int = 0) -> DfnSuParts:
    """Blocks A, G^h, C, B, G^u of the DFN system of section 4.1, eq. (sys) (see module docstring).

    Traces: ``n_frac - 1`` spanning-tree traces then random pairs of distinct
    fractures, lengths uniform in [L_lo, L_hi], an independent straight
    segment of L cells on each side (as in ``dfn_schur``).  Unknown l of a
    trace side is owned by that side's fracture; unknowns are ordered by owner
    (stable), so C is block diagonal by fracture in its columns.
    """
    if n_traces < n_frac - 1:
        raise ValueError("need at least n_frac - 1 traces for a connected network")
    if L_hi > G or L_lo < 1:
        raise ValueError("trace lengths must lie in [1, G]")
    rng = np.random.default_rng(seed)
    m = G * G
    n_h = n_frac * m
    kc = np.exp(sigma * rng.standard_normal(n_h))
    fa, fb = _grid_faces(n_frac, G)
    coef = 2.0 * kc[fa] * kc[fb] / (kc[fa] + kc[fb])
    nbr = np.zeros(n_h)
    np.add.at(nbr, fa, 1.0)
    np.add.at(nbr, fb, 1.0)
    diag_a = np.zeros(n_h)
    np.add.at(diag_a, fa, coef)
    np.add.at(diag_a, fb, coef)
    diag_a += (4.0 - nbr) * kc  # Dirichlet boundary faces
    cells = np.arange(n_h, dtype=np.int64)
    a = _csr_from_coo(n_h, n_h, np.concatenate([fa, fb, cells]), np.concatenate([fb, fa, cells]),
                      np.concatenate([-coef, -coef, diag_a]))
    gh = _csr_from_coo(n_h, n_h, np.concatenate([fa, fb, cells]), np.concatenate([fb, fa, cells]),
                       gamma * np.concatenate([-np.ones(fa.size), -np.ones(fb.size), nbr]))

    pa = np.empty(n_traces, dtype=np.int64)
    pb = np.empty(n_traces, dtype=np.int64)
    for f in range(1, n_frac):
        pa[f - 1] = f
        pb[f - 1] = int(rng.integers(0, f))
    for t in range(n_frac - 1, n_traces):
        x = int(rng.integers(0, n_frac))
        y = int(rng.integers(0, n_frac - 1))
        if y >= x:
            y += 1
        pa[t], pb[t] = x, y
    own, cell_own, cell_other, pair = [], [], [], []
    npair = 0
    for t in range(n_traces):
        L = int(rng.integers(L_lo, L_hi + 1))
        sa = _segment(rng, G, L) + pa[t] * m
        sb = _segment(rng, G, L) + pb[t] * m
        k = np.arange(npair, npair + L, dtype=np.int64)
        own += [np.full(L, pa[t]), np.full(L, pb[t])]
        cell_own += [sa, sb]
        cell_other += [sb, sa]
        pair += [k, k]
        npair += L
    own = np.concatenate(own)
    cell_own = np.concatenate(cell_own)
    cell_other = np.concatenate(cell_other)
    pair = np.concatenate(pair)
    order = np.argsort(own, kind="stable")
    own, cell_own, cell_other, pair = own[order], cell_own[order], cell_other[order], pair[order]
    n_u = own.size
    u = np.arange(n_u, dtype=np.int64)
    c = _csr_from_coo(n_h, n_u, cell_own, u, np.ones(n_u))
    b = _csr_from_coo(n_h, n_u, np.concatenate([cell_own, cell_other]), np.concatenate([u, u]),
                      np.concatenate([np.ones(n_u), -np.ones(n_u)]))
    # the two unknowns of every trace cell pair
    pos_sorted = np.argsort(pair, kind="stable")
    first = u[pos_sorted[0::2]]
    second = u[pos_sorted[1::2]]
    gu = _csr_from_coo(n_u, n_u, np.concatenate([first, second, first, second]),
                       np.concatenate([first, second, second, first]), np.full(4 * npair, g_u))
    u_off = np.zeros(n_frac + 1, dtype=np.int64)
    np.cumsum(np.bincount(own, minlength=n_frac), out=u_off[1:])
    return DfnSuParts(a, gh, c, b, gu, float(alpha), n_frac, G, u_off)

def _lap2d_block_pattern(G: int):
    """5-point Dirichlet Laplacian pattern of one G x G fracture grid.

    Returns (rowptr, col, unit_val) with unit_val the coefficients for a
    transmissivity of 1 (diagonal 4, -1 per neighbour), columns ascending.
    """
    m = G * G
    ii, jj = np.meshgrid(np.arange(G), np.arange(G), indexing="ij")  # row-major cell = ii*G + jj
    cell = (ii * G + jj).reshape(m)
    offs = np.array([-G, -1, 0, 1, G], dtype=np.int64)
    valid = np.stack([
        (ii > 0).reshape(m),
        (jj > 0).reshape(m),
        np.ones(m, dtype=bool),
        (jj < G - 1).reshape(m),
        (ii < G - 1).reshape(m),
    ], axis=1)
    cols = cell[:, None] + offs[None, :]
    vals = np.where(offs[None, :] == 0, 4.0, -1.0) * np.ones((m, 5))
    counts = valid.sum(axis=1, dtype=np.int64)
    rowptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    return rowptr, cols[valid].astype(np.int64), vals[valid]


def _segment(rng, G: int, L: int) -> np.ndarray:
    """Cells (row-major local index) of a straight segment of L cells inside a G x G grid.

    Direction: along a row, along a column, or either diagonal; start uniform
    over the positions that keep the whole segment inside the grid.
    """
    d = int(rng.integers(0, 4))
    di, dj = [(0, 1), (1, 0), (1, 1), (1, -1)][d]
    span = L - 1
    i_lo, i_hi = 0, G - 1 - di * span
    if dj >= 0:
        j_lo, j_hi = 0, G - 1 - dj * span
    else:
        j_lo, j_hi = span, G - 1
    i0 = int(rng.integers(i_lo, i_hi + 1))
    j0 = int(rng.integers(j_lo, j_hi + 1))
    t = np.arange(L, dtype=np.int64)
    return (i0 + di * t) * G + (j0 + dj * t)


def dfn_schur(n_frac: int = 2000, G: int = 64, n_traces: int = 5000, L_lo: int = 10,
              L_hi: int = 60, sigma: float = 1.5, seed: int = 0) -> SchurParts:
    """DFN-shaped Schur operator parts (see module docstring).

    Traces: ``n_frac - 1`` spanning-tree traces (fracture f with a uniformly
    chosen earlier fracture) followed by random pairs of distinct fractures,
    ``n_traces`` in total; each has a length L uniform in [L_lo, L_hi] and an
    independent straight segment of L cells on each side.  Trace cell pair l
    gives one row of C.  M is uniform in [0.5, 2].
    """
    if n_traces < n_frac - 1:
        raise ValueError("need at least n_frac - 1 traces for a connected network")
    if L_hi > G:
        raise ValueError("trace longer than the fracture grid")
    rng = np.random.default_rng(seed)
    kf = np.exp(sigma * rng.standard_normal(n_frac))
    m = G * G
    n = n_frac * m
    brp, bcol, bval = _lap2d_block_pattern(G)
    bnnz = int(brp[-1])
    # block-diagonal A_ff
    a_rowptr = np.zeros(n + 1, dtype=np.int64)
    a_rowptr[1:] = (np.arange(n_frac, dtype=np.int64)[:, None] * bnnz + brp[None, 1:]).reshape(n)
    a_col = (np.arange(n_frac, dtype=np.int64)[:, None] * m + bcol[None, :]).reshape(-1).astype(np.int32)
    a_val = (kf[:, None] * bval[None, :]).reshape(-1)
    a = CSR(n, n, a_rowptr, a_col, a_val)

    # trace endpoints
    pa = np.empty(n_traces, dtype=np.int64)
    pb = np.empty(n_traces, dtype=np.int64)
    for f in range(1, n_frac):
        pa[f - 1] = f
        pb[f - 1] = int(rng.integers(0, f))
    for t in range(n_frac - 1, n_traces):
        x = int(rng.integers(0, n_frac))
        y = int(rng.integers(0, n_frac - 1))
        if y >= x:
            y += 1
        pa[t], pb[t] = x, y
    ca_list, cb_list = [], []
    for t in range(n_traces):
        L = int(rng.integers(L_lo, L_hi + 1))
        sa = _segment(rng, G, L) + pa[t] * m
        sb = _segment(rng, G, L) + pb[t] * m
        ca_list.append(sa)
        cb_list.append(sb)
    ca = np.concatenate(ca_list)
    cb = np.concatenate(cb_list)
    nt = ca.size
    lo = np.minimum(ca, cb)
    hi = np.maximum(ca, cb)
    v_lo = np.where(ca < cb, 1.0, -1.0)
    c_rowptr = np.arange(0, 2 * nt + 1, 2, dtype=np.int64)
    c_col = np.stack([lo, hi], axis=1).reshape(-1).astype(np.int32)
    c_val = np.stack([v_lo, -v_lo], axis=1).reshape(-1)
    c = CSR(nt, n, c_rowptr, c_col, c_val)
    mdiag = rng.uniform(0.5, 2.0, nt)
    return SchurParts(a, c, mdiag, n_frac, G)


# ---------------------------------------------------------------------------
# irregular 3-D operator (no shared column offsets)
# ---------------------------------------------------------------------------

def irregular_fe(N: int = 160, keep: float = 0.8, sigma: float = 1.0, window: int = 4096, seed: int = 0) -> CSR:
    """An irregular sparse SPD operator on n = N^3 unknowns.

    The weighted graph Laplacian of the 27-point neighbourhood of an N^3 grid
    of nodes (the pattern of trilinear hexahedral finite elements), with
    every edge kept independently with probability ``keep`` (row lengths vary
    between about 5 and 27), edge weight the harmonic mean of lognormal node
    permeabilities exp(sigma z) over the squared edge length, and a Dirichlet
    term K_node on the diagonal of every boundary node (SPD).  The nodes are
    renumbered by an independent random permutation inside each window of
    ``window`` consecutive grid nodes: the numbering keeps a mesh ordering's
    locality without its regularity, so no column offset is shared by most
    rows.  Stands in for unstructured 3-D finite-element matrices such as
    Cube_5317k of the paper's section 3.2 (not available here).
    """
    rng = np.random.default_rng(seed)
    n = N * N * N
    K = np.exp(sigma * rng.standard_normal(n))
    idx = np.arange(n, dtype=np.int64).reshape(N, N, N)  # [k, j, i]

    def src(d):
        return slice(max(0, -d), N - max(0, d))

    def dst(d):
        return slice(max(0, d), N - max(0, -d))

    diag = np.zeros(n)
    rr, cc, vv = [], [], []
    for dk in (-1, 0, 1):
        for dj in (-1, 0, 1):
            for di in (-1, 0, 1):
                if (dk, dj, di) <= (0, 0, 0):
                    continue  # each undirected edge once: 13 directions
                a = idx[src(dk), src(dj), src(di)].ravel()
                b = idx[dst(dk), dst(dj), dst(di)].ravel()
                m = rng.random(a.size) < keep
                a, b = a[m], b[m]
                w = 2.0 * K[a] * K[b] / (K[a] + K[b]) / float(dk * dk + dj * dj + di * di)
                diag += np.bincount(a, weights=w, minlength=n) + np.bincount(b, weights=w, minlength=n)
                rr += [a, b]
                cc += [b, a]
                vv += [-w, -w]
    kk, jj, ii = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    bnd = ((kk == 0) | (kk == N - 1) | (jj == 0) | (jj == N - 1) | (ii == 0) | (ii == N - 1)).ravel()
    diag += np.where(bnd, K, 0.0)
    # new number of grid node g: its window's start plus a random position inside the window
    order = np.lexsort((rng.random(n), np.arange(n) // window))
    new = np.empty(n, dtype=np.int64)
    new[order] = np.arange(n, dtype=np.int64)
    ar = np.arange(n, dtype=np.int64)
    r = np.concatenate([new[x] for x in rr] + [new[ar]])
    c = np.concatenate([new[x] for x in cc] + [new[ar]])
    v = np.concatenate(vv + [diag])
    del rr, cc, vv
    return _csr_from_coo(n, n, r, c, v)


# ---------------------------------------------------------------------------
# named workloads
# ---------------------------------------------------------------------------

def config_poisson32():
    """3-D Poisson 32^3, rhs U[-1,1] seed 0, Jacobi off, degree 10."""
    a = poisson3d(32)
    return a, rhs_uniform(a.n_rows, 0)


def config_hetero(N: int = 256, sigma: float = 2.0):
    """Heterogeneous diffusion N^3, permeability seed 0, rhs seed 1, Jacobi on."""
    a = hetero_diffusion(N, sigma, 0)
    return a, rhs_uniform(a.n_rows, 1)


def config_dfn(n_frac: int = 2000, G: int = 64, n_traces: int = 5000, L_lo: int = 10, L_hi: int = 60):
    """DFN-shaped Schur operator, transmissivity/trace seed 0, rhs seed 1, Jacobi on."""
    s = dfn_schur(n_frac, G, n_traces, L_lo, L_hi, 1.5, 0)
    return s, rhs_uniform(s.n, 1)


def batch_sizes(count: int = 256, lo: float = 1e4, hi: float = 2e6, seed: int = 4):
    """Grid sides of a batch of uneven 7-point systems: n ~ U[lo, hi], side = round(cbrt(n))."""
    u = np.random.default_rng(seed).uniform(lo, hi, count)
    return np.array([int(round(math.pow(x, 1.0 / 3.0))) for x in u], dtype=np.int64)


def batch_system(i: int, N: int, sigma: float = 2.0):
    """Member i of a batch: permeability seed 1000+i, rhs seed 2000+i."""
    a = hetero_diffusion(N, sigma, 1000 + i)
    return a, rhs_uniform(a.n_rows, 2000 + i)


def block_rhs(n: int, width: int, first_seed: int = 3000) -> np.ndarray:
    """Row-major [n][width] block of right-hand sides, column j from seed first_seed + j."""
    out = np.empty((n, width), dtype=np.float64)
    for j in range(width):
        out[:, j] = rhs_uniform(n, first_seed + j)
    return out


def block_diag(systems):
    """Stack CSR systems into one block-diagonal CSR; returns (CSR, sys_ptr int64 [nsys+1])."""
    n = [s.n_rows for s in systems]
    sys_ptr = np.zeros(len(systems) + 1, dtype=np.int64)
    np.cumsum(n, out=sys_ptr[1:])
    nnz = [s.nnz for s in systems]
    nz_ptr = np.zeros(len(systems) + 1, dtype=np.int64)
    np.cumsum(nnz, out=nz_ptr[1:])
    rowptr = np.empty(sys_ptr[-1] + 1, dtype=np.int64)
    col = np.empty(nz_ptr[-1], dtype=np.int32)
    val = np.empty(nz_ptr[-1], dtype=np.float64)
    for i, s in enumerate(systems):
        rowptr[sys_ptr[i]:sys_ptr[i + 1]] = s.rowptr[:-1] + nz_ptr[i]
        col[nz_ptr[i]:nz_ptr[i + 1]] = s.col + np.int32(sys_ptr[i])
        val[nz_ptr[i]:nz_ptr[i + 1]] = s.val
    rowptr[-1] = nz_ptr[-1]
    N = int(sys_ptr[-1])
    return CSR(N, N, rowptr, col, val), sys_ptr
