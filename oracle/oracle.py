"""Python face of the CPU oracle (test infrastructure only).

Thin ctypes marshalling around ``ppcg_oracle.c`` plus the few steps that are
plain library calls (a symmetric tridiagonal eigensolve for the Lanczos
bounds).  Arrays are numpy float64 / int64 / int32 on the host.

Only tests, the smoke check and the CPU-baseline leg of the benchmark may use
this module; the GPU library never does.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ppcg_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# The same source built with OpenMP: used only to time the oracle on all host
# cores (its dot products sum in another order; it is never a parity reference).
_LIB_OMP = os.path.join(_HERE, "liboracle_omp.so")

OK, NOT_CONVERGED, BREAKDOWN, ERR_ARG = 0, 1, 2, -1

_CFLAGS = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no FMA contraction, no fast-math), and its
    OpenMP timing build."""
    for out, extra in ((_LIB, []), (_LIB_OMP, ["-fopenmp"])):
        if force or not os.path.exists(out):
            subprocess.check_call(_CFLAGS + extra + ["-o", out + ".tmp", _SRC, "-lm"])
            os.replace(out + ".tmp", out)
    return _LIB


_libs = {}


def lib(omp: bool = False):
    """The checker build, or with ``omp`` the OpenMP timing build."""
    key = bool(omp)
    if key not in _libs:
        path = _LIB_OMP if omp else _LIB
        override = os.environ.get("PPCG_ORACLE_LIB")  # a sanitizer build of the same source (tests)
        if override and not omp:
            path = override
        elif not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(path)
        P = C.c_void_p
        L.orc_dot.restype = C.c_double
        L.orc_dot.argtypes = [C.c_int64, P, P]
        L.orc_csr_matvec.argtypes = [C.c_int64, P, P, P, P, P]
        L.orc_op_apply.argtypes = [P, P, P]
        L.orc_op_diag.argtypes = [P, P]
        L.orc_cheb_coeffs.restype = C.c_int
        L.orc_cheb_coeffs.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, P, P, P, P]
        L.orc_cheb_apply.restype = C.c_int
        L.orc_cheb_apply.argtypes = [P, C.c_int, C.c_double, C.c_double, C.c_double, P, P, P]
        L.orc_newton_apply.restype = C.c_int
        L.orc_newton_apply.argtypes = [P, C.c_int, C.c_double, C.c_double, C.c_double, P, P]
        L.orc_pcg.restype = C.c_int
        L.orc_pcg.argtypes = [P, C.c_int, C.c_double, C.c_double, C.c_double, P, P, C.c_double,
                              C.c_int, P]
        L.orc_pcg_newton.restype = C.c_int
        L.orc_pcg_newton.argtypes = [P, C.c_int, C.c_double, C.c_double, C.c_double, P, P, C.c_double,
                                     C.c_int, P]
        L.orc_lowrank_setup.restype = C.c_int
        L.orc_lowrank_setup.argtypes = [P, C.c_int, P, P]
        L.orc_lowrank_apply.restype = C.c_int
        L.orc_lowrank_apply.argtypes = [P, C.c_int, C.c_double, C.c_double, C.c_double, C.c_int, P, P, P, P, P]
        L.orc_pcg_lowrank.restype = C.c_int
        L.orc_pcg_lowrank.argtypes = [P, C.c_int, C.c_double, C.c_double, C.c_double, C.c_int, P, P, P, P,
                                      C.c_double, C.c_int, P]
        L.orc_lanczos.restype = C.c_int
        L.orc_lanczos.argtypes = [P, C.c_int, P, P]
        L.orc_fmix32_start.argtypes = [C.c_int64, P]
        L.orc_dfn_factor.restype = C.c_int
        L.orc_dfn_factor.argtypes = [P]
        L.orc_dfn_ainv.argtypes = [P, P, P]
        L.orc_dfn_su.argtypes = [P, P, P]
        L.orc_dfn_diag.argtypes = [P, P]
        L.orc_dfn_rhs.argtypes = [P, P, P]
        L.orc_dfn_recover.argtypes = [P, P, P, P, P]
        _libs[key] = L
    return _libs[key]


class _OpStruct(C.Structure):
    _fields_ = [
        ("kind", C.c_int32), ("pad0", C.c_int32), ("n", C.c_int64),
        ("arp", C.c_void_p), ("aci", C.c_void_p), ("av", C.c_void_p),
        ("nt", C.c_int64), ("crp", C.c_void_p), ("cci", C.c_void_p), ("cv", C.c_void_p),
        ("m", C.c_void_p), ("dis", C.c_void_p), ("work_n", C.c_void_p), ("work_nt", C.c_void_p),
        ("n_apply", C.c_int64), ("dfn", C.c_void_p),
    ]


class _DfnStruct(C.Structure):
    _fields_ = [("n_frac", C.c_int64), ("G", C.c_int64), ("nf", C.c_int64), ("nh", C.c_int64),
                ("nu", C.c_int64)] + [
        (nm + sfx, C.c_void_p) for nm in ("a", "gh", "c", "b", "gu") for sfx in ("rp", "ci", "v")] + [
        ("alpha", C.c_double), ("L", C.c_void_p), ("w1", C.c_void_p), ("w2", C.c_void_p),
        ("w3", C.c_void_p), ("w4", C.c_void_p), ("wu", C.c_void_p)]


class _PcgStats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("status", C.c_int32), ("relres", C.c_double),
                ("n_apply", C.c_int64), ("n_dot", C.c_int64)]


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class Operator:
    """A CSR matrix or the Schur-shaped operator A_ff + C^T M^{-1} C.

    ``a`` is any object with ``rowptr``, ``col``, ``val`` (CSR, n x n); for the
    Schur shape pass ``c`` (nt x n CSR) and ``m`` (nt).  With ``jacobi`` the
    operator seen by every routine is D^{-1/2} op D^{-1/2}, D = diag(op)
    (section 3 with W = D^{-1/2}; section 4.3 for the Schur case).
    """

    def __init__(self, a, c=None, m=None, jacobi: bool = False):
        self.n = int(len(a.rowptr) - 1)
        self._arp = np.ascontiguousarray(a.rowptr, dtype=np.int64)
        self._aci = np.ascontiguousarray(a.col, dtype=np.int32)
        self._av = _f64(a.val)
        self.kind = 0 if c is None else 1
        self._work_n = np.zeros(self.n)
        s = _OpStruct()
        s.kind = self.kind
        s.n = self.n
        s.arp, s.aci, s.av = _p(self._arp), _p(self._aci), _p(self._av)
        s.work_n = _p(self._work_n)
        if c is not None:
            self.nt = int(len(c.rowptr) - 1)
            self._crp = np.ascontiguousarray(c.rowptr, dtype=np.int64)
            self._cci = np.ascontiguousarray(c.col, dtype=np.int32)
            self._cv = _f64(c.val)
            self._m = _f64(m)
            self._work_nt = np.zeros(self.nt)
            s.nt = self.nt
            s.crp, s.cci, s.cv = _p(self._crp), _p(self._cci), _p(self._cv)
            s.m, s.work_nt = _p(self._m), _p(self._work_nt)
        else:
            self.nt = 0
        self._s = s
        self.jacobi = bool(jacobi)
        self.dis = None
        if jacobi:
            d = self.diag_raw()
            if not np.all(d > 0):
                raise ValueError("Jacobi scaling needs a positive diagonal")
            self.dis = 1.0 / np.sqrt(d)
            s.dis = _p(self.dis)

    @property
    def n_apply(self) -> int:
        return int(self._s.n_apply)

    def reset_count(self):
        self._s.n_apply = 0

    def diag_raw(self) -> np.ndarray:
        """diag(op) of the unscaled operator."""
        d = np.zeros(self.n)
        lib().orc_op_diag(C.byref(self._s), _p(d))
        return d

    def apply(self, x) -> np.ndarray:
        """op-hat x (scaled when jacobi)."""
        x = _f64(x)
        y = np.empty(self.n)
        lib().orc_op_apply(C.byref(self._s), _p(x), _p(y))
        return y

    def apply_raw(self, x) -> np.ndarray:
        """op x, unscaled, whatever the jacobi flag."""
        saved = self._s.dis
        self._s.dis = None
        try:
            return self.apply(x)
        finally:
            self._s.dis = saved


class DfnOperator(Operator):
    """The DFN Schur complement S_u(alpha) of section 4.2, applied from the
    expansion of eq. (schur) with the exact (banded) Cholesky factor of A; with
    ``jacobi`` the operator is D_S^{-1/2} S_u D_S^{-1/2}, D_S = diag(S_u)
    (section 4.3, the quantity of Algorithm 4).

    ``parts`` carries the CSR blocks ``a, gh, c, b, gu``, ``alpha``, ``n_frac``
    and ``grid`` (each fracture a block of grid^2 rows of A and G^h).  Every
    routine of this module that takes an ``Operator`` takes this one.
    """

    def __init__(self, parts, jacobi: bool = True):
        G = int(parts.grid)
        nf = G * G
        nh = int(len(parts.a.rowptr) - 1)
        nu = int(len(parts.gu.rowptr) - 1)
        self.n = nu
        self.kind = 2
        self._keep = []
        d = _DfnStruct()
        d.n_frac, d.G, d.nf, d.nh, d.nu = int(parts.n_frac), G, nf, nh, nu
        for nm in ("a", "gh", "c", "b", "gu"):
            m = getattr(parts, nm)
            rp = np.ascontiguousarray(m.rowptr, dtype=np.int64)
            ci = np.ascontiguousarray(m.col, dtype=np.int32)
            v = _f64(m.val)
            self._keep += [rp, ci, v]
            setattr(d, nm + "rp", _p(rp).value)
            setattr(d, nm + "ci", _p(ci).value)
            setattr(d, nm + "v", _p(v).value)
        d.alpha = float(parts.alpha)
        self.L = np.zeros(nh * (G + 1))
        self._w = [np.zeros(nh) for _ in range(4)] + [np.zeros(nu)]
        d.L = _p(self.L).value
        d.w1, d.w2, d.w3, d.w4, d.wu = (_p(w).value for w in self._w)
        self._d = d
        self.nh = nh
        if lib().orc_dfn_factor(C.byref(d)) != OK:
            raise ValueError("A is not block diagonal within the band, or not SPD")
        self._work_n = np.zeros(nu)
        s = _OpStruct()
        s.kind = 2
        s.n = nu
        s.work_n = _p(self._work_n)
        s.dfn = C.cast(C.pointer(d), C.c_void_p)
        self._s = s
        self.nt = 0
        self.jacobi = bool(jacobi)
        self.dis = None
        if jacobi:
            dd = self.diag_raw()
            if not np.all(dd > 0):
                raise ValueError("diag(S_u) must be positive")
            self.dis = 1.0 / np.sqrt(dd)
            s.dis = _p(self.dis)

    def ainv(self, b) -> np.ndarray:
        """A^{-1} b with the Cholesky factor."""
        b = _f64(b)
        x = np.empty(self.nh)
        lib().orc_dfn_ainv(C.byref(self._d), _p(b), _p(x))
        return x

    def rhs(self, q) -> np.ndarray:
        """r = W^T M^{-1} (q, 0) = a B^T A^{-1} q - C^T A^{-1} G^h A^{-1} q (unscaled)."""
        q = _f64(q)
        r = np.empty(self.n)
        lib().orc_dfn_rhs(C.byref(self._d), _p(q), _p(r))
        return r

    def recover(self, q, u):
        """(h, p) = (A^{-1} (q + C u), A^{-1} (a B u - G^h h))."""
        q, u = _f64(q), _f64(u)
        h = np.empty(self.nh)
        p = np.empty(self.nh)
        lib().orc_dfn_recover(C.byref(self._d), _p(q), _p(u), _p(h), _p(p))
        return h, p


def csr_matvec(a, x) -> np.ndarray:
    x = _f64(x)
    n = len(a.rowptr) - 1
    y = np.empty(n)
    rp = np.ascontiguousarray(a.rowptr, dtype=np.int64)
    ci = np.ascontiguousarray(a.col, dtype=np.int32)
    v = _f64(a.val)
    lib().orc_csr_matvec(n, _p(rp), _p(ci), _p(v), _p(x), _p(y))
    return y


def cheb_coeffs(k: int, lmin: float, lmax: float, xi: float):
    """(theta_bar, delta, sigma, rho[0..k]) of the xi-modified Chebyshev polynomial."""
    rho = np.zeros(k + 1)
    th, de, si = C.c_double(), C.c_double(), C.c_double()
    st = lib().orc_cheb_coeffs(k, lmin, lmax, xi, C.byref(th), C.byref(de), C.byref(si), _p(rho))
    if st != OK:
        raise ValueError("invalid polynomial parameters")
    return th.value, de.value, si.value, rho


def cheb_apply_hat(op: Operator, k: int, lmin: float, lmax: float, xi: float, r) -> np.ndarray:
    """p_k(op-hat) r by Algorithm 2 (scaled space when op.jacobi)."""
    r = _f64(r)
    z = np.empty(op.n)
    work = np.empty(3 * op.n)
    st = lib().orc_cheb_apply(C.byref(op._s), k, lmin, lmax, xi, _p(r), _p(z), _p(work))
    if st != OK:
        raise ValueError("invalid polynomial parameters")
    return z


def cheb_apply(op: Operator, k: int, lmin: float, lmax: float, xi: float, r) -> np.ndarray:
    """Effective preconditioner applied to r: D^{-1/2} p_k(op-hat) D^{-1/2} r (or p_k(op) r)."""
    r = _f64(r)
    if op.dis is None:
        return cheb_apply_hat(op, k, lmin, lmax, xi, r)
    return op.dis * cheb_apply_hat(op, k, lmin, lmax, xi, op.dis * r)


def newton_apply_hat(op: Operator, nlev: int, lmin: float, lmax: float, xi: float, r) -> np.ndarray:
    """P_nlev r by Algorithm 1 (degree 2^nlev - 1), scaled space when op.jacobi."""
    r = _f64(r)
    z = np.empty(op.n)
    st = lib().orc_newton_apply(C.byref(op._s), nlev, lmin, lmax, xi, _p(r), _p(z))
    if st != OK:
        raise ValueError("invalid polynomial parameters")
    return z


def pcg(op: Operator, k: int, lmin: float, lmax: float, xi: float, b, x0=None, tol: float = 1e-8,
        maxit: int = 1000, omp: bool = False):
    """CG on op x = b preconditioned by p_k; returns (x, stats).

    ``omp`` runs the OpenMP timing build (CSR and Schur operators only)."""
    b = _f64(b)
    x = np.zeros(op.n) if x0 is None else _f64(x0).copy()
    st = _PcgStats()
    t0 = time.perf_counter()
    ret = lib(omp).orc_pcg(C.byref(op._s), k, lmin, lmax, xi, _p(b), _p(x), tol, maxit, C.byref(st))
    dt = time.perf_counter() - t0
    if ret == ERR_ARG:
        raise ValueError("invalid PCG arguments")
    return x, dict(iters=int(st.iters), status=int(st.status), relres=float(st.relres),
                   n_apply=int(st.n_apply), n_dot=int(st.n_dot), seconds=dt)


def pcg_newton(op: Operator, nlev: int, lmin: float, lmax: float, xi: float, b, x0=None, tol: float = 1e-8,
               maxit: int = 1000):
    """CG on op x = b preconditioned by P_nlev of Algorithm 1; returns (x, stats)."""
    b = _f64(b)
    x = np.zeros(op.n) if x0 is None else _f64(x0).copy()
    st = _PcgStats()
    ret = lib().orc_pcg_newton(C.byref(op._s), nlev, lmin, lmax, xi, _p(b), _p(x), tol, maxit, C.byref(st))
    if ret == ERR_ARG:
        raise ValueError("invalid PCG arguments")
    return x, dict(iters=int(st.iters), status=int(st.status), relres=float(st.relres),
                   n_apply=int(st.n_apply), n_dot=int(st.n_dot))


def _cols(V) -> np.ndarray:
    """n x p array -> contiguous column-major storage (column j at j*n)."""
    V = np.asarray(V, dtype=np.float64)
    if V.ndim == 1:
        V = V[:, None]
    return np.ascontiguousarray(V.T)


def lowrank_setup(op: Operator, V) -> np.ndarray:
    """(V^T op-hat V)^{-1} for the spectral low-rank correction of section 3.1 (p x p)."""
    Vc = _cols(V)
    p = Vc.shape[0]
    hinv = np.empty((p, p))
    if lib().orc_lowrank_setup(C.byref(op._s), p, _p(Vc), _p(hinv)) != OK:
        raise ValueError("V^T A V is singular")
    return hinv


def lowrank_apply_hat(op: Operator, k: int, lmin: float, lmax: float, xi: float, V, hinv, r) -> np.ndarray:
    """(p_k(op-hat) + V (V^T op-hat V)^{-1} V^T) r in the scaled space."""
    Vc = _cols(V)
    r = _f64(r)
    z = np.empty(op.n)
    work = np.empty(3 * op.n)
    h = np.ascontiguousarray(hinv, dtype=np.float64)
    st = lib().orc_lowrank_apply(C.byref(op._s), k, lmin, lmax, xi, Vc.shape[0], _p(Vc), _p(h), _p(r), _p(z),
                                 _p(work))
    if st != OK:
        raise ValueError("invalid polynomial parameters")
    return z


def pcg_lowrank(op: Operator, k: int, lmin: float, lmax: float, xi: float, V, b, x0=None, tol: float = 1e-8,
                maxit: int = 1000, hinv=None):
    """CG preconditioned by p_k + V (V^T A V)^{-1} V^T (V in the scaled space); returns (x, stats)."""
    Vc = _cols(V)
    h = lowrank_setup(op, V) if hinv is None else np.ascontiguousarray(hinv, dtype=np.float64)
    b = _f64(b)
    x = np.zeros(op.n) if x0 is None else _f64(x0).copy()
    st = _PcgStats()
    ret = lib().orc_pcg_lowrank(C.byref(op._s), k, lmin, lmax, xi, Vc.shape[0], _p(Vc), _p(h), _p(b), _p(x),
                                tol, maxit, C.byref(st))
    if ret == ERR_ARG:
        raise ValueError("invalid PCG arguments")
    return x, dict(iters=int(st.iters), status=int(st.status), relres=float(st.relres),
                   n_apply=int(st.n_apply), n_dot=int(st.n_dot))


def lanczos_basis(op: Operator, m: int):
    """The Lanczos recurrence of orc_lanczos, keeping the basis: (alpha, beta, Q) with Q n x j."""
    n = op.n
    v = fmix32_start(n)
    v = v / np.sqrt(v @ v)
    vprev = np.zeros(n)
    bprev = 0.0
    a, b, Q = [], [], []
    for _ in range(m):
        Q.append(v.copy())
        w = op.apply(v) - bprev * vprev
        al = float(v @ w)
        w = w - al * v
        be = float(np.sqrt(w @ w))
        a.append(al)
        b.append(be)
        if be == 0.0:
            break
        vprev, v = v, w / be
        bprev = be
    return np.array(a), np.array(b), np.array(Q).T


def ritz_vectors(op: Operator, m: int, p: int):
    """Ritz values and vectors of the p smallest Ritz values after m Lanczos steps (scaled space)."""
    from scipy.linalg import eigh_tridiagonal

    a, b, Q = lanczos_basis(op, m)
    j = len(a)
    w, S = eigh_tridiagonal(a, b[: j - 1]) if j > 1 else (a.copy(), np.ones((1, 1)))
    return w[:p], Q @ S[:, :p]


def poly_ritz_vectors(op: Operator, k: int, lmin: float, lmax: float, xi: float, m: int, p: int):
    """Ritz pairs of the smallest eigenvalues of op-hat from m Lanczos steps on the
    preconditioner p_k(op-hat) (Algorithm 2 for each product) with full
    reorthogonalisation: the Ritz vectors of the p largest Ritz values of
    p_k(op-hat), which p_k maps from the smallest eigenvalues of op-hat, and
    their Rayleigh quotients v^T op-hat v / v^T v.  Returns (theta, V n x p)."""
    from scipy.linalg import eigh_tridiagonal

    n = op.n
    v = fmix32_start(n)
    v = v / np.sqrt(v @ v)
    vprev = np.zeros(n)
    bprev = 0.0
    a, b, Q = [], [], []
    for _ in range(m):
        Q.append(v.copy())
        w = cheb_apply_hat(op, k, lmin, lmax, xi, v) - bprev * vprev
        al = float(v @ w)
        w = w - al * v
        Qm = np.array(Q).T
        w = w - Qm @ (Qm.T @ w)
        be = float(np.sqrt(w @ w))
        a.append(al)
        b.append(be)
        if be == 0.0:
            break
        vprev, v = v, w / be
        bprev = be
    j = len(a)
    wv, S = eigh_tridiagonal(np.array(a), np.array(b)[: j - 1]) if j > 1 else (np.array(a), np.ones((1, 1)))
    top = np.argsort(-wv)[:p]
    V = np.array(Q).T @ S[:, top]
    theta = np.array([float(V[:, c] @ op.apply(V[:, c])) / float(V[:, c] @ V[:, c]) for c in range(V.shape[1])])
    return theta, V


def fmix32_start(n: int) -> np.ndarray:
    v = np.empty(n)
    lib().orc_fmix32_start(n, _p(v))
    return v


def lanczos(op: Operator, m: int = 20):
    """alpha_1..alpha_j, beta_1..beta_j of j <= m Lanczos steps on op-hat."""
    a = np.zeros(m)
    b = np.zeros(m)
    done = lib().orc_lanczos(C.byref(op._s), m, _p(a), _p(b))
    return a[:done], b[:done]


def lanczos_bounds(op: Operator, m: int = 20):
    """Spectral bounds for the polynomial from m Lanczos steps.

    lambda_min = smallest Ritz value; lambda_max = largest Ritz value plus the
    Ritz residual |beta_m s_{m,max}| (s = eigenvector of T_m for the largest
    Ritz value), which makes lambda_max an upper bound of the closest
    eigenvalue of op-hat.
    """
    from scipy.linalg import eigh_tridiagonal

    a, b = lanczos(op, m)
    j = len(a)
    if j == 1:
        w = a.copy()
        s = np.ones((1, 1))
    else:
        w, s = eigh_tridiagonal(a, b[: j - 1])
    pad = abs(b[j - 1] * s[j - 1, -1])
    return float(w[0]), float(w[-1] + pad)
