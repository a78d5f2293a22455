"""ctypes binding of include/pp.h (argument marshalling only).

Every function keeps the C name and forwards to libppcg.so; device arrays are
torch CUDA tensors, streams are torch streams.  All computation happens in the
HIP kernels of the library: if it is not built or cannot be loaded, every call
raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libppcg.so")

PP_OK, PP_NOT_CONVERGED, PP_BREAKDOWN = 0, 1, 2
PP_ERR_ARG, PP_ERR_OOM, PP_ERR_HIP, PP_ERR_STATE, PP_ERR_TIMEOUT = -1, -2, -3, -4, -5
PP_JACOBI, PP_MIXED, PP_SLICED, PP_NO_REORDER = 1, 2, 4, 8
PP_OPT_GRID, PP_OPT_CHUNK, PP_OPT_TIMING, PP_OPT_DRIVER, PP_OPT_NT_LOADS, PP_OPT_TWO_STEP, PP_OPT_VERIFY = 1, 2, 3, 4, 5, 6, 7
PP_OPT_RITZ, PP_OPT_LDS_TILES, PP_OPT_BARRIER, PP_OPT_SPIN_LIMIT = 8, 9, 10, 11

PP_BOPT_GRAPH, PP_BOPT_DRIVER = 100, 101

ABI_FUNCTIONS = (
    "pp_create_csr", "pp_create_schur", "pp_setup", "pp_apply", "pcg_solve", "pp_estimate_bounds",
    "pp_operator_apply", "pp_get_stats", "pp_set_option", "pp_destroy", "pp_status_str",
    "pp_last_error", "pp_create_batch", "pp_batch_estimate_bounds", "pp_batch_setup",
    "pcg_solve_batch", "pp_batch_apply", "pp_batch_set_layout", "pp_batch_autotune",
    "pp_batch_set_option", "pp_batch_get_stats", "pp_destroy_batch", "pp_mlp_create", "pp_mlp_destroy",
    "pp_mlp_num_params", "pp_mlp_get_params", "pp_mlp_set_params", "pp_mlp_set_normalization",
    "pp_mlp_forward", "pp_mlp_loss_grad", "pp_mlp_train_step", "pp_features", "pp_predict_bounds",
    "pp_lowrank_set", "pp_lowrank_ritz", "pp_lowrank_get", "pp_lowrank_info", "pp_setup_newton",
    "pp_create_dfn", "pp_dfn_rhs", "pp_dfn_recover", "pcg_solve_csr_noalloc",
)


class PPError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (_status_name(status), msg))
        self.status = status


class pp_stats(C.Structure):
    _fields_ = [
        ("iters", C.c_int32), ("status", C.c_int32), ("relres", C.c_double),
        ("op_applies", C.c_int64), ("dots", C.c_int64), ("cheb_ms", C.c_double),
        ("cheb_steps", C.c_int64), ("solve_ms", C.c_double), ("n", C.c_int64),
        ("nnz_stored", C.c_int64), ("nnz_matrix", C.c_int64), ("driver", C.c_int32),
        ("grid", C.c_int32), ("diagonals", C.c_int32), ("two_step", C.c_int32),
        ("pair_ms", C.c_double), ("pair_launches", C.c_int64), ("restarts", C.c_int32), ("reordered", C.c_int32),
        ("true_relres", C.c_double), ("gather_spread", C.c_double), ("lds_tiles", C.c_int32), ("unit_diagonal", C.c_int32),
        ("barrier", C.c_int32),
    ]


class pp_batch_stats(C.Structure):
    _fields_ = [
        ("n", C.c_int64), ("nsys", C.c_int32), ("nb", C.c_int32), ("nrhs", C.c_int32), ("w", C.c_int32),
        ("nnz_stored", C.c_int64), ("grid", C.c_int32), ("graph", C.c_int32), ("solve_ms", C.c_double),
        ("max_iters", C.c_int32), ("diag_systems", C.c_int32), ("restarts", C.c_int32), ("verified", C.c_int32),
        ("driver", C.c_int32),
    ]


_lib = None


def lib():
    """Load libppcg.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        path = os.environ.get("PPCG_LIB", LIB_PATH)  # another build of the same sources (sanitizer tests)
        if not os.path.exists(path):
            raise RuntimeError("libppcg.so is not built; run __graft_entry__.build() "
                               "(python -m paper_2208_01339_amd.build)")
        L = C.CDLL(path)
        P, I64, I32, D = C.c_void_p, C.c_int64, C.c_int, C.c_double
        L.pp_create_csr.argtypes = [C.POINTER(P), I64, I64, P, P, P, C.c_uint, P]
        L.pp_create_schur.argtypes = [C.POINTER(P), I64, I64, P, P, P, I64, I64, P, P, P, P, C.c_uint, P]
        L.pp_create_dfn.argtypes = [C.POINTER(P), C.POINTER(pp_dfn_desc), C.c_uint, P]
        L.pp_dfn_rhs.argtypes = [P, P, P]
        L.pp_dfn_recover.argtypes = [P, P, P, P, P]
        L.pp_setup.argtypes = [P, I32, D, D, D]
        L.pp_apply.argtypes = [P, P, P]
        L.pcg_solve.argtypes = [P, P, P, D, I32, C.POINTER(I32), C.POINTER(D)]
        L.pcg_solve_csr_noalloc.argtypes = [I64, I64, P, P, P, C.c_uint, I32, D, D, D, P, P, D, I32,
                                            C.POINTER(I32), C.POINTER(D), P]
        L.pp_estimate_bounds.argtypes = [P, I32, C.POINTER(D), C.POINTER(D)]
        L.pp_operator_apply.argtypes = [P, P, P]
        L.pp_get_stats.argtypes = [P, C.POINTER(pp_stats)]
        L.pp_set_option.argtypes = [P, I32, I64]
        L.pp_destroy.argtypes = [P]
        L.pp_destroy.restype = None
        L.pp_status_str.argtypes = [I32]
        L.pp_status_str.restype = C.c_char_p
        L.pp_last_error.argtypes = []
        L.pp_last_error.restype = C.c_char_p
        L.pp_create_batch.argtypes = [C.POINTER(P), I32, P, I64, P, P, P, I32, C.c_uint, P]
        L.pp_batch_estimate_bounds.argtypes = [P, I32, P, P]
        L.pp_batch_setup.argtypes = [P, I32, P, P, D]
        L.pcg_solve_batch.argtypes = [P, P, P, D, I32, P, P, P]
        L.pp_batch_apply.argtypes = [P, P, P]
        L.pp_batch_set_layout.argtypes = [P, I32]
        L.pp_batch_autotune.argtypes = [P, C.POINTER(I32), C.POINTER(D)]
        L.pp_batch_set_option.argtypes = [P, I32, I64]
        L.pp_batch_get_stats.argtypes = [P, C.POINTER(pp_batch_stats)]
        L.pp_destroy_batch.argtypes = [P]
        L.pp_destroy_batch.restype = None
        F32 = C.c_float
        L.pp_mlp_create.argtypes = [C.POINTER(P), I32, I32, I32, I32, C.c_uint64, P]
        L.pp_mlp_destroy.argtypes = [P]
        L.pp_mlp_destroy.restype = None
        L.pp_mlp_num_params.argtypes = [P, C.POINTER(I64)]
        L.pp_mlp_get_params.argtypes = [P, P]
        L.pp_mlp_set_params.argtypes = [P, P]
        L.pp_mlp_set_normalization.argtypes = [P, P, P, P, P]
        L.pp_mlp_forward.argtypes = [P, I32, P, P]
        L.pp_mlp_loss_grad.argtypes = [P, I32, P, P, P, C.POINTER(D)]
        L.pp_mlp_train_step.argtypes = [P, I32, P, P, F32, C.POINTER(D)]
        L.pp_features.argtypes = [P, I32, P]
        L.pp_lowrank_set.argtypes = [P, I32, P]
        L.pp_setup_newton.argtypes = [P, I32, D, D, D]
        L.pp_lowrank_ritz.argtypes = [P, I32, I32, P]
        L.pp_lowrank_get.argtypes = [P, C.POINTER(I32), P]
        L.pp_lowrank_info.argtypes = [P, P, P]
        L.pp_predict_bounds.argtypes = [P, P, I32, C.POINTER(D), C.POINTER(D), C.POINTER(D), C.POINTER(I32)]
        for f in ABI_FUNCTIONS:
            if f not in ("pp_destroy", "pp_status_str", "pp_last_error", "pp_destroy_batch", "pp_mlp_destroy"):
                getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def _status_name(s: int) -> str:
    try:
        return lib().pp_status_str(s).decode()
    except Exception:  # pragma: no cover - only while reporting another error
        return str(s)


def _check(s: int, ok=(PP_OK,)) -> int:
    if s not in ok:
        raise PPError(s, lib().pp_last_error().decode())
    return s


def _ptr(t):
    """Device pointer of a contiguous torch CUDA tensor (or None -> NULL)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device (CUDA/HIP) tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    import torch

    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _dtype_check(t, dt, name):
    if t.dtype != dt:
        raise ValueError("%s must be %s" % (name, dt))


# ---------------------------------------------------------------------------
# the C ABI, one wrapper per function
# ---------------------------------------------------------------------------

def pp_create_csr(n, nnz, rowptr, colind, val, flags=0, stream=None):
    import torch

    _dtype_check(rowptr, torch.int64, "rowptr")
    _dtype_check(colind, torch.int32, "colind")
    _dtype_check(val, torch.float64, "val")
    h = C.c_void_p()
    _check(lib().pp_create_csr(C.byref(h), int(n), int(nnz), _ptr(rowptr), _ptr(colind), _ptr(val),
                               int(flags), _stream(stream)))
    return h


def pp_create_schur(n, nnz_a, a_rowptr, a_col, a_val, nt, nnz_c, c_rowptr, c_col, c_val, m_diag,
                    flags=0, stream=None):
    import torch

    for t, dt, nm in ((a_rowptr, torch.int64, "a_rowptr"), (a_col, torch.int32, "a_col"),
                      (a_val, torch.float64, "a_val"), (c_rowptr, torch.int64, "c_rowptr"),
                      (c_col, torch.int32, "c_col"), (c_val, torch.float64, "c_val"),
                      (m_diag, torch.float64, "m_diag")):
        _dtype_check(t, dt, nm)
    h = C.c_void_p()
    _check(lib().pp_create_schur(C.byref(h), int(n), int(nnz_a), _ptr(a_rowptr), _ptr(a_col),
                                 _ptr(a_val), int(nt), int(nnz_c), _ptr(c_rowptr), _ptr(c_col),
                                 _ptr(c_val), _ptr(m_diag), int(flags), _stream(stream)))
    return h


class pp_csr(C.Structure):
    _fields_ = [("rows", C.c_int64), ("cols", C.c_int64), ("nnz", C.c_int64), ("rowptr", C.c_void_p),
                ("col", C.c_void_p), ("val", C.c_void_p)]


class pp_dfn_desc(C.Structure):
    _fields_ = [("n_frac", C.c_int64), ("grid", C.c_int64), ("a", pp_csr), ("gh", pp_csr), ("c", pp_csr),
                ("b", pp_csr), ("gu", pp_csr), ("u_off", C.c_void_p), ("alpha", C.c_double)]


def pp_create_dfn(n_frac, grid, mats, u_off, alpha, flags=0, stream=None):
    """mats: dict a, gh, c, b, gu -> (rows, cols, rowptr, col, val) with device tensors
    (int64, int32, float64); u_off: host numpy int64 [n_frac + 1]."""
    import numpy as np
    import torch

    d = pp_dfn_desc()
    d.n_frac, d.grid, d.alpha = int(n_frac), int(grid), float(alpha)
    for nm in ("a", "gh", "c", "b", "gu"):
        rows, cols, rp, cl, v = mats[nm]
        _dtype_check(rp, torch.int64, nm + ".rowptr")
        _dtype_check(cl, torch.int32, nm + ".col")
        _dtype_check(v, torch.float64, nm + ".val")
        m = getattr(d, nm)
        m.rows, m.cols, m.nnz = int(rows), int(cols), int(v.numel())
        m.rowptr, m.col, m.val = _ptr(rp), _ptr(cl), _ptr(v)
    uo = np.ascontiguousarray(u_off, dtype=np.int64)
    d.u_off = uo.ctypes.data_as(C.c_void_p)
    h = C.c_void_p()
    _check(lib().pp_create_dfn(C.byref(h), C.byref(d), int(flags), _stream(stream)))
    return h


def pp_dfn_rhs(op, q, r):
    import torch

    _dtype_check(q, torch.float64, "q")
    _dtype_check(r, torch.float64, "r")
    _check(lib().pp_dfn_rhs(op, _ptr(q), _ptr(r)))


def pp_dfn_recover(op, q, u, h, p):
    import torch

    for t, nm in ((q, "q"), (u, "u"), (h, "h"), (p, "p")):
        _dtype_check(t, torch.float64, nm)
    _check(lib().pp_dfn_recover(op, _ptr(q), _ptr(u), _ptr(h), _ptr(p)))


def pp_setup(op, k, lambda_min, lambda_max, scaling=0.0):
    return _check(lib().pp_setup(op, int(k), float(lambda_min), float(lambda_max), float(scaling)))


def pp_apply(op, r, z):
    return _check(lib().pp_apply(op, _ptr(r), _ptr(z)))


def pcg_solve(op, b, x, tol=1e-8, maxit=1000):
    """Returns (status, iters, relres); raises on argument/HIP errors only."""
    it = C.c_int(0)
    rel = C.c_double(0.0)
    s = lib().pcg_solve(op, _ptr(b), _ptr(x), float(tol), int(maxit), C.byref(it), C.byref(rel))
    _check(s, ok=(PP_OK, PP_NOT_CONVERGED, PP_BREAKDOWN))
    return s, it.value, rel.value


def pcg_solve_csr_noalloc(n, nnz, rowptr, colind, val, flags, k, lambda_min, lambda_max, scaling, b, x,
                          tol=1e-8, maxit=1000, stream=None):
    """The allocation-free solve on a plain device CSR matrix; returns (status, iters, relres)."""
    it = C.c_int(0)
    rel = C.c_double(0.0)
    s = lib().pcg_solve_csr_noalloc(int(n), int(nnz), _ptr(rowptr), _ptr(colind), _ptr(val), int(flags), int(k),
                                    float(lambda_min), float(lambda_max), float(scaling), _ptr(b), _ptr(x),
                                    float(tol), int(maxit), C.byref(it), C.byref(rel), _stream(stream))
    _check(s, ok=(PP_OK, PP_NOT_CONVERGED, PP_BREAKDOWN))
    return s, it.value, rel.value


def pp_estimate_bounds(op, steps=20):
    lo, hi = C.c_double(), C.c_double()
    _check(lib().pp_estimate_bounds(op, int(steps), C.byref(lo), C.byref(hi)))
    return lo.value, hi.value


def pp_setup_newton(op, nlev, lambda_min, lambda_max, scaling=0.0):
    return _check(lib().pp_setup_newton(op, int(nlev), float(lambda_min), float(lambda_max), float(scaling)))


def pp_lowrank_set(op, p, V=None):
    """V: device tensor [p][n] (row j = vector j, i.e. column-major n x p), or None with p = 0."""
    return _check(lib().pp_lowrank_set(op, int(p), _ptr(V)))


def pp_lowrank_ritz(op, steps, p):
    """Installs the Ritz vectors of the p smallest Ritz values; returns those Ritz values."""
    import numpy as np

    th = np.zeros(int(p))
    _check(lib().pp_lowrank_ritz(op, int(steps), int(p), _hptr(th)))
    return th


def pp_lowrank_get(op, V=None):
    """Rank in use; copies the vectors into V (device [p][n]) when given."""
    p = C.c_int()
    _check(lib().pp_lowrank_get(op, C.byref(p), _ptr(V)))
    return p.value


def pp_lowrank_info(op):
    """(theta, resid) host arrays of the installed correction: Rayleigh quotients and relative
    Ritz residuals ||A-hat v - theta v|| / (|theta| ||v||)."""
    import numpy as np

    p = pp_lowrank_get(op)
    th = np.zeros(max(1, p))
    rs = np.zeros(max(1, p))
    _check(lib().pp_lowrank_info(op, _hptr(th), _hptr(rs)))
    return th[:p], rs[:p]


def pp_operator_apply(op, x, y):
    return _check(lib().pp_operator_apply(op, _ptr(x), _ptr(y)))


def pp_get_stats(op):
    st = pp_stats()
    _check(lib().pp_get_stats(op, C.byref(st)))
    return {f: getattr(st, f) for f, _ in pp_stats._fields_}


def pp_set_option(op, key, value):
    return _check(lib().pp_set_option(op, int(key), int(value)))


def pp_destroy(op):
    if op:
        lib().pp_destroy(op)


def pp_status_str(s):
    return lib().pp_status_str(int(s)).decode()


def pp_last_error():
    return lib().pp_last_error().decode()


# ---------------------------------------------------------------------------
# batches
# ---------------------------------------------------------------------------

def _hptr(a):
    """Host pointer of a contiguous numpy array."""
    return a.ctypes.data_as(C.c_void_p)


def pp_create_batch(nsys, sys_ptr, nnz, rowptr, colind, val, nrhs=1, flags=0, stream=None):
    import numpy as np
    import torch

    sp = np.ascontiguousarray(sys_ptr, dtype=np.int64)
    if sp.size != nsys + 1:
        raise ValueError("sys_ptr must hold nsys + 1 entries")
    _dtype_check(rowptr, torch.int64, "rowptr")
    _dtype_check(colind, torch.int32, "colind")
    _dtype_check(val, torch.float64, "val")
    h = C.c_void_p()
    _check(lib().pp_create_batch(C.byref(h), int(nsys), _hptr(sp), int(nnz), _ptr(rowptr), _ptr(colind),
                                 _ptr(val), int(nrhs), int(flags), _stream(stream)))
    return h


def pp_batch_estimate_bounds(op, nsys, steps=20):
    import numpy as np

    lo = np.zeros(nsys)
    hi = np.zeros(nsys)
    _check(lib().pp_batch_estimate_bounds(op, int(steps), _hptr(lo), _hptr(hi)))
    return lo, hi


def pp_batch_setup(op, k, lambda_min, lambda_max, scaling=0.0):
    import numpy as np

    lo = np.ascontiguousarray(lambda_min, dtype=np.float64)
    hi = np.ascontiguousarray(lambda_max, dtype=np.float64)
    return _check(lib().pp_batch_setup(op, int(k), _hptr(lo), _hptr(hi), float(scaling)))


def pcg_solve_batch(op, nsys, nrhs, B, X, tol=1e-8, maxit=1000):
    """Returns (worst status, iters[nsys, nrhs], relres[nsys, nrhs], status[nsys, nrhs])."""
    import numpy as np

    it = np.zeros(nsys * nrhs, dtype=np.int32)
    rel = np.zeros(nsys * nrhs)
    stt = np.zeros(nsys * nrhs, dtype=np.int32)
    s = lib().pcg_solve_batch(op, _ptr(B), _ptr(X), float(tol), int(maxit), _hptr(it), _hptr(rel), _hptr(stt))
    _check(s, ok=(PP_OK, PP_NOT_CONVERGED, PP_BREAKDOWN))
    return s, it.reshape(nsys, nrhs), rel.reshape(nsys, nrhs), stt.reshape(nsys, nrhs)


def pp_batch_apply(op, R, Z):
    return _check(lib().pp_batch_apply(op, _ptr(R), _ptr(Z)))


def pp_batch_set_layout(op, w):
    return _check(lib().pp_batch_set_layout(op, int(w)))


def pp_batch_autotune(op):
    w = C.c_int(0)
    us = C.c_double(0.0)
    _check(lib().pp_batch_autotune(op, C.byref(w), C.byref(us)))
    return w.value, us.value


def pp_batch_set_option(op, key, value):
    return _check(lib().pp_batch_set_option(op, int(key), int(value)))


def pp_batch_get_stats(op):
    st = pp_batch_stats()
    _check(lib().pp_batch_get_stats(op, C.byref(st)))
    return {f: getattr(st, f) for f, _ in pp_batch_stats._fields_ if f != "pad"}


def pp_destroy_batch(op):
    if op:
        lib().pp_destroy_batch(op)


class BatchOperator:
    """Owns a pp_batch built from a list of host CSR systems (block-diagonal stacking)."""

    def __init__(self, systems, nrhs=1, flags=0, device="cuda:0", stream=None):
        import torch

        from .workloads import block_diag

        a, sys_ptr = block_diag(systems)
        dev = torch.device(device)
        self.nsys = len(systems)
        self.nrhs = nrhs
        self.n = a.n_rows
        self.sys_ptr = sys_ptr
        self.handle = pp_create_batch(
            self.nsys, sys_ptr, a.nnz, torch.from_numpy(a.rowptr).to(dev), torch.from_numpy(a.col).to(dev),
            torch.from_numpy(a.val).to(dev), nrhs, flags, stream)

    def close(self):
        if self.handle:
            pp_destroy_batch(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# learned bounds
# ---------------------------------------------------------------------------

NFEAT = 16


def pp_mlp_create(n_in=16, hidden=128, depth=3, n_out=3, seed=0, stream=None):
    h = C.c_void_p()
    _check(lib().pp_mlp_create(C.byref(h), int(n_in), int(hidden), int(depth), int(n_out), int(seed),
                               _stream(stream)))
    return h


def pp_mlp_destroy(h):
    if h:
        lib().pp_mlp_destroy(h)


def pp_mlp_num_params(h):
    c = C.c_int64()
    _check(lib().pp_mlp_num_params(h, C.byref(c)))
    return c.value


def pp_mlp_get_params(h, dst):
    return _check(lib().pp_mlp_get_params(h, _ptr(dst)))


def pp_mlp_set_params(h, src):
    return _check(lib().pp_mlp_set_params(h, _ptr(src)))


def pp_mlp_set_normalization(h, in_mean, in_std, out_mean, out_std):
    import numpy as np

    a = [np.ascontiguousarray(v, dtype=np.float64) for v in (in_mean, in_std, out_mean, out_std)]
    return _check(lib().pp_mlp_set_normalization(h, *[_hptr(v) for v in a]))


def pp_mlp_forward(h, X, Y):
    return _check(lib().pp_mlp_forward(h, int(X.shape[0]), _ptr(X), _ptr(Y)))


def pp_mlp_loss_grad(h, X, T, grad=None):
    loss = C.c_double()
    _check(lib().pp_mlp_loss_grad(h, int(X.shape[0]), _ptr(X), _ptr(T), _ptr(grad), C.byref(loss)))
    return loss.value


def pp_mlp_train_step(h, X, T, lr):
    loss = C.c_double()
    _check(lib().pp_mlp_train_step(h, int(X.shape[0]), _ptr(X), _ptr(T), float(lr), C.byref(loss)))
    return loss.value


def pp_features(op, power_steps=8):
    import numpy as np

    f = np.zeros(NFEAT)
    _check(lib().pp_features(op, int(power_steps), _hptr(f)))
    return f


def pp_predict_bounds(op, mlp, power_steps=8):
    """Returns (lambda_min, lambda_max, xi, fallback)."""
    lo, hi, xi = C.c_double(), C.c_double(), C.c_double()
    fb = C.c_int()
    _check(lib().pp_predict_bounds(op, mlp, int(power_steps), C.byref(lo), C.byref(hi), C.byref(xi),
                                   C.byref(fb)))
    return lo.value, hi.value, xi.value, bool(fb.value)


# ---------------------------------------------------------------------------
# convenience: upload host CSR / Schur parts and own the handle
# ---------------------------------------------------------------------------

class Operator:
    """Owns a pp_op built from host CSR arrays (or Schur parts) uploaded to ``device``."""

    def __init__(self, a=None, schur=None, dfn=None, flags=0, device="cuda:0", stream=None):
        import torch

        self.device = torch.device(device)
        dev = self.device

        def up(x, dt):
            return torch.from_numpy(x).to(device=dev, dtype=dt).contiguous()

        if dfn is not None:
            d = dfn
            self.n = d.n_u
            self._dev = {}
            for nm in ("a", "gh", "c", "b", "gu"):
                m = getattr(d, nm)
                self._dev[nm] = (m.n_rows, m.n_cols, up(m.rowptr, torch.int64), up(m.col, torch.int32),
                                 up(m.val, torch.float64))
            self.handle = pp_create_dfn(d.n_frac, d.grid, self._dev, d.u_off, d.alpha, flags, stream)
            self._dev = None
        elif schur is not None:
            s = schur
            self.n = s.a.n_rows
            self.handle = pp_create_schur(
                s.a.n_rows, s.a.nnz, up(s.a.rowptr, torch.int64), up(s.a.col, torch.int32),
                up(s.a.val, torch.float64), s.c.n_rows, s.c.nnz, up(s.c.rowptr, torch.int64),
                up(s.c.col, torch.int32), up(s.c.val, torch.float64), up(s.m, torch.float64), flags,
                stream)
        else:
            self.n = a.n_rows
            self.handle = pp_create_csr(a.n_rows, a.nnz, up(a.rowptr, torch.int64),
                                        up(a.col, torch.int32), up(a.val, torch.float64), flags,
                                        stream)

    def close(self):
        if self.handle:
            pp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
