"""The C-ABI library loads without a GPU and exports every symbol the header declares.

No compute call is made here: only argument validation that returns before
any device work.
"""
import ctypes as C
import os
import re

import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "pp.h")


def header_functions():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^PP_API\s+[\w\s\*]*?\b(\w+)\s*\(", txt, re.M)))


@pytest.fixture(scope="module")
def B():
    from paper_2208_01339_amd import binding, build

    if build.stale():
        build.build(verbose=False)
    binding.lib()
    return binding


def test_header_lists_the_boundary():
    fns = header_functions()
    for f in ("pp_create_csr", "pp_create_schur", "pp_setup", "pp_apply", "pcg_solve"):
        assert f in fns


def test_every_declared_symbol_is_exported(B):
    L = C.CDLL(B.LIB_PATH)
    missing = [f for f in header_functions() if not hasattr(L, f)]
    assert not missing, missing
    assert sorted(B.ABI_FUNCTIONS) == header_functions()


def test_status_strings(B):
    for code, name in [(0, "PP_OK"), (1, "PP_NOT_CONVERGED"), (2, "PP_BREAKDOWN"), (-1, "PP_ERR_ARG"),
                       (-2, "PP_ERR_OOM"), (-3, "PP_ERR_HIP"), (-4, "PP_ERR_STATE"),
                       (-5, "PP_ERR_TIMEOUT")]:
        assert B.pp_status_str(code) == name


def test_argument_validation_without_device_work(B):
    L = B.lib()
    h = C.c_void_p()
    assert L.pp_create_csr(None, 10, 10, None, None, None, 0, None) == B.PP_ERR_ARG
    assert L.pp_create_csr(C.byref(h), 0, 5, None, None, None, 0, None) == B.PP_ERR_ARG
    assert "positive" in B.pp_last_error()
    assert L.pp_create_csr(C.byref(h), 10, 10, C.c_void_p(8), C.c_void_p(8), C.c_void_p(8), 64, None) == B.PP_ERR_ARG
    assert L.pp_create_schur(C.byref(h), 10, 10, C.c_void_p(8), C.c_void_p(8), C.c_void_p(8), 0, 0, None, None,
                             None, None, 0, None) == B.PP_ERR_ARG
    assert L.pp_setup(None, 3, 0.1, 1.0, 0.0) == B.PP_ERR_ARG
    assert L.pp_apply(None, None, None) == B.PP_ERR_ARG
    assert L.pcg_solve(None, None, None, 1e-8, 10, None, None) == B.PP_ERR_ARG
    lo, hi = C.c_double(), C.c_double()
    assert L.pp_estimate_bounds(None, 20, C.byref(lo), C.byref(hi)) == B.PP_ERR_ARG
    assert L.pp_operator_apply(None, None, None) == B.PP_ERR_ARG
    assert L.pp_set_option(None, 1, 0) == B.PP_ERR_ARG
    L.pp_destroy(None)


def test_every_entry_point_refuses_null_handles(B):
    """Each entry point taking a handle returns PP_ERR_ARG for a NULL one (no device work)."""
    L = B.lib()
    d = C.c_double()
    i = C.c_int()
    i64 = C.c_int64()
    P = C.c_void_p(8)  # never dereferenced: the NULL handle is refused first
    calls = [
        lambda: L.pp_create_dfn(None, None, 0, None), lambda: L.pp_dfn_rhs(None, P, P),
        lambda: L.pp_dfn_recover(None, P, P, P, P), lambda: L.pp_setup_newton(None, 2, 0.1, 1.0, 0.0),
        lambda: L.pp_lowrank_set(None, 1, P), lambda: L.pp_lowrank_ritz(None, 10, 1, None),
        lambda: L.pp_lowrank_get(None, C.byref(i), None), lambda: L.pp_lowrank_info(None, None, None),
        lambda: L.pp_get_stats(None, None), lambda: L.pp_batch_estimate_bounds(None, 20, P, P),
        lambda: L.pp_batch_setup(None, 3, P, P, 0.0), lambda: L.pcg_solve_batch(None, P, P, 1e-8, 10, P, P, P),
        lambda: L.pp_batch_apply(None, P, P), lambda: L.pp_batch_set_layout(None, 1),
        lambda: L.pp_batch_autotune(None, C.byref(i), C.byref(d)), lambda: L.pp_batch_set_option(None, 2, 1),
        lambda: L.pp_batch_get_stats(None, None), lambda: L.pp_mlp_num_params(None, C.byref(i64)),
        lambda: L.pp_mlp_get_params(None, P), lambda: L.pp_mlp_set_params(None, P),
        lambda: L.pp_mlp_forward(None, 1, P, P), lambda: L.pp_features(None, 8, P),
        lambda: L.pp_predict_bounds(None, None, 8, C.byref(d), C.byref(d), C.byref(d), C.byref(i)),
    ]
    for k, f in enumerate(calls):
        assert f() == B.PP_ERR_ARG, k
    L.pp_destroy_batch(None)
    L.pp_mlp_destroy(None)


def test_noalloc_argument_validation_without_device_work(B):
    """The allocation-free solve checks its arguments before it looks for a device."""
    L = B.lib()
    P = C.c_void_p(8)

    def call(n=100, nnz=500, flags=0, k=4, lmin=0.1, lmax=2.0, xi=0.0, tol=1e-8, maxit=10, b=P, x=C.c_void_p(16)):
        return L.pcg_solve_csr_noalloc(n, nnz, P, P, P, flags, k, lmin, lmax, xi, b, x, tol, maxit, None, None, None)

    for kw in [dict(n=0), dict(n=(1 << 20) + 1), dict(nnz=-1), dict(flags=2), dict(k=-1), dict(k=1025),
               dict(lmin=0.0), dict(lmax=0.05), dict(lmin=float("nan")), dict(xi=-1.0), dict(tol=-1.0),
               dict(maxit=-1), dict(b=None), dict(x=P)]:
        assert call(**kw) == B.PP_ERR_ARG, kw
    assert "1048576" in (call(n=(1 << 20) + 1), B.pp_last_error())[1]


def test_product_path_refuses_missing_library(monkeypatch, tmp_path):
    from paper_2208_01339_amd import binding

    monkeypatch.setattr(binding, "_lib", None)
    monkeypatch.setattr(binding, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError):
        binding.lib()
