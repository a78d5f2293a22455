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
                       (-2, "PP_ERR_OOM"), (-3, "PP_ERR_HIP"), (-4, "PP_ERR_STATE")]:
        assert B.pp_status_str(code) == name


def test_argument_validation_without_device_work(B):
    L = B.lib()
    h = C.c_void_p()
    assert L.pp_create_csr(None, 10, 10, None, None, None, 0, None) == B.PP_ERR_ARG
    assert L.pp_create_csr(C.byref(h), 0, 5, None, None, None, 0, None) == B.PP_ERR_ARG
    assert "positive" in B.pp_last_error()
    assert L.pp_create_csr(C.byref(h), 10, 10, C.c_void_p(8), C.c_void_p(8), C.c_void_p(8), 8, None) == B.PP_ERR_ARG
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


def test_product_path_refuses_missing_library(monkeypatch, tmp_path):
    from paper_2208_01339_amd import binding

    monkeypatch.setattr(binding, "_lib", None)
    monkeypatch.setattr(binding, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError):
        binding.lib()
