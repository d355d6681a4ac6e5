"""The C ABI library, checked without a GPU: it loads, exports every function
declared in include/plm.h, and its host-only entry points behave."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "plm.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = set(re.findall(r"\b(plm_[a-z_0-9]+)\s*\(", txt))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    from paper_1401_4832_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libplm.so not built")
    return _lib.lib()


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("plm_reweight", "plm_objgrad", "plm_fit", "plm_score", "plm_fit_workspace_bytes",
              "plm_objgrad_workspace_bytes", "plm_ctx_create", "plm_status_string"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_header():
    from paper_1401_4832_amd import _lib
    assert set(_lib.exported_symbols()) == set(_declared())


def test_status_strings(lib):
    for code in (0, 1, -1, -2, -3, -4, -5, -6):
        assert lib.plm_status_string(code)


def test_workspace_sizes_are_host_computable(lib):
    from paper_1401_4832_amd import _lib
    small = lib.plm_objgrad_workspace_bytes(500, 40, 21, 0)
    large = lib.plm_objgrad_workspace_bytes(50000, 500, 21, 0)
    assert 0 < small < large
    # rejected sizes give zero
    assert lib.plm_objgrad_workspace_bytes(500, 40, 22, 0) == 0
    assert lib.plm_objgrad_workspace_bytes(0, 40, 21, 0) == 0
    o = _lib.FitOpts()
    lib.plm_fit_opts_default(ctypes.byref(o))
    assert o.lbfgs_m == 10 and o.tol == 1e-6 and o.lambda_h == 0.01 and o.lambda_J == 0.01
    fit_ws = lib.plm_fit_workspace_bytes(50000, 500, 21, ctypes.byref(o))
    # the L-BFGS history dominates: 2 (m + 1) N^2 q^2 FP32 values
    assert fit_ws > 2 * 11 * 500 * 500 * 441 * 4
    o.lbfgs_m = 0
    assert lib.plm_fit_workspace_bytes(500, 40, 21, ctypes.byref(o)) == 0


def test_null_context_is_rejected(lib):
    assert lib.plm_sync(None) == -1
    assert lib.plm_score(None, None, 10, 21, None, None) == -1


def test_fit_options_layout_matches_the_library(lib):
    from paper_1401_4832_amd import _lib
    assert lib.plm_fit_opts_size() == ctypes.sizeof(_lib.FitOpts)
    o = _lib.FitOpts()
    lib.plm_fit_opts_default(ctypes.byref(o))
    assert o.refine_tol == 0.0 and o.n_probe == 0 and o.history_fp64 == 0 and not o.probe_out
