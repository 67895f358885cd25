"""The C-ABI library loads without a GPU and exports every function include/mapi.h declares."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mapi.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"^\s*(?:mapi_status|void|const char\s*\*)\s+(\w+)\s*\(", txt, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def libpath():
    import paper_2110_12065_amd as pkg
    if not os.path.exists(pkg.LIB_PATH):
        from paper_2110_12065_amd import build
        build.build()
    return pkg.LIB_PATH


def test_header_declares_the_entry_points():
    names = _declared()
    for must in ("mapi_create", "mapi_destroy", "mapi_solve", "rpi_solve", "mapi_mavp", "mapi_pca_topk",
                 "mapi_pagerank", "mapi_quantize", "mapi_mingram", "mapi_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol(libpath):
    lib = ctypes.CDLL(libpath)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_checked_library_exports_the_same_symbols():
    # the device-checked build (MAPI_DEVICE_CHECKS) is the same ABI
    import paper_2110_12065_amd as pkg
    from paper_2110_12065_amd import build
    path = build.LIB_CHECKED
    if not os.path.exists(path):
        pytest.skip("libmapi_checked.so not built (python -m paper_2110_12065_amd.build)")
    lib = ctypes.CDLL(path)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    lib.mapi_version.restype = ctypes.c_char_p
    assert lib.mapi_version()
    assert os.path.basename(pkg.LIB_PATH) in ("libmapi.so", "libmapi_checked.so")


def test_binding_signatures_cover_header(libpath):
    import paper_2110_12065_amd as pkg
    declared = set(_declared())
    bound = set(pkg._SIGS)
    assert bound <= declared, bound - declared


def test_version_and_error_string_without_gpu(libpath):
    lib = ctypes.CDLL(libpath)
    lib.mapi_version.restype = ctypes.c_char_p
    lib.mapi_last_error.restype = ctypes.c_char_p
    assert lib.mapi_version().startswith(b"mapi-gfx950")
    assert lib.mapi_last_error() == b""


def test_null_arguments_are_rejected_without_gpu(libpath):
    import paper_2110_12065_amd as pkg
    L = pkg.lib()
    assert L.mapi_create(0, None, None) == 1          # MAPI_ERR_ARG, no device touched
    assert L.mapi_solve(None, None, None, None, None, None) == 1
    assert L.mapi_pagerank(None, None, 0.85, 0, None, None, None, None) == 1
    assert b"NULL" in L.mapi_last_error()


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in r.stdout
