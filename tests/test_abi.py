"""The C-ABI library loads and exports every entry point include/smki.h
declares; host-side argument checks answer without touching a GPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "smki.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(smki_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1909_04631_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1909_04631_amd import build
        build.build()
    return _lib.lib()


def test_every_declared_symbol_is_exported(lib):
    from paper_1909_04631_amd import _lib
    syms = declared_symbols()
    assert len(syms) >= 17
    for s in syms:
        assert hasattr(lib, s), f"{s} declared in smki.h but not exported"
    assert sorted(_lib.EXPORTED) == syms


def test_status_strings(lib):
    assert lib.smki_status_string(0) == b"ok"
    for code in range(-6, 0):
        assert lib.smki_status_string(code) not in (b"", b"unknown status")


def test_host_argument_checks_need_no_gpu(lib):
    from paper_1909_04631_amd._lib import Options
    h = C.c_void_p()
    # non-positive resolution, K out of range, block size not supported, bad free class
    assert lib.smki_create_map(0.0, 8, 0.3, 0.1, 4, 1e-3, 0, None, C.byref(h)) == -1
    assert lib.smki_create_map(0.1, 8, 0.3, 0.1, 1, 1e-3, 0, None, C.byref(h)) == -1
    # block sizes: powers of two in [1, 32]
    for bad_b in (0, 3, 6, 12, 64, -8):
        assert lib.smki_create_map(0.1, bad_b, 0.3, 0.1, 4, 1e-3, 0, None, C.byref(h)) == -1
    assert lib.smki_create_map(0.1, 8, 0.3, 0.1, 4, 1e-3, 4, None, C.byref(h)) == -1
    assert lib.smki_create_map(0.1, 8, float("nan"), 0.1, 4, 1e-3, 0, None, C.byref(h)) == -1
    for bad in (Options(-1, 0), Options(0, -1), Options(0, (1 << 24) + 1), Options(0, 0, 2),
                Options(0, 0, 0, 2), Options(0, 0, 0, 0, 2)):
        assert lib.smki_create_map(0.1, 8, 0.3, 0.1, 4, 1e-3, 0, C.byref(bad), C.byref(h)) == -1
    assert lib.smki_insert_scan(None, None, None, 0, None, 0.3) == -1
    from paper_1909_04631_amd._lib import ALLOC_FN, RELEASE_FN
    assert lib.smki_set_allocator(None, ALLOC_FN(), RELEASE_FN(), None) == -1
    assert lib.smki_batch_replay(None, None, None) == -1
    assert lib.smki_batch_destroy(None) == -1
    hb = C.c_void_p()
    assert lib.smki_batch_capture(None, None, None, None, None, 1, 0.3, 0.25, C.byref(hb)) == -1
    assert lib.smki_query(None, None, 0, None, None, None, None, None) == -1
    assert lib.smki_set_kernel_timing(None, 0) == -1
    n = C.c_int64()
    o = (C.c_float * 3)(0, 0, 0)
    assert lib.smki_free_samples(None, None, -1, o, 0.3, 4, None, C.byref(n), None, None) == -1
    assert lib.smki_bucket_cells(None, 5, 0.1, 8, None, C.byref(n), None, None, None, None) == -1
    assert lib.smki_loss_forward(None, None, 0, None, None, 0, 0.3, 1.0, 1e-3, 4, None, None, 0,
                                 None, None) == -1
    assert lib.smki_loss_workspace_bytes(1000, 100, 4) > 0


def test_product_path_has_no_cpu_fallback():
    # the package imports torch and the ctypes binding only; nothing under oracle/
    pkg = os.path.join(ROOT, "paper_1909_04631_amd")
    for f in os.listdir(pkg):
        if f.endswith(".py"):
            src = open(os.path.join(pkg, f)).read()
            assert "oracle" not in src.replace("correctness oracle", ""), f
