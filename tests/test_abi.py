"""The C ABI: the library loads, exports every declared entry point, and
rejects bad arguments before touching the GPU (no compute calls here)."""
import ctypes
import os
import re

import pytest

from paper_2504_13446_amd import rkr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rkr.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rkr_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("rkr_build", "rkr_query_exact", "rkr_query_approx", "rkr_query_batch",
                     "rkr_ranks", "rkr_destroy", "rkr_stats", "rkr_last_error"):
        assert required in names
    assert set(names) == set(rkr.SYMBOLS)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(rkr.LIB_PATH):
        pytest.skip("librkr.so not built")
    L = ctypes.CDLL(rkr.LIB_PATH)
    for name in _declared():
        assert hasattr(L, name), name


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(rkr.LIB_PATH):
        pytest.skip("librkr.so not built")
    return rkr.load()


def _err(L):
    return L.rkr_last_error().decode()


def test_build_validation_before_device_work(L):
    h = ctypes.c_void_p()
    dummy = ctypes.c_void_p(16)
    assert L.rkr_build(dummy, 0, dummy, 10, 8, 0, None, ctypes.byref(h)) == rkr.RKR_E_INVALID
    assert "n must be positive" in _err(L)
    assert L.rkr_build(dummy, 10, dummy, -1, 8, 0, None, ctypes.byref(h)) == rkr.RKR_E_INVALID
    assert L.rkr_build(dummy, 10, dummy, 10, 0, 0, None, ctypes.byref(h)) == rkr.RKR_E_INVALID
    assert L.rkr_build(dummy, 10, dummy, 10, 5000, 0, None, ctypes.byref(h)) == rkr.RKR_E_INVALID
    assert L.rkr_build(dummy, 10, dummy, 10, 8, 7, None, ctypes.byref(h)) == rkr.RKR_E_INVALID
    assert L.rkr_build(None, 10, dummy, 10, 8, 0, None, ctypes.byref(h)) == rkr.RKR_E_INVALID
    assert L.rkr_build(dummy, 10, None, 10, 8, 0, None, ctypes.byref(h)) == rkr.RKR_E_INVALID
    assert L.rkr_build(dummy, 1 << 31, dummy, 10, 8, 0, None, ctypes.byref(h)) == rkr.RKR_E_UNSUPPORTED
    bad_score = rkr.BuildOpts(9, 1, 0, 0, None)
    assert L.rkr_build(dummy, 10, dummy, 10, 8, 0, ctypes.byref(bad_score), ctypes.byref(h)) == rkr.RKR_E_INVALID
    bad_table = rkr.BuildOpts(1, 1, 0, -5, None)
    assert L.rkr_build(dummy, 10, dummy, 10, 8, 0, ctypes.byref(bad_table), ctypes.byref(h)) == rkr.RKR_E_INVALID
    assert "rank_table" in _err(L)
    # d beyond what the count kernel supports for BF16 scoring
    assert L.rkr_build(dummy, 10, dummy, 10, 4000, 0, None, ctypes.byref(h)) == rkr.RKR_E_UNSUPPORTED
    # split BF16 rows hold 3d terms: d = 107 needs 321 > 320
    split = rkr.BuildOpts(rkr.RKR_SCORE_BF16X3, 1, 0, 0, None)
    assert L.rkr_build(dummy, 10, dummy, 10, 107, 0, ctypes.byref(split), ctypes.byref(h)) == rkr.RKR_E_UNSUPPORTED
    assert "max 106" in _err(L)
    assert h.value is None
    assert L.rkr_build(dummy, 10, dummy, 10, 8, 0, None, None) == rkr.RKR_E_INVALID


def test_null_index_calls(L):
    k = (ctypes.c_int32 * 1)(5)
    assert L.rkr_query_batch(None, 1, None, k, None, None, None, None, None) == rkr.RKR_E_INVALID
    assert L.rkr_query_exact(None, None, 5, None, None) == rkr.RKR_E_INVALID
    assert L.rkr_query_approx(None, None, 5, 0.5, None, None) == rkr.RKR_E_INVALID
    assert "c must be >= 1" in _err(L)
    assert L.rkr_query_approx(None, None, 5, float("nan"), None, None) == rkr.RKR_E_INVALID
    assert L.rkr_ranks(None, None, None) == rkr.RKR_E_INVALID
    assert L.rkr_rank_table(None, None, None) == rkr.RKR_E_INVALID
    assert L.rkr_configure(None, None) == rkr.RKR_E_INVALID
    s = rkr.QueryStats()
    assert L.rkr_stats(None, ctypes.byref(s)) == rkr.RKR_E_INVALID
    L.rkr_destroy(None)
    assert L.rkr_train(None, 1, None, 10, 1, 10, 0.1, 0) == rkr.RKR_E_INVALID


def test_error_message_is_thread_local(L):
    import threading
    h = ctypes.c_void_p()
    dummy = ctypes.c_void_p(16)
    assert L.rkr_build(dummy, 0, dummy, 10, 8, 0, None, ctypes.byref(h)) == rkr.RKR_E_INVALID
    seen = []
    t = threading.Thread(target=lambda: seen.append(_err(L)))
    t.start(); t.join()
    assert seen == [""]
    assert "n must be positive" in _err(L)


def test_table_width_matches_header():
    src = open(HEADER).read()
    m = re.search(r"#define\s+RKR_TABLE_COLS\s+(\d+)", src)
    assert m and int(m.group(1)) == rkr.TABLE_COLS
