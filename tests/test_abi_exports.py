"""The C-ABI library loads on the host and exports every function include/spg.h declares."""
import ctypes
import os
import re

from paper_2103_11991_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "spg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(spg_[a-z_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    names = declared()
    assert "spg_symbolic" in names and "spg_numeric" in names
    L = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert sorted(_lib.EXPORTS) == names


def test_status_strings_and_argument_errors_without_gpu():
    assert _lib.spg_status_string(0) == "SPG_OK"
    assert _lib.spg_status_string(5) == "SPG_ERR_OVERFLOW"
    L = _lib.load()
    assert L.spg_create(None, None) == 1  # null output pointer -> SPG_ERR_ARG
    assert L.spg_destroy(None) == 0
    assert L.spg_mlp_forward(None, None, None, -1, None, None) == 1


def test_stats_struct_layout_matches_header():
    # 4 ints, 2 int64, 2x30 int32, 3x30 int64, 4 int32, 2 floats, 2x30 floats, 3 floats, then an
    # int64 on an 8-byte boundary
    expect = 16 + 16 + 240 + 720 + 16 + 8 + 240 + 12
    expect += -expect % 8
    assert _lib.spg_stats.list_pairs.offset == expect
    # then 30 floats, 30 int32 and four int32
    assert ctypes.sizeof(_lib.spg_stats) == expect + 8 + 120 + 120 + 16
