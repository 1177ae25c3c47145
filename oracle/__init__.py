"""CPU oracle for two-phase CSR SpGEMM and the learned row-size predictor.

TEST INFRASTRUCTURE ONLY.  Nothing in the ``paper_2103_11991_amd`` package
imports this package; only ``tests/``, ``__graft_entry__.smoke()`` and the
benchmark's CPU-baseline leg do.  It shares no code with the GPU library:
``oracle.c`` is plain C built with gcc, ``mlp.py`` is plain numpy in FP64.

* ``spgemm``          Gustavson with a dense accumulator (section 2.2.1, Eq. (1));
* ``row_nnz``         its symbolic phase alone (section 2.2.1);
* ``mlp``             forward, backward and Adam training of the 3-32-32-1
                      row-size predictor, in FP64 (parity unpinned against the
                      paper, which has no such network; pinned against finite
                      differences and closed-form special cases instead).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (FP contraction off)."""
    if force or not os.path.exists(_SO):
        src = os.path.join(_HERE, "oracle.c")
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                               "-shared", "-fPIC", "-std=c11", src, "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=True)
        L = ctypes.CDLL(_SO)
        i32, i64, p = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
        L.oracle_row_nnz.argtypes = [i32, i32, i32, p, p, p, p, i32, i32, p]
        L.oracle_row_nnz.restype = ctypes.c_int
        L.oracle_fill.argtypes = [i32, i32, i32, p, p, p, p, p, p, i32, i32, p, p, p, p]
        L.oracle_fill.restype = ctypes.c_int
        L.oracle_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def row_nnz(A, B, r0: int = 0, r1: int | None = None) -> np.ndarray:
    """Symbolic phase: int64 count of distinct columns of each C row in [r0, r1)."""
    r1 = A.m if r1 is None else r1
    if A.n != B.m:
        raise ValueError("inner dimensions differ")
    rpA, ciA, rpB, ciB = _i32(A.row_ptr), _i32(A.col_idx), _i32(B.row_ptr), _i32(B.col_idx)
    out = np.zeros(max(r1 - r0, 0), dtype=np.int64)
    if r1 <= r0:
        return out
    rc = lib().oracle_row_nnz(A.m, A.n, B.n, _ptr(rpA), _ptr(ciA), _ptr(rpB), _ptr(ciB), r0, r1, _ptr(out))
    if rc != 0:
        raise RuntimeError(f"oracle_row_nnz failed ({rc})")
    return out


def spgemm(A, B, r0: int = 0, r1: int | None = None):
    """Rows [r0, r1) of C = A*B.

    Returns ``(row_ptr, cols, vals, absv)``: ``row_ptr`` int64[r1-r0+1] starting
    at 0, sorted int32 columns, FP64 values and FP64 componentwise magnitudes
    sum |A(i,j)||B(j,c)|.
    """
    r1 = A.m if r1 is None else r1
    cnt = row_nnz(A, B, r0, r1)
    rp = np.zeros(cnt.size + 1, dtype=np.int64)
    np.cumsum(cnt, out=rp[1:])
    nnz = int(rp[-1])
    cols = np.empty(nnz, dtype=np.int32)
    vals = np.empty(nnz, dtype=np.float64)
    absv = np.empty(nnz, dtype=np.float64)
    if r1 > r0:
        rpA, ciA, rpB, ciB = _i32(A.row_ptr), _i32(A.col_idx), _i32(B.row_ptr), _i32(B.col_idx)
        vA = np.ascontiguousarray(A.values, dtype=np.float64)
        vB = np.ascontiguousarray(B.values, dtype=np.float64)
        rc = lib().oracle_fill(A.m, A.n, B.n, _ptr(rpA), _ptr(ciA), _ptr(vA), _ptr(rpB), _ptr(ciB), _ptr(vB),
                               r0, r1, _ptr(rp), _ptr(cols), _ptr(vals), _ptr(absv))
        if rc != 0:
            raise RuntimeError(f"oracle_fill failed ({rc})")
    return rp, cols, vals, absv
