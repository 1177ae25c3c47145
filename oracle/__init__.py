"""CPU oracle for two-phase CSR SpGEMM and the learned row-size predictor.

TEST INFRASTRUCTURE ONLY.  Nothing in the ``paper_2103_11991_amd`` package
imports this package; only ``tests/``, ``__graft_entry__.smoke()`` and the
benchmark's CPU-baseline leg do.  It shares no code with the GPU library:
``oracle.c`` is plain C built with gcc, ``mlp.py`` is plain numpy in FP64.

* ``spgemm``          Gustavson with a dense accumulator (section 2.2.1, Eq. (1));
* ``row_nnz``         its symbolic phase alone (section 2.2.1);
* ``jacobi_spgemm``   C = (I - omega D^-1 A) B composed from the paper's three
                      kernels: SpGEMM, row scaling, addition (section 2.2.2);
* ``spadd``           C = alpha A + beta B: union of the row patterns,
                      entries of one column merged by addition (section 2.3);
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
        L.oracle_set_num_threads.argtypes = [ctypes.c_int]
        L.oracle_set_num_threads.restype = None
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def set_num_threads(n: int) -> None:
    """Host threads of later oracle calls."""
    lib().oracle_set_num_threads(int(n))


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


def _rows_slice(A, r0: int, r1: int):
    """Row ids, columns and FP64 values of the entries of rows [r0, r1), in stored order."""
    rp = A.row_ptr.astype(np.int64)
    s, e = int(rp[r0]), int(rp[r1])
    rows = np.repeat(np.arange(r0, r1, dtype=np.int64), np.diff(rp[r0:r1 + 1]))
    return rows, A.col_idx[s:e].astype(np.int64), A.values[s:e].astype(np.float64)


def _merge_rows(r0: int, r1: int, rows, cols, vals, absv):
    """Entries (row, col, value) in their given order -> CSR rows [r0, r1): one
    entry per distinct (row, col), values summed in the given order, columns
    ascending.  Returns (row_ptr int64 from 0, cols int32, vals, absv)."""
    nrows = max(r1 - r0, 0)
    order = np.lexsort((np.arange(rows.size), cols, rows))  # stable: keeps the given order of equal keys
    rows, cols, vals, absv = rows[order], cols[order], vals[order], absv[order]
    new = np.ones(rows.size, dtype=bool)
    if rows.size:
        new[1:] = (rows[1:] != rows[:-1]) | (cols[1:] != cols[:-1])
    starts = np.flatnonzero(new)
    out_rows, out_cols = rows[starts], cols[starts]
    if rows.size:
        # sums inside each run of equal keys, left to right in the given order
        # (one step per position in the run, all runs at once)
        lens = np.diff(np.append(starts, rows.size))
        out_vals = vals[starts].copy()
        out_abs = absv[starts].copy()
        for k in range(1, int(lens.max())):
            sel = lens > k
            out_vals[sel] += vals[starts[sel] + k]
            out_abs[sel] += absv[starts[sel] + k]
    else:
        out_vals = np.zeros(0)
        out_abs = np.zeros(0)
    cnt = np.bincount(out_rows - r0, minlength=nrows) if nrows else np.zeros(0, dtype=np.int64)
    rp = np.zeros(nrows + 1, dtype=np.int64)
    np.cumsum(cnt, out=rp[1:])
    return rp, out_cols.astype(np.int32), out_vals, out_abs


def spadd(A, B, alpha: float, beta: float, r0: int = 0, r1: int | None = None):
    """Rows [r0, r1) of C = alpha*A + beta*B (section 2.3), A and B of the same
    shape.  Each row of C holds the union of the columns of A(i,:) and
    B(i,:); entries of one column (from A, from B, and repeats inside either)
    are merged by addition, A's contributions first and each matrix's in its
    stored order; columns ascending; explicit zeros kept.  Each contribution
    is rounded once (alpha * a, beta * b) before it is added.

    Returns ``(row_ptr, cols, vals, absv)`` like ``spgemm``; ``absv`` sums
    |alpha a| and |beta b| over the merged contributions (the scale of the
    summation's rounding error)."""
    if (A.m, A.n) != (B.m, B.n):
        raise ValueError("A and B must have the same shape")
    r1 = A.m if r1 is None else r1
    ra, ca, va = _rows_slice(A, r0, r1)
    rb, cb, vb = _rows_slice(B, r0, r1)
    fa, fb = alpha * va, beta * vb
    return _merge_rows(r0, r1, np.concatenate([ra, rb]), np.concatenate([ca, cb]), np.concatenate([fa, fb]),
                       np.concatenate([np.abs(fa), np.abs(fb)]))


def jacobi_spgemm(A, B, omega: float, dinv: np.ndarray, r0: int = 0, r1: int | None = None):
    """Rows [r0, r1) of C = (I - omega D^-1 A) B (section 2.2.2), A square
    (m x m), B m x k, ``dinv`` the m entries of D^-1.  Composed as the
    paper's three unfused kernels: E = A*B (``spgemm``), F = D^-1 E (row i of
    E times dinv[i]), and C = B - omega F (``spadd`` with alpha = 1, beta =
    -omega).  Returns ``(row_ptr, cols, vals, absv)`` like ``spgemm``;
    ``absv`` = |B(i,c)| + |omega dinv[i]| sum_j |A(i,j)||B(j,c)|, the scale of
    the rounding error of the whole composition."""
    if A.m != A.n or A.n != B.m:
        raise ValueError("A must be square with as many columns as B has rows")
    r1 = A.m if r1 is None else r1
    rpE, cE, vE, aE = spgemm(A, B, r0, r1)
    rowsE = np.repeat(np.arange(r0, r1, dtype=np.int64), np.diff(rpE))
    d = np.asarray(dinv, dtype=np.float64)
    vF = d[rowsE] * vE
    rb, cb, vb = _rows_slice(B, r0, r1)
    rows = np.concatenate([rb, rowsE])
    cols = np.concatenate([cb, cE.astype(np.int64)])
    vals = np.concatenate([vb, -omega * vF])
    absv = np.concatenate([np.abs(vb), np.abs(omega * d[rowsE]) * aE])
    return _merge_rows(r0, r1, rows, cols, vals, absv)
