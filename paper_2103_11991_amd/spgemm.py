"""Torch-facing wrapper of the spg C ABI (device memory and streams only).

    op = SpGEMM(A, B)                 # A, B: DeviceCsr on the GPU
    row_ptr, nnz = op.symbolic()      # section 2.2.1: row sizes, scanned
    col, val = op.numeric()           # column indices and values of C
    col, val = op.numeric(a_vals=new) # reuse of the symbolic result

Every step of the product runs in libspg.so; this module allocates the
output tensors with torch and passes pointers and the current stream.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from . import _lib


@dataclass
class DeviceCsr:
    m: int
    n: int
    row_ptr: torch.Tensor   # int32[m+1], on the GPU
    col_idx: torch.Tensor   # int32[nnz]
    values: torch.Tensor    # float32 or float64 [nnz]

    @property
    def nnz(self) -> int:
        return int(self.col_idx.numel())

    @staticmethod
    def from_host(csr, device="cuda") -> "DeviceCsr":
        """Copies a host CSR (any object with m, n, row_ptr, col_idx, values) to the GPU."""
        return DeviceCsr(int(csr.m), int(csr.n),
                         torch.from_numpy(np.ascontiguousarray(csr.row_ptr, dtype=np.int32)).to(device),
                         torch.from_numpy(np.ascontiguousarray(csr.col_idx, dtype=np.int32)).to(device),
                         torch.from_numpy(np.ascontiguousarray(csr.values)).to(device))


def _dtype_code(t: torch.dtype) -> int:
    if t == torch.float64:
        return _lib.SPG_F64
    if t == torch.float32:
        return _lib.SPG_F32
    raise TypeError(f"values must be float32 or float64, got {t}")


def _check_tensor(t: torch.Tensor, dtype, n: int, what: str):
    if not t.is_cuda:
        raise ValueError(f"{what} must be on the GPU")
    if t.dtype != dtype:
        raise TypeError(f"{what} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if t.numel() != n:
        raise ValueError(f"{what} has {t.numel()} elements, expected {n}")


class SpGEMM:
    """Two-phase C = A*B bound to one handle and one stream."""

    def __init__(self, A: DeviceCsr, B: DeviceCsr, stream: torch.cuda.Stream | None = None, **options):
        if A.n != B.m:
            raise ValueError(f"inner dimensions differ: A is {A.m}x{A.n}, B is {B.m}x{B.n}")
        self.A, self.B = A, B
        self.dtype = A.values.dtype
        if B.values.dtype != self.dtype:
            raise TypeError("A and B values must have the same dtype")
        for t, n, nm in ((A.row_ptr, A.m + 1, "A.row_ptr"), (B.row_ptr, B.m + 1, "B.row_ptr")):
            _check_tensor(t, torch.int32, n, nm)
        _check_tensor(A.col_idx, torch.int32, A.nnz, "A.col_idx")
        _check_tensor(B.col_idx, torch.int32, B.nnz, "B.col_idx")
        self.stream = stream or torch.cuda.current_stream()
        self.h = _lib.spg_create(self.stream.cuda_stream)
        for k, v in options.items():
            _lib.spg_set_option(self.h, k, int(v))
        self.set_matrices(A, B)

    def set_matrices(self, A: DeviceCsr, B: DeviceCsr):
        """New matrices on the same handle (its buffers are kept and grown as
        needed); the symbolic result of the old ones is dropped."""
        if A.n != B.m:
            raise ValueError(f"inner dimensions differ: A is {A.m}x{A.n}, B is {B.m}x{B.n}")
        if B.values.dtype != A.values.dtype:
            raise TypeError("A and B values must have the same dtype")
        for t, n, nm in ((A.row_ptr, A.m + 1, "A.row_ptr"), (B.row_ptr, B.m + 1, "B.row_ptr")):
            _check_tensor(t, torch.int32, n, nm)
        _check_tensor(A.col_idx, torch.int32, A.nnz, "A.col_idx")
        _check_tensor(B.col_idx, torch.int32, B.nnz, "B.col_idx")
        self.A, self.B = A, B
        self.dtype = A.values.dtype
        _lib.spg_set_matrices(self.h, _dtype_code(self.dtype), A.m, A.n, B.n,
                              A.row_ptr.data_ptr(), A.col_idx.data_ptr(), A.nnz,
                              B.row_ptr.data_ptr(), B.col_idx.data_ptr(), B.nnz)
        self.row_ptr = None
        self.nnz = None

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            try:
                _lib.spg_destroy(h)
            except Exception:
                pass
            self.h = None

    def set_option(self, name, value: int):
        _lib.spg_set_option(self.h, name, int(value))

    def set_mlp(self, w: np.ndarray):
        w = np.ascontiguousarray(w, dtype=np.float32)
        _lib.spg_set_mlp(self.h, w.ctypes.data, int(w.size))

    def symbolic(self):
        with torch.cuda.stream(self.stream):
            self.row_ptr = torch.empty(self.A.m + 1, dtype=torch.int32, device=self.A.row_ptr.device)
        self.nnz = _lib.spg_symbolic(self.h, self.row_ptr.data_ptr())
        return self.row_ptr, self.nnz

    def numeric(self, a_vals: torch.Tensor | None = None, b_vals: torch.Tensor | None = None,
                out_col: torch.Tensor | None = None, out_val: torch.Tensor | None = None):
        if self.nnz is None:
            raise RuntimeError("symbolic() must come first")
        a_vals = self.A.values if a_vals is None else a_vals
        b_vals = self.B.values if b_vals is None else b_vals
        _check_tensor(a_vals, self.dtype, self.A.nnz, "a_vals")
        _check_tensor(b_vals, self.dtype, self.B.nnz, "b_vals")
        dev = self.A.row_ptr.device
        with torch.cuda.stream(self.stream):
            if out_col is None:
                out_col = torch.empty(self.nnz, dtype=torch.int32, device=dev)
            if out_val is None:
                out_val = torch.empty(self.nnz, dtype=self.dtype, device=dev)
        _check_tensor(out_col, torch.int32, self.nnz, "out_col")
        _check_tensor(out_val, self.dtype, self.nnz, "out_val")
        _lib.spg_numeric(self.h, a_vals.data_ptr(), b_vals.data_ptr(), out_col.data_ptr(), out_val.data_ptr())
        return out_col, out_val

    def numeric_jacobi(self, omega: float, dinv: torch.Tensor, a_vals: torch.Tensor | None = None,
                       b_vals: torch.Tensor | None = None, out_col: torch.Tensor | None = None,
                       out_val: torch.Tensor | None = None):
        """C = (I - omega D^-1 A) B on the symbolic result of A*B (A square, its
        diagonal stored in every row); ``dinv``: the m entries of D^-1."""
        if self.nnz is None:
            raise RuntimeError("symbolic() must come first")
        a_vals = self.A.values if a_vals is None else a_vals
        b_vals = self.B.values if b_vals is None else b_vals
        _check_tensor(a_vals, self.dtype, self.A.nnz, "a_vals")
        _check_tensor(b_vals, self.dtype, self.B.nnz, "b_vals")
        _check_tensor(dinv, self.dtype, self.A.m, "dinv")
        dev = self.A.row_ptr.device
        with torch.cuda.stream(self.stream):
            if out_col is None:
                out_col = torch.empty(self.nnz, dtype=torch.int32, device=dev)
            if out_val is None:
                out_val = torch.empty(self.nnz, dtype=self.dtype, device=dev)
        _check_tensor(out_col, torch.int32, self.nnz, "out_col")
        _check_tensor(out_val, self.dtype, self.nnz, "out_val")
        _lib.spg_numeric_jacobi(self.h, omega, dinv.data_ptr(), a_vals.data_ptr(), b_vals.data_ptr(),
                                out_col.data_ptr(), out_val.data_ptr())
        return out_col, out_val

    def stats(self) -> dict:
        st = _lib.spg_get_stats(self.h)
        out = {}
        for name, _ in st._fields_:
            v = getattr(st, name)
            out[name] = list(v) if hasattr(v, "__len__") else v
        return out

    def export_rows(self):
        """Predictor training rows of the last symbolic call: (x[m,3], y[m], row_nnz[m])."""
        dev = self.A.row_ptr.device
        with torch.cuda.stream(self.stream):
            x = torch.empty((self.A.m, 3), dtype=torch.float32, device=dev)
            y = torch.empty(self.A.m, dtype=torch.float32, device=dev)
            r = torch.empty(self.A.m, dtype=torch.int32, device=dev)
        _lib.spg_export_rows(self.h, x.data_ptr(), y.data_ptr(), r.data_ptr())
        return x, y, r


class SpAdd:
    """Two-phase C = alpha*A + beta*B (section 2.3) bound to one handle and one stream.

        add = SpAdd(A, B)                       # A, B: DeviceCsr of one shape
        row_ptr, nnz = add.symbolic()           # union of the row patterns
        col, val = add.numeric(alpha, beta)     # any number of times
    """

    def __init__(self, A: DeviceCsr, B: DeviceCsr, stream: torch.cuda.Stream | None = None):
        if (A.m, A.n) != (B.m, B.n):
            raise ValueError(f"shapes differ: A is {A.m}x{A.n}, B is {B.m}x{B.n}")
        if A.values.dtype != B.values.dtype:
            raise TypeError("A and B values must have the same dtype")
        for t, n, nm in ((A.row_ptr, A.m + 1, "A.row_ptr"), (B.row_ptr, B.m + 1, "B.row_ptr")):
            _check_tensor(t, torch.int32, n, nm)
        _check_tensor(A.col_idx, torch.int32, A.nnz, "A.col_idx")
        _check_tensor(B.col_idx, torch.int32, B.nnz, "B.col_idx")
        self.A, self.B = A, B
        self.dtype = A.values.dtype
        self.stream = stream or torch.cuda.current_stream()
        self.h = _lib.spg_add_create(self.stream.cuda_stream)
        self.row_ptr = None
        self.nnz = None

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            try:
                _lib.spg_add_destroy(h)
            except Exception:
                pass
            self.h = None

    def symbolic(self):
        A, B = self.A, self.B
        with torch.cuda.stream(self.stream):
            self.row_ptr = torch.empty(A.m + 1, dtype=torch.int32, device=A.row_ptr.device)
        self.nnz = _lib.spg_add_symbolic(self.h, A.m, A.n, A.row_ptr.data_ptr(), A.col_idx.data_ptr(), A.nnz,
                                         B.row_ptr.data_ptr(), B.col_idx.data_ptr(), B.nnz, self.row_ptr.data_ptr())
        return self.row_ptr, self.nnz

    def numeric(self, alpha: float = 1.0, beta: float = 1.0, a_vals: torch.Tensor | None = None,
                b_vals: torch.Tensor | None = None, out_col: torch.Tensor | None = None,
                out_val: torch.Tensor | None = None):
        if self.nnz is None:
            raise RuntimeError("symbolic() must come first")
        a_vals = self.A.values if a_vals is None else a_vals
        b_vals = self.B.values if b_vals is None else b_vals
        _check_tensor(a_vals, self.dtype, self.A.nnz, "a_vals")
        _check_tensor(b_vals, self.dtype, self.B.nnz, "b_vals")
        dev = self.A.row_ptr.device
        with torch.cuda.stream(self.stream):
            if out_col is None:
                out_col = torch.empty(self.nnz, dtype=torch.int32, device=dev)
            if out_val is None:
                out_val = torch.empty(self.nnz, dtype=self.dtype, device=dev)
        _check_tensor(out_col, torch.int32, self.nnz, "out_col")
        _check_tensor(out_val, self.dtype, self.nnz, "out_val")
        _lib.spg_add_numeric(self.h, _dtype_code(self.dtype), alpha, a_vals.data_ptr(), beta, b_vals.data_ptr(),
                             out_col.data_ptr(), out_val.data_ptr())
        return out_col, out_val


def spgemm(A: DeviceCsr, B: DeviceCsr, **options) -> DeviceCsr:
    """One-shot C = A*B (symbolic, then numeric) on the current stream."""
    op = SpGEMM(A, B, **options)
    rp, nnz = op.symbolic()
    col, val = op.numeric()
    return DeviceCsr(A.m, B.n, rp, col, val)


class SpGEMMBatch:
    """Many independent products C_i = A_i * B_i run as one graph launch.

    Inputs are lists of DeviceCsr; their arrays are concatenated into pools
    (one device copy at construction).  ``plan()`` sizes the C pools,
    ``run()`` launches the captured graph, ``product(i)`` views C_i."""

    @classmethod
    def from_pools(cls, m, n, k, a_nnz, b_nnz, a_rp, a_ci, a_v, b_rp, b_ci, b_v,
                   stream: torch.cuda.Stream | None = None, **options) -> "SpGEMMBatch":
        """Batch over already pooled device arrays (layout of spg_batch_create)."""
        self = cls.__new__(cls)
        self.count = len(m)
        self.dtype = a_v.dtype
        self.stream = stream or torch.cuda.Stream()
        self.stream.wait_stream(torch.cuda.current_stream())
        self.a_rp, self.a_ci, self.a_v, self.b_rp, self.b_ci, self.b_v = a_rp, a_ci, a_v, b_rp, b_ci, b_v
        self.m = np.ascontiguousarray(m, dtype=np.int32)
        self.n = np.ascontiguousarray(n, dtype=np.int32)
        self.k = np.ascontiguousarray(k, dtype=np.int32)
        self.a_nnz = np.ascontiguousarray(a_nnz, dtype=np.int64)
        self.b_nnz = np.ascontiguousarray(b_nnz, dtype=np.int64)
        self._create(options)
        return self

    def __init__(self, As, Bs, stream: torch.cuda.Stream | None = None, **options):
        assert len(As) == len(Bs)
        self.count = len(As)
        self.dtype = As[0].values.dtype if As else torch.float64
        for A, B in zip(As, Bs):
            if A.n != B.m:
                raise ValueError("inner dimensions differ")
            if A.values.dtype != self.dtype or B.values.dtype != self.dtype:
                raise TypeError("all values must share one dtype")
        # graph capture needs a stream of its own (not the legacy default stream);
        # it is ordered after the caller's stream at every entry and before it at exit
        self.stream = stream or torch.cuda.Stream()
        self.stream.wait_stream(torch.cuda.current_stream())
        dev = As[0].row_ptr.device if As else torch.device("cuda")
        cat = lambda ts, dt: torch.cat(ts) if ts else torch.zeros(0, dtype=dt, device=dev)
        with torch.cuda.stream(self.stream):
            self.a_rp = cat([A.row_ptr for A in As], torch.int32)
            self.a_ci = cat([A.col_idx for A in As], torch.int32)
            self.a_v = cat([A.values for A in As], self.dtype)
            self.b_rp = cat([B.row_ptr for B in Bs], torch.int32)
            self.b_ci = cat([B.col_idx for B in Bs], torch.int32)
            self.b_v = cat([B.values for B in Bs], self.dtype)
        self.m = np.array([A.m for A in As], dtype=np.int32)
        self.n = np.array([A.n for A in As], dtype=np.int32)
        self.k = np.array([B.n for B in Bs], dtype=np.int32)
        self.a_nnz = np.array([A.nnz for A in As], dtype=np.int64)
        self.b_nnz = np.array([B.nnz for B in Bs], dtype=np.int64)
        self._create(options)

    def _create(self, options):
        self.b = _lib.spg_batch_create(self.stream.cuda_stream, _dtype_code(self.dtype), self.count,
                                       self.m.ctypes.data, self.n.ctypes.data, self.k.ctypes.data,
                                       self.a_nnz.ctypes.data, self.b_nnz.ctypes.data, self.a_rp.data_ptr(),
                                       self.a_ci.data_ptr() if self.a_ci.numel() else 0, self.b_rp.data_ptr(),
                                       self.b_ci.data_ptr() if self.b_ci.numel() else 0)
        for k_, v in options.items():
            _lib.spg_batch_set_option(self.b, k_, int(v))
        self.nnz = None

    def __del__(self):
        b = getattr(self, "b", None)
        if b:
            try:
                _lib.spg_batch_destroy(b)
            except Exception:
                pass
            self.b = None

    def set_option(self, name, value):
        _lib.spg_batch_set_option(self.b, name, int(value))
        self.nnz = None

    def set_mlp(self, w: np.ndarray):
        w = np.ascontiguousarray(w, dtype=np.float32)
        _lib.spg_batch_set_mlp(self.b, w.ctypes.data, int(w.size))
        self.nnz = None

    def plan(self):
        self.stream.wait_stream(torch.cuda.current_stream())
        self.c_row_off = np.zeros(self.count + 1, dtype=np.int64)
        self.c_nnz_off = np.zeros(self.count + 1, dtype=np.int64)
        self.nnz = _lib.spg_batch_plan(self.b, self.c_row_off.ctypes.data, self.c_nnz_off.ctypes.data)
        dev = self.a_rp.device
        with torch.cuda.stream(self.stream):
            self.c_rp = torch.empty(int(self.m.sum()) + 1, dtype=torch.int32, device=dev)
            self.c_col = torch.empty(max(self.nnz, 1), dtype=torch.int32, device=dev)
            self.c_val = torch.empty(max(self.nnz, 1), dtype=self.dtype, device=dev)
        return self.nnz

    def _ptrs(self, a_vals, b_vals):
        a_vals = self.a_v if a_vals is None else a_vals
        b_vals = self.b_v if b_vals is None else b_vals
        return (a_vals.data_ptr() if a_vals.numel() else 0, b_vals.data_ptr() if b_vals.numel() else 0,
                self.c_rp.data_ptr(), self.c_col.data_ptr(), self.c_val.data_ptr(), int(self.c_col.numel()))

    def run(self, numeric_only: bool = False, a_vals=None, b_vals=None):
        if self.nnz is None:
            self.plan()
        cur = torch.cuda.current_stream()
        self.stream.wait_stream(cur)
        _lib.spg_batch_run(self.b, *self._ptrs(a_vals, b_vals), 1 if numeric_only else 0)
        cur.wait_stream(self.stream)

    def tune(self):
        if self.nnz is None:
            self.plan()
        self.stream.wait_stream(torch.cuda.current_stream())
        chosen, best = _lib.spg_batch_tune(self.b, *self._ptrs(None, None))
        self.plan()
        return chosen, best

    def run_queued(self, capacity: int, a_vals=None, b_vals=None, stamps: bool = True):
        """Both phases of every product in one persistent kernel over a device
        work queue (no plan, no host work between products).  Pools: row
        pointers (sum of m_i + 1 entries), columns and values of `capacity`
        entries; ``q_offsets[i]`` is C_i's first pool entry (-1 if it did not
        fit) and ``q_stamps[2i:2i+2]`` the device clock (100 MHz) when C_i's
        first work item started and its last ended."""
        dev = self.a_rp.device
        if getattr(self, "q_cap", None) != capacity:
            with torch.cuda.stream(self.stream):
                self.q_rp = torch.empty(int(self.m.astype(np.int64).sum()) + self.count, dtype=torch.int32,
                                        device=dev)
                self.q_col = torch.empty(max(capacity, 1), dtype=torch.int32, device=dev)
                self.q_val = torch.empty(max(capacity, 1), dtype=self.dtype, device=dev)
                self.q_offsets = torch.empty(max(self.count, 1), dtype=torch.int64, device=dev)
                self.q_stamps = torch.empty(2 * max(self.count, 1), dtype=torch.int64, device=dev)
            self.q_cap = capacity
            self.q_rp_off = np.concatenate([[0], np.cumsum(self.m.astype(np.int64) + 1)])
        a_vals = self.a_v if a_vals is None else a_vals
        b_vals = self.b_v if b_vals is None else b_vals
        cur = torch.cuda.current_stream()
        self.stream.wait_stream(cur)
        _lib.spg_batch_run_queued(self.b, a_vals.data_ptr() if a_vals.numel() else 0,
                                  b_vals.data_ptr() if b_vals.numel() else 0, self.q_rp.data_ptr(),
                                  self.q_col.data_ptr(), self.q_val.data_ptr(), capacity,
                                  self.q_offsets.data_ptr(), self.q_stamps.data_ptr() if stamps else 0)
        cur.wait_stream(self.stream)

    def product_queued(self, i: int):
        """(row_ptr from 0, col_idx, values) of C_i after run_queued, or None if it did not fit."""
        off = int(self.q_offsets[i].item())
        if off < 0:
            return None
        r0 = int(self.q_rp_off[i])
        rp = self.q_rp[r0:r0 + int(self.m[i]) + 1].to(torch.int64) - off
        n = int(rp[-1].item())
        return rp, self.q_col[off:off + n], self.q_val[off:off + n]

    def product(self, i: int):
        """(row_ptr, col_idx, values) of C_i as views/copies on the device."""
        r0, r1 = int(self.c_row_off[i]), int(self.c_row_off[i + 1])
        e0, e1 = int(self.c_nnz_off[i]), int(self.c_nnz_off[i + 1])
        return self.c_rp[r0:r1 + 1] - e0, self.c_col[e0:e1], self.c_val[e0:e1]

    def stats(self) -> dict:
        st = _lib.spg_batch_get_stats(self.b)
        return {name: (list(getattr(st, name)) if hasattr(getattr(st, name), "__len__") else getattr(st, name))
                for name, _ in st._fields_}
