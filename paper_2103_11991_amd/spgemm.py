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


def spgemm(A: DeviceCsr, B: DeviceCsr, **options) -> DeviceCsr:
    """One-shot C = A*B (symbolic, then numeric) on the current stream."""
    op = SpGEMM(A, B, **options)
    rp, nnz = op.symbolic()
    col, val = op.numeric()
    return DeviceCsr(A.m, B.n, rp, col, val)
