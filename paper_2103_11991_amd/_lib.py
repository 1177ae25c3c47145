"""ctypes binding of libspg.so: one Python function per C entry point, same names.

Argument marshalling only: pointers are passed as integers (device addresses
from ``tensor.data_ptr()``, streams from ``torch.cuda.Stream.cuda_stream``),
every failing status raises :class:`SpgError` with the library's message.
There is no fallback: if the library was not built, loading raises.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libspg.so")

SPG_F32, SPG_F64 = 0, 1
OPT = {
    "binning": 0, "timing": 1, "force_class": 2, "work_per_lane": 3, "mlp_margin_milli": 4,
    "hash_max_blocks": 6, "lds_limit": 7, "keep_features": 8, "list_limit_mb": 9,
    "merge_classes": 10, "tiled_global": 11, "method": 12,
}
NTIER, NCLASS = 10, 30
STATUS = ["SPG_OK", "SPG_ERR_ARG", "SPG_ERR_SHAPE", "SPG_ERR_STATE", "SPG_ERR_INDEX", "SPG_ERR_OVERFLOW",
          "SPG_ERR_ALLOC", "SPG_ERR_HIP", "SPG_ERR_UNSUPPORTED"]
EXPORTS = ["spg_status_string", "spg_last_error", "spg_create", "spg_destroy", "spg_set_stream",
           "spg_set_matrices", "spg_symbolic", "spg_numeric", "spg_numeric_jacobi", "spg_set_option", "spg_set_mlp", "spg_get_stats",
           "spg_export_rows", "spg_mlp_forward", "spg_mlp_backward", "spg_mlp_backward_noalloc", "spg_mlp_train",
           "spg_batch_create", "spg_batch_destroy", "spg_batch_last_error", "spg_batch_set_option",
           "spg_batch_set_mlp", "spg_batch_plan", "spg_batch_run", "spg_batch_tune", "spg_batch_get_stats",
           "spg_batch_run_queued",
           "spg_add_create", "spg_add_destroy", "spg_add_last_error", "spg_add_symbolic", "spg_add_numeric"]


class SpgError(RuntimeError):
    def __init__(self, status: int, msg: str):
        self.status = status
        self.status_name = STATUS[status] if 0 <= status < len(STATUS) else str(status)
        super().__init__(f"{self.status_name}: {msg}")


class spg_stats(ctypes.Structure):
    _fields_ = [
        ("size", ctypes.c_int32), ("m", ctypes.c_int32), ("n", ctypes.c_int32), ("k", ctypes.c_int32),
        ("products", ctypes.c_int64), ("nnz_c", ctypes.c_int64),
        ("sym_rows", ctypes.c_int32 * NCLASS), ("num_rows", ctypes.c_int32 * NCLASS),
        ("num_a_nnz", ctypes.c_int64 * NCLASS), ("num_c_nnz", ctypes.c_int64 * NCLASS),
        ("num_products", ctypes.c_int64 * NCLASS),
        ("empty_rows", ctypes.c_int32), ("retried_rows", ctypes.c_int32), ("mispredicted_rows", ctypes.c_int32),
        ("binning", ctypes.c_int32), ("sym_ms", ctypes.c_float), ("num_ms", ctypes.c_float),
        ("sym_class_ms", ctypes.c_float * NCLASS), ("num_class_ms", ctypes.c_float * NCLASS),
        ("analysis_ms", ctypes.c_float), ("scan_ms", ctypes.c_float), ("mlp_ms", ctypes.c_float),
        ("list_pairs", ctypes.c_int64),
        ("num_class_ms_total", ctypes.c_float * NCLASS), ("num_class_launches", ctypes.c_int32 * NCLASS),
        ("num_tiles", ctypes.c_int32), ("tile_fallback_rows", ctypes.c_int32),
        ("sym_waits", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]


_lib = None


def load() -> ctypes.CDLL:
    """Loads libspg.so from the package directory (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it first (python -m paper_2103_11991_amd._build)")
    L = ctypes.CDLL(LIB_PATH)
    p, i32, i64, f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float
    sig = {
        "spg_status_string": ([ctypes.c_int], ctypes.c_char_p),
        "spg_last_error": ([p], ctypes.c_char_p),
        "spg_create": ([ctypes.POINTER(p), p], ctypes.c_int),
        "spg_destroy": ([p], ctypes.c_int),
        "spg_set_stream": ([p, p], ctypes.c_int),
        "spg_set_matrices": ([p, ctypes.c_int, i32, i32, i32, p, p, i64, p, p, i64], ctypes.c_int),
        "spg_symbolic": ([p, p, ctypes.POINTER(i64)], ctypes.c_int),
        "spg_numeric": ([p, p, p, p, p], ctypes.c_int),
        "spg_numeric_jacobi": ([p, ctypes.c_double, p, p, p, p, p], ctypes.c_int),
        "spg_set_option": ([p, i32, i64], ctypes.c_int),
        "spg_set_mlp": ([p, p, i32], ctypes.c_int),
        "spg_get_stats": ([p, ctypes.POINTER(spg_stats), i32], ctypes.c_int),
        "spg_export_rows": ([p, p, p, p], ctypes.c_int),
        "spg_mlp_forward": ([p, p, p, i32, p, p], ctypes.c_int),
        "spg_mlp_backward": ([p, p, p, p, p, i32, p], ctypes.c_int),
        "spg_mlp_backward_noalloc": ([p, p, p, p, p, i32, p], ctypes.c_int),
        "spg_mlp_train": ([p, p, p, i32, i32, i32, f32, f32, p, p], ctypes.c_int),
        "spg_batch_create": ([ctypes.POINTER(p), p, ctypes.c_int, i32, p, p, p, p, p, p, p, p, p], ctypes.c_int),
        "spg_batch_destroy": ([p], ctypes.c_int),
        "spg_batch_last_error": ([p], ctypes.c_char_p),
        "spg_batch_set_option": ([p, i32, i64], ctypes.c_int),
        "spg_batch_set_mlp": ([p, p, i32], ctypes.c_int),
        "spg_batch_plan": ([p, ctypes.POINTER(i64), p, p], ctypes.c_int),
        "spg_batch_run": ([p, p, p, p, p, p, i64, i32], ctypes.c_int),
        "spg_batch_tune": ([p, p, p, p, p, p, i64, p, p], ctypes.c_int),
        "spg_batch_get_stats": ([p, ctypes.POINTER(spg_stats), i32], ctypes.c_int),
        "spg_batch_run_queued": ([p, p, p, p, p, p, i64, p, p], ctypes.c_int),
        "spg_add_create": ([ctypes.POINTER(p), p], ctypes.c_int),
        "spg_add_destroy": ([p], ctypes.c_int),
        "spg_add_last_error": ([p], ctypes.c_char_p),
        "spg_add_symbolic": ([p, i32, i32, p, p, i64, p, p, i64, p, ctypes.POINTER(i64)], ctypes.c_int),
        "spg_add_numeric": ([p, ctypes.c_int, ctypes.c_double, p, ctypes.c_double, p, p, p], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def _check(rc: int, h=None):
    if rc != 0:
        msg = load().spg_last_error(h).decode() if h else ""
        raise SpgError(rc, msg or STATUS[rc] if 0 <= rc < len(STATUS) else str(rc))


def spg_status_string(s: int) -> str:
    return load().spg_status_string(s).decode()


def spg_create(stream: int = 0) -> int:
    h = ctypes.c_void_p()
    _check(load().spg_create(ctypes.byref(h), stream or None))
    return h.value


def spg_destroy(h: int) -> None:
    _check(load().spg_destroy(h))


def spg_set_stream(h: int, stream: int) -> None:
    _check(load().spg_set_stream(h, stream or None), h)


def spg_set_matrices(h: int, dtype: int, m: int, n: int, k: int, a_row_ptr: int, a_col_idx: int, a_nnz: int,
                     b_row_ptr: int, b_col_idx: int, b_nnz: int) -> None:
    _check(load().spg_set_matrices(h, dtype, m, n, k, a_row_ptr or None, a_col_idx or None, a_nnz,
                                   b_row_ptr or None, b_col_idx or None, b_nnz), h)


def spg_symbolic(h: int, c_row_ptr: int) -> int:
    nnz = ctypes.c_int64(-1)
    _check(load().spg_symbolic(h, c_row_ptr or None, ctypes.byref(nnz)), h)
    return nnz.value


def spg_numeric(h: int, a_vals: int, b_vals: int, c_col_idx: int, c_vals: int) -> None:
    _check(load().spg_numeric(h, a_vals or None, b_vals or None, c_col_idx or None, c_vals or None), h)


def spg_numeric_jacobi(h: int, omega: float, dinv: int, a_vals: int, b_vals: int, c_col_idx: int,
                       c_vals: int) -> None:
    _check(load().spg_numeric_jacobi(h, float(omega), dinv or None, a_vals or None, b_vals or None,
                                     c_col_idx or None, c_vals or None), h)


def spg_set_option(h: int, opt, val: int) -> None:
    opt = OPT[opt] if isinstance(opt, str) else int(opt)
    _check(load().spg_set_option(h, opt, int(val)), h)


def spg_set_mlp(h: int, w_host_ptr: int, nw: int) -> None:
    _check(load().spg_set_mlp(h, w_host_ptr, nw), h)


def spg_get_stats(h: int) -> spg_stats:
    st = spg_stats()
    _check(load().spg_get_stats(h, ctypes.byref(st), ctypes.sizeof(spg_stats)), h)
    return st


def spg_export_rows(h: int, x: int, y: int, row_nnz: int = 0) -> None:
    _check(load().spg_export_rows(h, x or None, y or None, row_nnz or None), h)


def spg_mlp_forward(stream: int, w: int, x: int, rows: int, y: int, act: int = 0) -> None:
    _check(load().spg_mlp_forward(stream or None, w, x, rows, y, act or None))


def spg_mlp_backward(stream: int, w: int, x: int, act: int, dy: int, rows: int, dw: int) -> None:
    _check(load().spg_mlp_backward(stream or None, w, x, act, dy, rows, dw))


def spg_mlp_backward_noalloc(stream: int, w: int, x: int, act: int, dy: int, rows: int, dw: int) -> None:
    _check(load().spg_mlp_backward_noalloc(stream or None, w, x, act, dy, rows, dw))


def spg_mlp_train(stream: int, x: int, y: int, rows: int, epochs: int, batch: int, lr: float, quantile: float,
                  w_inout: int, loss_out: int = 0) -> None:
    _check(load().spg_mlp_train(stream or None, x, y, rows, epochs, batch, lr, quantile, w_inout, loss_out or None))


def _bcheck(rc: int, b=None):
    if rc != 0:
        msg = load().spg_batch_last_error(b).decode() if b else ""
        raise SpgError(rc, msg or (STATUS[rc] if 0 <= rc < len(STATUS) else str(rc)))


def spg_batch_create(stream: int, dtype: int, count: int, m_ptr: int, n_ptr: int, k_ptr: int, a_nnz_ptr: int,
                     b_nnz_ptr: int, a_row_ptr_pool: int, a_col_pool: int, b_row_ptr_pool: int,
                     b_col_pool: int) -> int:
    """Host pointers m_ptr..b_nnz_ptr (int32/int64 arrays), device pools."""
    b = ctypes.c_void_p()
    _bcheck(load().spg_batch_create(ctypes.byref(b), stream or None, dtype, count, m_ptr, n_ptr, k_ptr, a_nnz_ptr,
                                    b_nnz_ptr, a_row_ptr_pool or None, a_col_pool or None, b_row_ptr_pool or None,
                                    b_col_pool or None))
    return b.value


def spg_batch_destroy(b: int) -> None:
    _bcheck(load().spg_batch_destroy(b))


def spg_batch_set_option(b: int, opt, val: int) -> None:
    opt = OPT[opt] if isinstance(opt, str) else int(opt)
    _bcheck(load().spg_batch_set_option(b, opt, int(val)), b)


def spg_batch_set_mlp(b: int, w_host_ptr: int, nw: int) -> None:
    _bcheck(load().spg_batch_set_mlp(b, w_host_ptr, nw), b)


def spg_batch_plan(b: int, c_row_off_ptr: int = 0, c_nnz_off_ptr: int = 0) -> int:
    nnz = ctypes.c_int64(-1)
    _bcheck(load().spg_batch_plan(b, ctypes.byref(nnz), c_row_off_ptr or None, c_nnz_off_ptr or None), b)
    return nnz.value


def spg_batch_run(b: int, a_val_pool: int, b_val_pool: int, c_row_ptr: int, c_col: int, c_val: int,
                  capacity: int, numeric_only: int = 0) -> None:
    _bcheck(load().spg_batch_run(b, a_val_pool or None, b_val_pool or None, c_row_ptr, c_col or None, c_val or None,
                                 capacity, numeric_only), b)


def spg_batch_tune(b: int, a_val_pool: int, b_val_pool: int, c_row_ptr: int, c_col: int, c_val: int,
                   capacity: int):
    chosen = (ctypes.c_int32 * 3)()
    best = ctypes.c_float(0)
    _bcheck(load().spg_batch_tune(b, a_val_pool or None, b_val_pool or None, c_row_ptr, c_col or None, c_val or None,
                                  capacity, chosen, ctypes.byref(best)), b)
    return list(chosen), best.value


def spg_batch_run_queued(b: int, a_val_pool: int, b_val_pool: int, c_row_ptr: int, c_col: int, c_val: int,
                         capacity: int, c_offsets: int, stamps: int = 0) -> None:
    _bcheck(load().spg_batch_run_queued(b, a_val_pool or None, b_val_pool or None, c_row_ptr or None, c_col or None,
                                        c_val or None, capacity, c_offsets or None, stamps or None), b)


def spg_batch_get_stats(b: int) -> spg_stats:
    st = spg_stats()
    _bcheck(load().spg_batch_get_stats(b, ctypes.byref(st), ctypes.sizeof(spg_stats)), b)
    return st


def _acheck(rc: int, h=None):
    if rc != 0:
        msg = load().spg_add_last_error(h).decode() if h else ""
        raise SpgError(rc, msg or (STATUS[rc] if 0 <= rc < len(STATUS) else str(rc)))


def spg_add_create(stream: int = 0) -> int:
    h = ctypes.c_void_p()
    _acheck(load().spg_add_create(ctypes.byref(h), stream or None))
    return h.value


def spg_add_destroy(h: int) -> None:
    _acheck(load().spg_add_destroy(h))


def spg_add_last_error(h: int) -> str:
    return load().spg_add_last_error(h).decode()


def spg_add_symbolic(h: int, m: int, n: int, a_row_ptr: int, a_col_idx: int, a_nnz: int, b_row_ptr: int,
                     b_col_idx: int, b_nnz: int, c_row_ptr: int) -> int:
    nnz = ctypes.c_int64(-1)
    _acheck(load().spg_add_symbolic(h, m, n, a_row_ptr or None, a_col_idx or None, a_nnz, b_row_ptr or None,
                                    b_col_idx or None, b_nnz, c_row_ptr or None, ctypes.byref(nnz)), h)
    return nnz.value


def spg_add_numeric(h: int, dtype: int, alpha: float, a_vals: int, beta: float, b_vals: int, c_col_idx: int,
                    c_vals: int) -> None:
    _acheck(load().spg_add_numeric(h, dtype, float(alpha), a_vals or None, float(beta), b_vals or None,
                                   c_col_idx or None, c_vals or None), h)
