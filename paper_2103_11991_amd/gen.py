"""Seeded synthetic CSR workloads.

This module only *produces inputs*: it holds none of the product's
arithmetic, and both the GPU library's tests and the CPU oracle consume the
same matrices from it.  Every random number is counter based, so a matrix is a
pure function of (generator, sizes, seed):

    u64(seed, stream, i) = mix(key(seed, stream) + (i + 1) * GAMMA)

where ``mix`` is the splitmix64 output function (Steele, Lea and Flood,
"Fast splittable pseudorandom number generators", OOPSLA 2014, with
Vigna's constants) and ``key(seed, stream) = mix(seed * GAMMA ^ mix(stream +
GAMMA))``.  ``i`` is an element index fixed by each generator below, never a
call count, so any sub-range can be regenerated on its own.

The structured matrices are stand-ins for the multigrid and graph inputs the
paper names as SpGEMM's applications (section 2.2): 2D/3D Laplacian and
27-point stencils, piecewise-constant aggregation prolongators, R-MAT
power-law graphs and banded random products for batched runs.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

# stream ids: one per independent quantity a generator draws
S_VALUES = 1
S_RMAT = 2
S_ROWLEN = 3
S_COLS = 4
S_PERM = 5
S_BATCH = 6
S_SWEEP_DIAG = 7
S_SWEEP_OFF = 8


def _mul(a: np.ndarray, b) -> np.ndarray:
    """uint64 product modulo 2^64 (done on the int64 view: numpy's uint64
    multiply takes a slow path, the wrapped int64 product has the same bits)."""
    a = np.ascontiguousarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return (a.view(np.int64) * b.view(np.int64)).view(np.uint64)


def _mix(z: np.ndarray) -> np.ndarray:
    z = np.asarray(z, dtype=np.uint64)
    z = _mul(z ^ (z >> np.uint64(30)), _M1)
    z = _mul(z ^ (z >> np.uint64(27)), _M2)
    return z ^ (z >> np.uint64(31))


def _key(seed: int, stream: int) -> np.uint64:
    with np.errstate(over="ignore"):
        s = _mul(np.asarray([seed], dtype=np.uint64), GAMMA)
        t = _mix(np.asarray([stream], dtype=np.uint64) + GAMMA)
        return _mix(s ^ t)[0]


def u64(seed: int, stream: int, idx) -> np.ndarray:
    """Counter-based 64-bit draws for element indices ``idx``."""
    idx = np.asarray(idx, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return _mix(_key(seed, stream) + _mul(idx + np.uint64(1), GAMMA))


def uniform(seed: int, stream: int, idx) -> np.ndarray:
    """float64 uniform on [0, 1): top 53 bits of the draw."""
    return (u64(seed, stream, idx) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def uniform_f32(seed: int, stream: int, idx) -> np.ndarray:
    """float32 uniform on [0, 1): top 24 bits, so every value is exact in fp32."""
    return ((u64(seed, stream, idx) >> np.uint64(40)).astype(np.float64) * (2.0 ** -24)).astype(np.float32)


def normal(seed: int, stream: int, idx) -> np.ndarray:
    """N(0,1) by Box-Muller from the draws at 2*idx and 2*idx+1."""
    idx = np.asarray(idx, dtype=np.uint64)
    u1 = uniform(seed, stream, idx << np.uint64(1))
    u2 = uniform(seed, stream, (idx << np.uint64(1)) + np.uint64(1))
    return np.sqrt(-2.0 * np.log1p(-u1)) * np.cos(2.0 * np.pi * u2)


@dataclass
class Csr:
    """Compressed sparse row matrix (m x n) with int32 indices."""
    m: int
    n: int
    row_ptr: np.ndarray  # int32[m+1]
    col_idx: np.ndarray  # int32[nnz]
    values: np.ndarray   # float64[nnz] or float32[nnz]

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def dtype(self):
        return self.values.dtype

    def row_lengths(self) -> np.ndarray:
        return np.diff(self.row_ptr.astype(np.int64))

    def with_values(self, values: np.ndarray) -> "Csr":
        assert values.shape == self.col_idx.shape
        return Csr(self.m, self.n, self.row_ptr, self.col_idx, values)

    def astype(self, dt) -> "Csr":
        return Csr(self.m, self.n, self.row_ptr, self.col_idx, self.values.astype(dt))


def csr_from_rows_cols(m: int, n: int, rows: np.ndarray, cols: np.ndarray, values: np.ndarray) -> Csr:
    """Build CSR from entries already grouped by row (rows non-decreasing)."""
    rows = np.asarray(rows, dtype=np.int64)
    counts = np.bincount(rows, minlength=m)
    rp = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(counts, out=rp[1:])
    assert rp[-1] < 2 ** 31
    return Csr(m, n, rp.astype(np.int32), np.asarray(cols, dtype=np.int32), np.asarray(values))


# ----------------------------------------------------------------------------
# structured stencils (lexicographic ordering, x fastest, Dirichlet truncation)
# ----------------------------------------------------------------------------

def _stencil_pattern(dims, offsets):
    """Rows and columns of a truncated stencil; columns ascend within a row."""
    dims = tuple(int(d) for d in dims)
    while len(dims) < 3:
        dims = dims + (1,)
    nx, ny, nz = dims
    offsets = [tuple(o) + (0,) * (3 - len(o)) for o in offsets]
    offsets.sort(key=lambda o: (o[2], o[1], o[0]))  # ascending column order
    N = nx * ny * nz
    idx = np.arange(N, dtype=np.int64)
    x = idx % nx
    y = (idx // nx) % ny
    z = idx // (nx * ny)
    cols = np.empty((N, len(offsets)), dtype=np.int64)
    ok = np.empty((N, len(offsets)), dtype=bool)
    for t, (dx, dy, dz) in enumerate(offsets):
        ok[:, t] = ((x + dx >= 0) & (x + dx < nx) & (y + dy >= 0) & (y + dy < ny)
                    & (z + dz >= 0) & (z + dz < nz))
        cols[:, t] = idx + dx + nx * (dy + ny * dz)
    rows = np.broadcast_to(idx[:, None], cols.shape)[ok]
    is_diag = np.broadcast_to(np.array([o == (0, 0, 0) for o in offsets])[None, :], cols.shape)[ok]
    return N, rows, cols[ok], is_diag


def laplace2d_5pt(nx: int, ny: int | None = None) -> Csr:
    """2D 5-point Laplacian: 4 on the diagonal, -1 to grid neighbours."""
    ny = nx if ny is None else ny
    offs = [(0, 0), (-1, 0), (1, 0), (0, -1), (0, 1)]
    N, rows, cols, diag = _stencil_pattern((nx, ny), offs)
    vals = np.where(diag, 4.0, -1.0)
    return csr_from_rows_cols(N, N, rows, cols, vals)


def laplace3d_7pt(n: int, scale: float = 1.0) -> Csr:
    """3D 7-point Laplacian on n^3: 6 on the diagonal, -1 to face neighbours (times ``scale``)."""
    offs = [(0, 0, 0), (-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]
    N, rows, cols, diag = _stencil_pattern((n, n, n), offs)
    vals = np.where(diag, 6.0, -1.0) * scale
    return csr_from_rows_cols(N, N, rows, cols, vals)


def stencil27(n: int, seed: int = 2) -> Csr:
    """3D 27-point stencil on n^3: off-diagonal values uniform in [-1, 1], diagonal 27.

    Off-diagonal entry e (its index in CSR order) takes 2*u(seed, S_VALUES, e) - 1.
    """
    offs = [(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
    N, rows, cols, diag = _stencil_pattern((n, n, n), offs)
    e = np.arange(cols.size, dtype=np.uint64)
    vals = 2.0 * uniform(seed, S_VALUES, e) - 1.0
    vals[diag] = 27.0
    return csr_from_rows_cols(N, N, rows, cols, vals)


def identity(n: int, dtype=np.float64) -> Csr:
    i = np.arange(n, dtype=np.int64)
    return csr_from_rows_cols(n, n, i, i, np.ones(n, dtype=dtype))


# ----------------------------------------------------------------------------
# multigrid aggregation (Galerkin products R*A*P)
# ----------------------------------------------------------------------------

def aggregation_P(n: int) -> Csr:
    """Piecewise-constant prolongator from n^3 onto (n/2)^3 aggregates of 2x2x2 nodes."""
    assert n % 2 == 0
    N = n ** 3
    h = n // 2
    i = np.arange(N, dtype=np.int64)
    x, y, z = i % n, (i // n) % n, i // (n * n)
    agg = (x // 2) + h * (y // 2) + h * h * (z // 2)
    return csr_from_rows_cols(N, h ** 3, i, agg, np.ones(N))


def transpose(A: Csr) -> Csr:
    """Explicit transpose with sorted rows (used to materialise R = P^T)."""
    rows = np.repeat(np.arange(A.m, dtype=np.int64), A.row_lengths())
    order = np.lexsort((rows, A.col_idx.astype(np.int64)))
    return csr_from_rows_cols(A.n, A.m, A.col_idx[order].astype(np.int64), rows[order], A.values[order])


def galerkin_hierarchy(n0: int = 128, levels: int = 5):
    """Fine grid sizes and (P, R) pairs for ``levels`` Galerkin products starting at n0^3."""
    out = []
    n = n0
    for _ in range(levels):
        P = aggregation_P(n)
        out.append((n, P, transpose(P)))
        n //= 2
    return out


def sweep_values(A: Csr, t: int) -> np.ndarray:
    """Changed values for numeric sweep t of a symmetric Laplacian pattern.

    Off-diagonal (i, j): -(1 + 0.5 * s_t(min(i,j), max(i,j))), diagonal 6 + 0.5 * s_t(i),
    so the matrix stays symmetric.
    """
    rows = np.repeat(np.arange(A.m, dtype=np.int64), A.row_lengths())
    cols = A.col_idx.astype(np.int64)
    lo = np.minimum(rows, cols).astype(np.uint64)
    hi = np.maximum(rows, cols).astype(np.uint64)
    with np.errstate(over="ignore"):
        pair = _mul(lo, np.uint64(A.n)) + hi
    off = -(1.0 + 0.5 * uniform(t, S_SWEEP_OFF, pair))
    dg = 6.0 + 0.5 * uniform(t, S_SWEEP_DIAG, rows.astype(np.uint64))
    return np.where(rows == cols, dg, off)


# ----------------------------------------------------------------------------
# R-MAT power-law graphs
# ----------------------------------------------------------------------------

def rmat(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         seed: int = 1, dtype=np.float32) -> Csr:
    """R-MAT graph on 2^scale vertices with edge_factor * 2^scale edge draws.

    Per edge e and level l (bit scale-1-l, most significant first) the draw
    u = uniform(seed, S_RMAT, e*scale + l) picks a quadrant: u < a top-left,
    u < a+b top-right (column bit), u < a+b+c bottom-left (row bit), else
    bottom-right (both bits).  No noise and no vertex permutation; self loops
    are kept; duplicate edges are merged into one entry.  Values are uniform
    on [0, 1), drawn after merging, one per entry in CSR order.
    """
    V = 1 << scale
    E = edge_factor * V
    r = np.zeros(E, dtype=np.int64)
    cc = np.zeros(E, dtype=np.int64)
    e = np.arange(E, dtype=np.uint64)
    for lvl in range(scale):
        u = uniform(seed, S_RMAT, _mul(e, np.uint64(scale)) + np.uint64(lvl))
        bit = np.int64(1 << (scale - 1 - lvl))
        colbit = ((u >= a) & (u < a + b)) | (u >= a + b + c)
        rowbit = u >= a + b
        r += rowbit * bit
        cc += colbit * bit
    key = np.unique(r * V + cc)
    rows = key // V
    cols = key % V
    if np.dtype(dtype) == np.float32:
        vals = uniform_f32(seed, S_VALUES, np.arange(key.size, dtype=np.uint64))
    else:
        vals = uniform(seed, S_VALUES, np.arange(key.size, dtype=np.uint64))
    return csr_from_rows_cols(V, V, rows, cols, vals.astype(dtype))


# ----------------------------------------------------------------------------
# random matrices for tests, and banded products for batched runs
# ----------------------------------------------------------------------------

def random_csr(m: int, n: int, min_len: int = 0, max_len: int = 8, seed: int = 0,
               sorted_rows: bool = True, duplicates: bool = False, dtype=np.float64,
               value_kind: str = "normal", empty_frac: float = 0.0) -> Csr:
    """Random CSR: row lengths uniform on [min_len, max_len], columns uniform in [0, n).

    ``duplicates`` keeps repeated columns inside a row; ``sorted_rows=False``
    permutes each row's entries.  ``value_kind`` is ``normal``, ``uniform``
    (on [0,1)), ``int`` (small integers, exact in any float type) or ``ones``.
    """
    rows_i = np.arange(m, dtype=np.uint64)
    span = max_len - min_len + 1
    lens = min_len + (u64(seed, S_ROWLEN, rows_i) % np.uint64(span)).astype(np.int64)
    if empty_frac > 0:
        lens[uniform(seed, S_ROWLEN + 100, rows_i) < empty_frac] = 0
    if n == 0:
        lens[:] = 0
    tot = int(lens.sum())
    rows = np.repeat(np.arange(m, dtype=np.int64), lens)
    cols = (u64(seed, S_COLS, np.arange(tot, dtype=np.uint64)) % np.uint64(max(n, 1))).astype(np.int64)
    key = rows * max(n, 1) + cols
    if not duplicates:
        key = np.unique(key)
    else:
        key = np.sort(key)
    rows = key // max(n, 1)
    cols = key % max(n, 1)
    if not sorted_rows and key.size:
        perm_key = u64(seed, S_PERM, np.arange(key.size, dtype=np.uint64))
        order = np.lexsort((perm_key, rows))
        rows, cols = rows[order], cols[order]
    idx = np.arange(key.size, dtype=np.uint64)
    if value_kind == "normal":
        vals = normal(seed, S_VALUES, idx)
    elif value_kind == "uniform":
        vals = uniform(seed, S_VALUES, idx)
    elif value_kind == "int":
        vals = (u64(seed, S_VALUES, idx) % np.uint64(7)).astype(np.float64) - 3.0
    elif value_kind == "ones":
        vals = np.ones(key.size)
    else:
        raise ValueError(value_kind)
    return csr_from_rows_cols(m, n, rows, cols, vals.astype(dtype))


_GEN_LIB = None


def build_native(force: bool = True) -> str:
    """Compiles gen_banded.c (the banded-matrix generator) into libspggen.so."""
    import os
    import subprocess
    here = os.path.dirname(os.path.abspath(__file__))
    out = os.path.join(here, "libspggen.so")
    if force or not os.path.exists(out):
        tmp = out + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", os.path.join(here, "gen_banded.c"),
                               "-o", tmp, "-lm"])
        os.replace(tmp, out)
    return out


def _native():
    global _GEN_LIB
    if _GEN_LIB is None:
        import ctypes
        L = ctypes.CDLL(build_native(force=False))
        p, i32, u64_ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint64
        L.gen_banded_nnz.argtypes = [i32, p, p, u64_, p, ctypes.c_int, ctypes.c_int, p]
        L.gen_banded_nnz.restype = None
        L.gen_banded_fill.argtypes = [i32, p, p, u64_, p, ctypes.c_int, ctypes.c_int, p, p, p]
        L.gen_banded_fill.restype = ctypes.c_int
        _GEN_LIB = L
    return _GEN_LIB


def _banded_pool(n, bw, seed: int, streams, lo: int = 3, hi: int = 30):
    """Rows of several square banded random matrices at once (see gen_banded.c
    for the exact draws): matrix t has n[t] rows, bandwidth bw[t], counter
    stream streams[t]; row r has k_r ~ U{lo..hi} (capped at its window)
    distinct columns uniform in [r-bw, r+bw] cut to [0, n), values N(0,1).
    Returns (row_ptr pool with one n[t]+1 block per matrix, columns, values,
    nnz per matrix)."""
    n = np.ascontiguousarray(n, dtype=np.int64)
    bw = np.ascontiguousarray(bw, dtype=np.int64)
    st = np.ascontiguousarray(streams, dtype=np.uint64)
    P = n.size
    L = _native()
    nnz = np.zeros(P, dtype=np.int64)
    L.gen_banded_nnz(P, n.ctypes.data, bw.ctypes.data, seed, st.ctypes.data, lo, hi, nnz.ctypes.data)
    tot = int(nnz.sum())
    rp = np.empty(int(n.sum()) + P, dtype=np.int32)
    cols = np.empty(tot, dtype=np.int32)
    vals = np.empty(tot, dtype=np.float64)
    rc = L.gen_banded_fill(P, n.ctypes.data, bw.ctypes.data, seed, st.ctypes.data, lo, hi, rp.ctypes.data,
                           cols.ctypes.data, vals.ctypes.data)
    if rc != 0:
        raise ValueError("band window wider than 192 columns")
    return rp, cols, vals, nnz


def banded_random(n: int, bw: int, seed: int, stream_base: int, lo: int = 3, hi: int = 30) -> Csr:
    """Square banded random matrix: row r has k_r ~ U{lo..hi} (capped at the window
    width) distinct columns uniform in [r-bw, r+bw] cut to [0, n), values N(0,1)."""
    rp, cols, vals, _ = _banded_pool([n], [bw], seed, [stream_base], lo, hi)
    return Csr(n, n, rp, cols, vals)


def batch_sizes(count: int, seed: int = 12345, lo: int = 200, hi: int = 50000):
    """Per-product (n, bwA, bwB): n = round(exp(U(ln lo, ln hi))), bandwidths U{5..64}."""
    i = np.arange(count, dtype=np.uint64)
    u = uniform(seed, S_BATCH, _mul(i, np.uint64(3)))
    n = np.rint(np.exp(np.log(lo) + u * (np.log(hi) - np.log(lo)))).astype(np.int64)
    bwa = 5 + (u64(seed, S_BATCH, _mul(i, np.uint64(3)) + np.uint64(1)) % np.uint64(60)).astype(np.int64)
    bwb = 5 + (u64(seed, S_BATCH, _mul(i, np.uint64(3)) + np.uint64(2)) % np.uint64(60)).astype(np.int64)
    return n, bwa, bwb


def banded_batch_pools(count: int, seed: int = 12345, lo: int = 200, hi: int = 50000):
    """The ``count`` banded products as pooled arrays (the batch API's layout):
    dict with n (rows = columns of every A_i, B_i), per-product nnz and
    (row_ptr, col, val) pools for A and for B.  A_i uses stream 2i, B_i 2i+1."""
    n, bwa, bwb = batch_sizes(count, seed, lo, hi)
    i = np.arange(count, dtype=np.uint64)
    a = _banded_pool(n, bwa, seed, 2 * i)
    b = _banded_pool(n, bwb, seed, 2 * i + np.uint64(1))
    return {"n": n, "a_rp": a[0], "a_ci": a[1], "a_v": a[2], "a_nnz": a[3],
            "b_rp": b[0], "b_ci": b[1], "b_v": b[2], "b_nnz": b[3]}


def pools_to_pairs(pools):
    """Splits pooled batch arrays into a list of (A_i, B_i) CSR pairs."""
    n = pools["n"]
    out = []
    ra = eb = ea = 0
    for t in range(n.size):
        m = int(n[t])
        A = Csr(m, m, pools["a_rp"][ra: ra + m + 1], pools["a_ci"][ea: ea + pools["a_nnz"][t]],
                pools["a_v"][ea: ea + pools["a_nnz"][t]])
        B = Csr(m, m, pools["b_rp"][ra: ra + m + 1], pools["b_ci"][eb: eb + pools["b_nnz"][t]],
                pools["b_v"][eb: eb + pools["b_nnz"][t]])
        out.append((A, B))
        ra += m + 1
        ea += int(pools["a_nnz"][t])
        eb += int(pools["b_nnz"][t])
    return out


def banded_batch(count: int, seed: int = 12345, lo: int = 200, hi: int = 50000):
    """``count`` independent products (A_i, B_i), each banded random, FP64."""
    return pools_to_pairs(banded_batch_pools(count, seed, lo, hi))


def products_per_row(A: Csr, B: Csr) -> np.ndarray:
    """Number of scalar products each row of A*B takes (sum of the referenced B row lengths).

    This is a workload size (it prices GFLOP/s), not part of the product itself.
    """
    bl = B.row_lengths()
    per = bl[A.col_idx.astype(np.int64)] if A.nnz else np.zeros(0, dtype=np.int64)
    cs = np.zeros(A.nnz + 1, dtype=np.int64)
    np.cumsum(per, out=cs[1:])
    rp = A.row_ptr.astype(np.int64)
    return cs[rp[1:]] - cs[rp[:-1]]
