"""Helpers shared by the GPU tests: run the HIP path through the C ABI and
compare its output with the oracle row by row."""
import numpy as np

import oracle

TOL = {np.dtype(np.float64): 1e-12, np.dtype(np.float32): 1e-5}


def run_gpu(A, B, values=None, repeat=1, **opts):
    """C = A*B on the GPU; returns host (row_ptr int64, cols, vals, op)."""
    import torch
    from paper_2103_11991_amd.spgemm import DeviceCsr, SpGEMM
    dA = DeviceCsr.from_host(A)
    dB = dA if B is A else DeviceCsr.from_host(B)
    op = SpGEMM(dA, dB, **opts)
    rp, nnz = op.symbolic()
    col, val = op.numeric()
    torch.cuda.synchronize()
    return rp.cpu().numpy().astype(np.int64), col.cpu().numpy(), val.cpu().numpy(), op


def compare(A, B, rp, cols, vals, rows=None, exact=False):
    """Structure bit-exact and values within the componentwise tolerance.

    ``rows``: None for all rows, else a list of (r0, r1) row ranges compared
    against the oracle's rows of the same range."""
    dt = np.dtype(A.values.dtype)
    tol = TOL[dt]
    ranges = [(0, A.m)] if rows is None else rows
    for r0, r1 in ranges:
        orp, ocol, oval, oabs = oracle.spgemm(A, B, r0, r1)
        g0, g1 = int(rp[r0]), int(rp[r1])
        np.testing.assert_array_equal(rp[r0:r1 + 1] - rp[r0], orp, err_msg=f"row_ptr rows {r0}:{r1}")
        np.testing.assert_array_equal(cols[g0:g1], ocol, err_msg=f"col_idx rows {r0}:{r1}")
        v = vals[g0:g1].astype(np.float64)
        if exact:
            np.testing.assert_array_equal(v, oval, err_msg=f"values rows {r0}:{r1}")
        else:
            err = np.abs(v - oval)
            bad = err > tol * oabs
            if bad.any():
                i = int(np.argmax(bad))
                raise AssertionError(f"values rows {r0}:{r1}: {int(bad.sum())} entries beyond {tol} x |A||B|; "
                                     f"first at {i}: gpu {v[i]!r} oracle {oval[i]!r} scale {oabs[i]!r}")


def compare_all_rows(A, B, rp, col, val, chunk_entries=1 << 25, exact=False):
    """Every row of C = A*B against the oracle, in row chunks of about
    ``chunk_entries`` entries of C (rows of one chunk come from one oracle
    call; device slices are copied to the host one chunk at a time, so a C of
    billions of entries is never held twice).  ``rp``: host int64 row pointer;
    ``col``, ``val``: device tensors.  Structure bit-exact, values within the
    componentwise tolerance (or exactly equal).  Returns the largest plain
    relative error over entries whose oracle value is nonzero."""
    dt = np.dtype(A.values.dtype)
    tol = TOL[dt]
    m = A.m
    worst = 0.0
    r0 = 0
    while r0 < m:
        # the rows whose entries fit the chunk (at least one row)
        r1 = int(np.searchsorted(rp, rp[r0] + chunk_entries, side="right")) - 1
        r1 = min(max(r1, r0 + 1), m)
        orp, ocol, oval, oabs = oracle.spgemm(A, B, r0, r1)
        g0, g1 = int(rp[r0]), int(rp[r1])
        np.testing.assert_array_equal(rp[r0:r1 + 1] - rp[r0], orp, err_msg=f"row_ptr rows {r0}:{r1}")
        c = col[g0:g1].cpu().numpy()
        if not np.array_equal(c, ocol):
            i = int(np.argmax(c != ocol))
            raise AssertionError(f"col_idx rows {r0}:{r1}: first difference at entry {g0 + i}: "
                                 f"gpu {int(c[i])} oracle {int(ocol[i])}")
        v = val[g0:g1].cpu().numpy().astype(np.float64)
        if exact:
            np.testing.assert_array_equal(v, oval, err_msg=f"values rows {r0}:{r1}")
        else:
            err = np.abs(v - oval)
            bad = err > tol * oabs
            if bad.any():
                i = int(np.argmax(bad))
                raise AssertionError(f"values rows {r0}:{r1}: {int(bad.sum())} entries beyond {tol} x |A||B|; "
                                     f"first at entry {g0 + i}: gpu {v[i]!r} oracle {oval[i]!r} scale {oabs[i]!r}")
            nz = oval != 0
            if nz.any():
                worst = max(worst, float((err[nz] / np.abs(oval[nz])).max()))
        r0 = r1
    return worst
