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
