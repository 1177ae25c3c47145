"""The Jacobi-fused numeric phase, C = (I - omega D^-1 A) B on the plain
symbolic result, against the oracle's composition of SpGEMM, row scaling and
sparse addition: structure bit-exact, values within the componentwise
tolerance, on every accumulator class, the tiled and segment global paths,
both dtypes, and the smoothed-aggregation prolongator of a 3D Laplacian."""
import numpy as np
import pytest
import torch

import oracle
from paper_2103_11991_amd import gen
from paper_2103_11991_amd._lib import SpgError
from paper_2103_11991_amd.spgemm import DeviceCsr, SpGEMM
from gpu_util import TOL

pytestmark = pytest.mark.gpu


def setup_module(module):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def with_diagonal(m, lo, hi, seed, dtype=np.float64, empty_diag_rows=()):
    """A random m x m matrix storing every row's diagonal entry (value 4..6)
    except in the rows listed."""
    A = gen.random_csr(m, m, lo, hi, seed=seed, dtype=np.float64)
    rows = np.repeat(np.arange(m), A.row_lengths())
    keep = A.col_idx.astype(np.int64) != rows  # drop any random diagonal entry
    rows, cols, vals = rows[keep], A.col_idx[keep].astype(np.int64), A.values[keep]
    d = np.setdiff1d(np.arange(m), np.asarray(empty_diag_rows, dtype=np.int64))
    rows = np.concatenate([rows, d])
    cols = np.concatenate([cols, d])
    vals = np.concatenate([vals, 4.0 + d % 3])
    order = np.lexsort((cols, rows))
    return gen.csr_from_rows_cols(m, m, rows[order], cols[order], vals[order].astype(dtype))


def diag_inv(A):
    rows = np.repeat(np.arange(A.m), A.row_lengths())
    d = np.zeros(A.m)
    sel = A.col_idx.astype(np.int64) == rows
    np.add.at(d, rows[sel], A.values[sel].astype(np.float64))
    return (1.0 / d).astype(A.values.dtype)


def run_jacobi(A, B, omega, dinv, **opts):
    dA, dB = DeviceCsr.from_host(A), DeviceCsr.from_host(B)
    op = SpGEMM(dA, dB, **opts)
    rp, nnz = op.symbolic()
    col, val = op.numeric_jacobi(omega, torch.from_numpy(dinv).cuda())
    torch.cuda.synchronize()
    return rp.cpu().numpy().astype(np.int64), col.cpu().numpy(), val.cpu().numpy(), op


def check(A, B, omega, dinv, rp, col, val, exact=False):
    orp, ocol, oval, oabs = oracle.jacobi_spgemm(A, B, omega, dinv.astype(np.float64))
    np.testing.assert_array_equal(rp, orp)
    np.testing.assert_array_equal(col, ocol)
    v = val.astype(np.float64)
    if exact:
        np.testing.assert_array_equal(v, oval)
        return
    tol = TOL[np.dtype(A.values.dtype)]
    bad = np.abs(v - oval) > tol * oabs
    assert not bad.any(), (int(bad.sum()), v[bad][:4], oval[bad][:4])


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("seed", range(3))
def test_random_jacobi(dtype, seed):
    A = with_diagonal(700, 0, 30, seed, dtype)
    B = gen.random_csr(700, 500, 0, 25, seed=seed + 10, dtype=dtype, empty_frac=0.1)
    dinv = diag_inv(A)
    rp, col, val, op = run_jacobi(A, B, 2.0 / 3.0, dinv)
    check(A, B, 2.0 / 3.0, dinv, rp, col, val)


@pytest.mark.parametrize("cls", [c for c in range(29) if c % 10 != 9] + [9])
def test_jacobi_on_every_accumulator_class(cls):
    A = with_diagonal(160, 5, 60, 20 + cls)
    B = gen.random_csr(160, 3000, 0, 40, seed=21 + cls)
    dinv = diag_inv(A)
    rp, col, val, op = run_jacobi(A, B, 0.75, dinv, force_class=cls)
    check(A, B, 0.75, dinv, rp, col, val)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("tiled", [1, 0])
def test_jacobi_long_rows_on_both_global_paths(dtype, tiled):
    A = with_diagonal(300, 100, 400, 31, dtype)
    B = gen.random_csr(300, 40000, 100, 300, seed=32, dtype=dtype)
    dinv = diag_inv(A)
    rp, col, val, op = run_jacobi(A, B, 0.5, dinv, tiled_global=tiled)
    st = op.stats()
    assert st["num_rows"][9] > 0 and (st["num_tiles"] > 0) == bool(tiled)
    check(A, B, 0.5, dinv, rp, col, val)


def test_jacobi_long_rows_in_global_atomics():
    """FP64 rows of more than eight LDS segments (and too many tiles for the
    tiled path): the Jacobi step runs in C's own storage."""
    A = with_diagonal(8, 500, 600, 41)
    B = gen.random_csr(8, 3000000, 90000, 100000, seed=42)
    dinv = diag_inv(A)
    rp, col, val, op = run_jacobi(A, B, 0.9, dinv)
    assert op.stats()["num_rows"][9] > 0 and op.stats()["num_tiles"] == 0
    check(A, B, 0.9, dinv, rp, col, val)


def test_smoothed_aggregation_prolongator_3d():
    """(I - 2/3 D^-1 A) P with A the 7-point Laplacian on 24^3 and P the 2x2x2
    aggregation: the prolongator smoothing of algebraic multigrid."""
    A = gen.laplace3d_7pt(24)
    P = gen.aggregation_P(24)
    dinv = np.full(A.m, 1.0 / 6.0)
    rp, col, val, op = run_jacobi(A, P, 2.0 / 3.0, dinv)
    check(A, P, 2.0 / 3.0, dinv, rp, col, val)
    # every row of a smoothed piecewise-constant prolongator sums to 1 - omega/6 * (row sum of A)
    rows = np.repeat(np.arange(A.m), np.diff(rp))
    rowsum_a = np.add.reduceat(A.values, A.row_ptr[:-1].astype(np.int64))
    np.testing.assert_allclose(np.bincount(rows, weights=val), 1.0 - (2.0 / 3.0) / 6.0 * rowsum_a, atol=1e-13)


def test_jacobi_exact_on_diagonal_a_and_zero_omega():
    m = 500
    D = gen.csr_from_rows_cols(m, m, np.arange(m), np.arange(m), 2.0 + np.arange(m) % 5)
    B = gen.random_csr(m, 300, 0, 20, seed=51, value_kind="int")
    rp, col, val, _ = run_jacobi(D, B, 0.5, (1.0 / D.values).astype(np.float64))
    np.testing.assert_array_equal(rp, B.row_ptr.astype(np.int64))
    np.testing.assert_array_equal(col, B.col_idx)
    np.testing.assert_array_equal(val, 0.5 * B.values)
    A = with_diagonal(m, 0, 20, 52)
    rp, col, val, _ = run_jacobi(A, B, 0.0, diag_inv(A))
    check(A, B, 0.0, diag_inv(A), rp, col, val, exact=True)


def test_plain_and_jacobi_numeric_share_one_symbolic():
    A = with_diagonal(400, 0, 30, 61)
    B = gen.random_csr(400, 350, 0, 25, seed=62)
    dA, dB = DeviceCsr.from_host(A), DeviceCsr.from_host(B)
    op = SpGEMM(dA, dB)
    rp, nnz = op.symbolic()
    dinv = diag_inv(A)
    for _ in range(2):
        c1, v1 = op.numeric()
        c2, v2 = op.numeric_jacobi(0.6, torch.from_numpy(dinv).cuda())
        torch.cuda.synchronize()
        orp, ocol, oval, oabs = oracle.spgemm(A, B)
        np.testing.assert_array_equal(c1.cpu().numpy(), ocol)
        assert (np.abs(v1.cpu().numpy() - oval) <= 1e-12 * oabs).all()
        check(A, B, 0.6, dinv, rp.cpu().numpy().astype(np.int64), c2.cpu().numpy(), v2.cpu().numpy())


def test_jacobi_refuses_a_missing_diagonal_and_non_square_a():
    A = with_diagonal(100, 0, 10, 71, empty_diag_rows=[5, 77])
    B = gen.random_csr(100, 80, 0, 10, seed=72)
    dA, dB = DeviceCsr.from_host(A), DeviceCsr.from_host(B)
    op = SpGEMM(dA, dB)
    op.symbolic()
    with pytest.raises(SpgError) as e:
        op.numeric_jacobi(0.5, torch.ones(100, dtype=torch.float64, device="cuda"))
    assert e.value.status_name == "SPG_ERR_SHAPE" and "2 rows" in str(e.value)
    R = gen.random_csr(60, 100, 1, 10, seed=73)
    op = SpGEMM(DeviceCsr.from_host(R), dB)
    op.symbolic()
    with pytest.raises(SpgError) as e:
        op.numeric_jacobi(0.5, torch.ones(60, dtype=torch.float64, device="cuda"))
    assert e.value.status_name == "SPG_ERR_SHAPE"
