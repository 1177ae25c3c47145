"""Sparse addition C = alpha*A + beta*B (both phases, through the C ABI)
against the oracle: structure bit-exact, values within the componentwise
tolerance (exact where each column has at most one entry of each matrix), on
rows sorted in registers, in a wavefront's LDS and on the long-row path,
sorted and unsorted inputs, repeats, empty rows and shapes, and numeric
reuse with new values."""
import numpy as np
import pytest
import torch

import oracle
from paper_2103_11991_amd import gen
from paper_2103_11991_amd._lib import SpgError
from paper_2103_11991_amd.spgemm import DeviceCsr, SpAdd
from gpu_util import TOL

pytestmark = pytest.mark.gpu


def setup_module(module):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def run_add(A, B, alpha, beta):
    add = SpAdd(DeviceCsr.from_host(A), DeviceCsr.from_host(B))
    rp, nnz = add.symbolic()
    col, val = add.numeric(alpha, beta)
    torch.cuda.synchronize()
    return rp.cpu().numpy().astype(np.int64), col.cpu().numpy(), val.cpu().numpy(), add


def check(A, B, alpha, beta, rp, col, val, exact=False):
    orp, ocol, oval, oabs = oracle.spadd(A, B, alpha, beta)
    np.testing.assert_array_equal(rp, orp)
    np.testing.assert_array_equal(col, ocol)
    v = val.astype(np.float64)
    if exact:
        np.testing.assert_array_equal(v, oval)
    else:
        bad = np.abs(v - oval) > TOL[np.dtype(A.values.dtype)] * oabs
        assert not bad.any(), (int(bad.sum()), v[bad][:4], oval[bad][:4])


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("lo,hi", [(0, 30), (20, 400), (600, 3000)])
@pytest.mark.parametrize("sorted_rows", [True, False])
def test_random_rows(dtype, lo, hi, sorted_rows):
    m, n = (3000, 40000) if hi <= 400 else (300, 200000)
    A = gen.random_csr(m, n, lo, hi, seed=lo + hi, dtype=dtype, sorted_rows=sorted_rows, empty_frac=0.05)
    B = gen.random_csr(m, n, lo, hi, seed=lo + hi + 1, dtype=dtype, sorted_rows=sorted_rows, empty_frac=0.05)
    rp, col, val, _ = run_add(A, B, 0.75, -1.25)
    # one entry of each matrix per column at most, FP64: alpha*a + beta*b exactly as the oracle rounds it
    check(A, B, 0.75, -1.25, rp, col, val, exact=dtype == np.float64)


@pytest.mark.parametrize("sorted_rows", [True, False])
def test_repeats_and_overlap(sorted_rows):
    """Repeated columns inside rows, and B's columns drawn from A's so most
    columns of C have entries of both."""
    A = gen.random_csr(2000, 300, 0, 60, seed=5, duplicates=True, sorted_rows=sorted_rows)
    B = gen.random_csr(2000, 300, 0, 60, seed=6, duplicates=True, sorted_rows=sorted_rows)
    rp, col, val, _ = run_add(A, B, 2.0, 3.0)
    check(A, B, 2.0, 3.0, rp, col, val)
    Ai = gen.random_csr(2000, 300, 0, 60, seed=7, duplicates=True, value_kind="int", sorted_rows=sorted_rows)
    Bi = gen.random_csr(2000, 300, 0, 60, seed=8, duplicates=True, value_kind="int", sorted_rows=sorted_rows)
    rp, col, val, _ = run_add(Ai, Bi, 2.0, -3.0)
    check(Ai, Bi, 2.0, -3.0, rp, col, val, exact=True)  # small integers: any order is exact


def test_a_minus_a_keeps_explicit_zeros():
    A = gen.random_csr(1500, 5000, 0, 200, seed=9)
    rp, col, val, _ = run_add(A, A, 1.0, -1.0)
    check(A, A, 1.0, -1.0, rp, col, val, exact=True)
    assert not val.any() and int(rp[-1]) == A.nnz


def test_one_side_empty_rows_and_shapes():
    A = gen.random_csr(500, 700, 0, 50, seed=10, empty_frac=0.5)
    Z = gen.Csr(500, 700, np.zeros(501, dtype=np.int32), np.zeros(0, dtype=np.int32), np.zeros(0))
    for X, Y in ((A, Z), (Z, A), (Z, Z)):
        rp, col, val, _ = run_add(X, Y, 1.5, 0.5)
        check(X, Y, 1.5, 0.5, rp, col, val, exact=True)
    E = gen.Csr(0, 10, np.zeros(1, dtype=np.int32), np.zeros(0, dtype=np.int32), np.zeros(0))
    rp, col, val, _ = run_add(E, E, 1.0, 1.0)
    assert rp.tolist() == [0] and col.size == 0


def test_numeric_reuse_with_new_values():
    A = gen.random_csr(4000, 900, 0, 80, seed=11)
    B = gen.random_csr(4000, 900, 0, 80, seed=12, sorted_rows=False)
    add = SpAdd(DeviceCsr.from_host(A), DeviceCsr.from_host(B))
    rp, nnz = add.symbolic()
    for t in range(3):
        A2 = A.with_values(np.random.default_rng(100 + t).normal(size=A.nnz))
        col, val = add.numeric(0.5 * t, 2.0, a_vals=torch.from_numpy(A2.values).cuda())
        torch.cuda.synchronize()
        check(A2, B, 0.5 * t, 2.0, rp.cpu().numpy().astype(np.int64), col.cpu().numpy(), val.cpu().numpy())


def test_row_pair_beyond_the_long_path_is_unsupported_and_bad_index_is_reported():
    A = gen.random_csr(4, 100000, 9000, 9000, seed=13)
    B = gen.random_csr(4, 100000, 9000, 9000, seed=14)
    add = SpAdd(DeviceCsr.from_host(A), DeviceCsr.from_host(B))
    with pytest.raises(SpgError) as e:
        add.symbolic()
    assert e.value.status_name == "SPG_ERR_UNSUPPORTED"
    A = gen.random_csr(50, 60, 1, 10, seed=15)
    bad = A.col_idx.copy()
    bad[7] = 60
    Ab = gen.Csr(50, 60, A.row_ptr, bad, A.values)
    add = SpAdd(DeviceCsr.from_host(Ab), DeviceCsr.from_host(A))
    with pytest.raises(SpgError) as e:
        add.symbolic()
    assert e.value.status_name == "SPG_ERR_INDEX"
