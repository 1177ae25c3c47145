"""The paper's design kept for comparison (SPG_OPT_METHOD 1..3: one
parallelisation method for the whole matrix, two-level hash maps with a lazily
created global level) against the oracle.  Its numeric phase leaves rows in
hash order, so each row is compared as a set: the row pointer bit-exact, the
row's columns once sorted bit-exact, values matched to their columns within
the componentwise tolerance."""
import numpy as np
import pytest
import torch

import oracle
from paper_2103_11991_amd import gen
from paper_2103_11991_amd._lib import SpgError
from paper_2103_11991_amd.spgemm import DeviceCsr, SpGEMM
from gpu_util import TOL, run_gpu

pytestmark = pytest.mark.gpu


def setup_module(module):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def check_rows_as_sets(A, B, rp, col, val):
    orp, ocol, oval, oabs = oracle.spgemm(A, B)
    np.testing.assert_array_equal(rp, orp)
    rows = np.repeat(np.arange(A.m), np.diff(rp))
    order = np.lexsort((col, rows))  # sort each row by column
    np.testing.assert_array_equal(col[order], ocol)
    v = val[order].astype(np.float64)
    bad = np.abs(v - oval) > TOL[np.dtype(A.values.dtype)] * oabs
    assert not bad.any(), (int(bad.sum()), v[bad][:4], oval[bad][:4])


@pytest.mark.parametrize("method", [1, 2, 3])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_random_products(method, dtype):
    A = gen.random_csr(900, 700, 0, 40, seed=3, dtype=dtype, empty_frac=0.1, duplicates=True)
    B = gen.random_csr(700, 5000, 0, 60, seed=4, dtype=dtype, sorted_rows=False)
    rp, col, val, _ = run_gpu(A, B, method=method)
    check_rows_as_sets(A, B, rp, col, val)


@pytest.mark.parametrize("method", [2, 3])
def test_level_two_is_created_for_long_rows(method):
    """Rows of thousands of columns overflow level 1 in both phases (256
    slots per row for the group method, 4096 for the team method) and go on
    in the global level; short rows in the same product never create it."""
    A = gen.random_csr(200, 600, 0, 300, seed=5, empty_frac=0.2)
    B = gen.random_csr(600, 60000, 0, 200, seed=6)
    rp, col, val, _ = run_gpu(A, B, method=method)
    assert np.diff(rp).max() > 8000
    check_rows_as_sets(A, B, rp, col, val)


def test_auto_method_on_stencil_and_rmat():
    A = gen.stencil27(14, seed=2)
    rp, col, val, _ = run_gpu(A, A, method=1)
    assert int(rp[-1]) == (5 * 14 - 6) ** 3
    check_rows_as_sets(A, A, rp, col, val)
    R = gen.rmat(12, seed=1)
    rp, col, val, _ = run_gpu(R, R, method=1)
    check_rows_as_sets(R, R, rp, col, val)


def test_numeric_reuse_and_jacobi_refused():
    A = gen.laplace2d_5pt(40)
    dA = DeviceCsr.from_host(A)
    op = SpGEMM(dA, dA, method=2)
    rp, nnz = op.symbolic()
    for t in range(2):
        A2 = A.with_values(np.random.default_rng(t).normal(size=A.nnz))
        col, val = op.numeric(a_vals=torch.from_numpy(A2.values).cuda())
        torch.cuda.synchronize()
        check_rows_as_sets(A2, A, rp.cpu().numpy().astype(np.int64), col.cpu().numpy(), val.cpu().numpy())
    with pytest.raises(SpgError) as e:
        op.numeric_jacobi(0.5, torch.full((A.m,), 0.25, dtype=torch.float64, device="cuda"))
    assert e.value.status_name == "SPG_ERR_UNSUPPORTED"
