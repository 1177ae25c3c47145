"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Structure (row pointer, sorted column indices) must be bit-identical; values
within 1e-12 (FP64) or 1e-5 (FP32) of the FP64 oracle, componentwise against
sum |A(i,j)||B(j,c)|; exactly equal where all arithmetic is exact.
"""
import numpy as np
import pytest

from paper_2103_11991_amd import gen
from gpu_util import compare, run_gpu

pytestmark = pytest.mark.gpu


def setup_module(module):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_laplace2d_squared_is_bit_exact():
    A = gen.laplace2d_5pt(64)
    rp, c, v, op = run_gpu(A, A)
    assert int(rp[-1]) == 51972
    compare(A, A, rp, c, v, exact=True)


@pytest.mark.parametrize("binning", [2, 0])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("seed", range(6))
def test_random_shapes(seed, dtype, binning):
    rng = np.random.default_rng(seed)
    m, n, k = (int(x) for x in rng.integers(1, 700, size=3))
    A = gen.random_csr(m, n, 0, int(rng.integers(1, 40)), seed=seed, dtype=dtype, empty_frac=0.15,
                       duplicates=seed % 3 == 0, sorted_rows=seed % 2 == 0)
    B = gen.random_csr(n, k, 0, int(rng.integers(1, 60)), seed=seed + 77, dtype=dtype, empty_frac=0.1,
                       duplicates=seed % 4 == 1, sorted_rows=seed % 3 != 1)
    rp, c, v, _ = run_gpu(A, B, binning=binning)
    compare(A, B, rp, c, v)


@pytest.mark.parametrize("cls", list(range(29)))
def test_every_accumulator_class(cls):
    """All rows forced through one (mode, tier) class; rows that cannot fit fall back."""
    A = gen.random_csr(400, 300, 0, 12, seed=cls, empty_frac=0.1)
    B = gen.random_csr(300, 2000, 0, 20, seed=cls + 1)
    rp, c, v, op = run_gpu(A, B, force_class=cls)
    compare(A, B, rp, c, v)
    S = gen.stencil27(9, seed=3)
    rp, c, v, op = run_gpu(S, S, force_class=cls)
    compare(S, S, rp, c, v)


@pytest.mark.parametrize("cls", [3, 4, 5, 6, 7, 8, 13, 14, 15, 16, 23, 24, 25, 26, 27, 28])
def test_many_batches_and_chunks(cls):
    """Rows of ~150 A entries and ~3000 products (onto at most 200 columns),
    forced into groups of 64 to 1024 lanes: several chunks of A per row and
    several batches of products and runs per chunk, with empty B rows among
    the staged entries."""
    A = gen.random_csr(96, 800, 100, 200, seed=40 + cls, empty_frac=0.05)
    B = gen.random_csr(800, 200, 0, 40, seed=41 + cls, empty_frac=0.2)
    rp, c, v, op = run_gpu(A, B, force_class=cls)
    st = op.stats()
    assert st["num_rows"][cls] > 0
    compare(A, B, rp, c, v)


def test_global_path_with_global_slabs():
    """Rows spanning ~2^21 columns: mask tables exceed LDS and live in global slabs."""
    A = gen.random_csr(40, 60, 1, 10, seed=5)
    B = gen.random_csr(60, 1 << 21, 20, 400, seed=6)
    rp, c, v, op = run_gpu(A, B)
    compare(A, B, rp, c, v)
    # the same rows forced onto the global path: their tables exceed LDS
    rp, c, v, op = run_gpu(A, B, force_class=9)
    st = op.stats()
    assert st["sym_rows"][9] == st["num_rows"][9] == A.m - st["empty_rows"] > 0
    compare(A, B, rp, c, v)


def test_long_rows_accumulate_in_output():
    """Dense-ish rows with thousands of entries go to the global path (values in C)."""
    A = gen.random_csr(30, 500, 50, 400, seed=8)
    B = gen.random_csr(500, 20000, 50, 500, seed=9, dtype=np.float64)
    rp, c, v, op = run_gpu(A, B)
    assert op.stats()["num_rows"][9] > 0
    compare(A, B, rp, c, v)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_long_rows_in_lds_segments_and_global_atomics(dtype):
    """Global-path rows: ~25k-entry rows summed in a few LDS segments,
    ~100k-entry rows in up to eight (FP64) or five (FP32), and ~250k-entry
    rows (more than eight segments) with global atomics."""
    for k, lo, hi in ((30000, 100, 300), (400000, 300, 400), (4000000, 600, 700)):
        A = gen.random_csr(12, 600, lo, hi, seed=k, dtype=dtype)
        B = gen.random_csr(600, k, 300, 500, seed=k + 1, dtype=dtype)
        rp, c, v, op = run_gpu(A, B)
        assert op.stats()["num_rows"][9] > 0
        compare(A, B, rp, c, v)


@pytest.mark.parametrize("seed", range(3))
def test_identity_products(seed):
    A = gen.random_csr(500, 400, 0, 30, seed=seed, empty_frac=0.2)
    for X, Y in ((A, gen.identity(400)), (gen.identity(500), A)):
        rp, c, v, _ = run_gpu(X, Y)
        np.testing.assert_array_equal(rp, A.row_ptr.astype(np.int64))
        np.testing.assert_array_equal(c, A.col_idx)
        np.testing.assert_array_equal(v, A.values)


def test_stencil27_closed_form_and_parity():
    N = 20
    A = gen.stencil27(N, seed=2)
    rp, c, v, op = run_gpu(A, A)
    assert int(rp[-1]) == (5 * N - 6) ** 3
    assert op.stats()["products"] == (9 * N - 10) ** 3
    compare(A, A, rp, c, v)


def test_rmat_fp32():
    A = gen.rmat(12, seed=1)
    rp, c, v, _ = run_gpu(A, A)
    compare(A, A, rp, c, v)


def test_galerkin_exact():
    N = 16
    A = gen.laplace3d_7pt(N)
    P = gen.aggregation_P(N)
    R = gen.transpose(P)
    rp, c, v, _ = run_gpu(A, P)
    AP = gen.Csr(A.m, P.n, rp.astype(np.int32), c, v)
    rp2, c2, v2, _ = run_gpu(R, AP)
    ref = gen.laplace3d_7pt(N // 2, scale=4.0)
    np.testing.assert_array_equal(rp2, ref.row_ptr.astype(np.int64))
    np.testing.assert_array_equal(c2, ref.col_idx)
    np.testing.assert_array_equal(v2, ref.values)


def test_rows_past_the_list_limit_take_the_global_path():
    """With 1 MiB of list memory (131072 pairs) only some rows of a 27-point
    stencil on 30^3 get a list (each reserves 100-250 pairs): the others are
    computed by the numeric global path from compressed B.  The product is
    unchanged, also when numeric is run again with new values."""
    import torch
    A = gen.stencil27(30, seed=4)
    rp, c, v, op = run_gpu(A, A, list_limit_mb=1)
    st = op.stats()
    assert 0 < st["list_pairs"] <= (1 << 20) // 8
    assert st["num_rows"][9] > 0 and sum(st["num_rows"][:9]) + sum(st["num_rows"][10:]) > 0
    compare(A, A, rp, c, v)
    A2 = A.with_values(gen.sweep_values(A, 2))
    col, val = op.numeric(a_vals=torch.from_numpy(A2.values).cuda())
    torch.cuda.synchronize()
    compare(A2, A, rp, col.cpu().numpy(), val.cpu().numpy())


def test_small_classes_merge_into_larger_tiers():
    """The boundary rows of a stencil form small classes beside the interior
    class; merged, they run in the larger tier of the same mode.  The product
    is the same either way, and rows only move to larger tiers of their mode."""
    A = gen.stencil27(40, seed=6)
    rp1, c1, v1, op1 = run_gpu(A, A, merge_classes=0)
    rp2, c2, v2, op2 = run_gpu(A, A)
    compare(A, A, rp2, c2, v2)
    np.testing.assert_array_equal(rp1, rp2)
    np.testing.assert_array_equal(c1, c2)
    for key in ("sym_rows", "num_rows"):
        off, on = np.array(op1.stats()[key]), np.array(op2.stats()[key])
        assert off.sum() == on.sum()
        assert np.count_nonzero(on) < np.count_nonzero(off)
        for mode in range(3):
            a, b = off[mode * 10:mode * 10 + 9], on[mode * 10:mode * 10 + 9]
            # merged counts are suffix sums' worth: no rows move to a smaller tier
            assert all(b[t:].sum() >= a[t:].sum() for t in range(9))


def test_numeric_launch_times_are_summed_without_waiting():
    """Timing level 2 sums every numeric class launch since the option was
    set: three products and two reused numeric calls give five launches per
    launched class, and setting the option again starts from zero."""
    import torch
    from paper_2103_11991_amd.spgemm import DeviceCsr, SpGEMM
    A = gen.stencil27(20, seed=3)
    dA = DeviceCsr.from_host(A)
    op = SpGEMM(dA, dA, timing=2)
    for _ in range(3):
        op.symbolic()
        col, val = op.numeric()
    for _ in range(2):
        op.numeric(out_col=col, out_val=val)
    torch.cuda.synchronize()
    st = op.stats()
    launched = [c for c in range(30) if st["num_rows"][c]]
    assert launched
    for c in range(30):
        assert st["num_class_launches"][c] == (5 if c in launched else 0)
        assert (st["num_class_ms_total"][c] > 0) == (c in launched)
        if c in launched:  # the last launch is one of the five summed
            assert 0 < st["num_class_ms"][c] <= st["num_class_ms_total"][c]
    assert st["sym_ms"] == 0.0  # level 2 times no symbolic stage
    compare(A, A, op.row_ptr.cpu().numpy().astype(np.int64), col.cpu().numpy(), val.cpu().numpy())
    op.set_option("timing", 2)
    assert sum(op.stats()["num_class_launches"]) == 0


def test_list_memory_is_the_run_bound():
    """Each row reserves min(compressed-B runs of its products, words of its
    column range) list pairs."""
    A = gen.random_csr(500, 3000, 0, 30, seed=8, empty_frac=0.1)
    B = gen.random_csr(3000, 9000, 0, 25, seed=9)
    rp, c, v, op = run_gpu(A, B)
    compare(A, B, rp, c, v)
    def runs_of_row(j):  # maximal runs of consecutive stored entries in one 32-column block
        blk = B.col_idx[B.row_ptr[j]:B.row_ptr[j + 1]] >> 5
        return int(len(blk) > 0) + int(np.count_nonzero(blk[1:] != blk[:-1]))
    runs = np.array([runs_of_row(j) for j in range(B.m)])
    want = 0
    for i in range(A.m):
        js = A.col_idx[A.row_ptr[i]:A.row_ptr[i + 1]]
        cols = np.concatenate([B.col_idx[B.row_ptr[j]:B.row_ptr[j + 1]] for j in js]) if len(js) else []
        if len(cols):
            want += min(int(runs[js].sum()), int((cols.max() >> 5) - (cols.min() >> 5) + 1))
    assert op.stats()["list_pairs"] == want


def test_symbolic_reuse_with_new_values():
    import torch
    from paper_2103_11991_amd.spgemm import DeviceCsr, SpGEMM
    A0 = gen.laplace3d_7pt(12)
    P = gen.aggregation_P(12)
    dA = DeviceCsr.from_host(A0)
    dP = DeviceCsr.from_host(P)
    op = SpGEMM(dA, dP)
    rp, nnz = op.symbolic()
    rph = rp.cpu().numpy().astype(np.int64)
    for t in range(1, 4):
        A = A0.with_values(gen.sweep_values(A0, t))
        col, val = op.numeric(a_vals=torch.from_numpy(A.values).cuda())
        torch.cuda.synchronize()
        compare(A, P, rph, col.cpu().numpy(), val.cpu().numpy())


def test_empty_and_degenerate():
    for m, n, k, la, lb in ((0, 5, 5, 3, 3), (5, 0, 5, 0, 3), (5, 5, 0, 3, 0), (7, 6, 5, 0, 0), (1, 1, 1, 1, 1)):
        A = gen.random_csr(m, n, 0, la, seed=1)
        B = gen.random_csr(n, k, 0, lb, seed=2)
        rp, c, v, _ = run_gpu(A, B)
        assert rp.shape == (m + 1,)
        compare(A, B, rp, c, v)


def test_bad_index_is_reported():
    import torch
    from paper_2103_11991_amd._lib import SpgError
    from paper_2103_11991_amd.spgemm import DeviceCsr, SpGEMM
    A = gen.random_csr(50, 40, 1, 5, seed=3)
    bad = A.col_idx.copy()
    bad[7] = 40  # one past the last column
    dA = DeviceCsr.from_host(gen.Csr(50, 40, A.row_ptr, bad, A.values))
    dB = DeviceCsr.from_host(gen.random_csr(40, 30, 1, 5, seed=4))
    op = SpGEMM(dA, dB)
    with pytest.raises(SpgError) as e:
        op.symbolic()
    assert e.value.status_name == "SPG_ERR_INDEX"
    rp = A.row_ptr.copy()
    rp[10] = rp[11] + 1  # not monotone
    dA2 = DeviceCsr.from_host(gen.Csr(50, 40, rp, A.col_idx, A.values))
    with pytest.raises(SpgError):
        SpGEMM(dA2, dB).symbolic()
    torch.cuda.synchronize()


def test_numeric_before_symbolic_is_state_error():
    from paper_2103_11991_amd import _lib
    from paper_2103_11991_amd.spgemm import DeviceCsr, SpGEMM
    A = DeviceCsr.from_host(gen.random_csr(10, 10, 1, 3, seed=1))
    op = SpGEMM(A, A)
    with pytest.raises(_lib.SpgError) as e:
        _lib.spg_numeric(op.h, A.values.data_ptr(), A.values.data_ptr(), A.col_idx.data_ptr(), A.values.data_ptr())
    assert e.value.status_name == "SPG_ERR_STATE"


def test_nnz_beyond_int32_is_an_overflow_error():
    """A = 46341 x 1 column of ones, B = 1 x 46341 row of ones: every row of C
    is full, so nnz(C) = 46341^2 = 2,147,488,281 >= 2^31.  Symbolic reports
    SPG_ERR_OVERFLOW and leaves no symbolic result (numeric is a state error).
    The row-pointer scan runs in 64 bits and only its int32 store is
    truncated; nothing indexes with the truncated values before the error is
    returned.  A square of one row less fits (46340^2 < 2^31)."""
    import torch
    from paper_2103_11991_amd import _lib
    from paper_2103_11991_amd.spgemm import DeviceCsr, SpGEMM
    for n, overflow in ((46341, True), (46340, False)):
        dev = "cuda"
        A = DeviceCsr(n, 1, torch.arange(n + 1, dtype=torch.int32, device=dev),
                      torch.zeros(n, dtype=torch.int32, device=dev), torch.ones(n, dtype=torch.float64, device=dev))
        B = DeviceCsr(1, n, torch.tensor([0, n], dtype=torch.int32, device=dev),
                      torch.arange(n, dtype=torch.int32, device=dev), torch.ones(n, dtype=torch.float64, device=dev))
        op = SpGEMM(A, B)
        if overflow:
            assert n * n >= 2 ** 31
            with pytest.raises(_lib.SpgError) as e:
                op.symbolic()
            assert e.value.status_name == "SPG_ERR_OVERFLOW"
            with pytest.raises(_lib.SpgError) as e:
                _lib.spg_numeric(op.h, A.values.data_ptr(), B.values.data_ptr(), A.col_idx.data_ptr(),
                                 A.values.data_ptr())
            assert e.value.status_name == "SPG_ERR_STATE"
        else:
            rp, nnz = op.symbolic()
            torch.cuda.synchronize()
            assert nnz == n * n < 2 ** 31
            rph = rp.cpu().numpy().astype(np.int64)
            np.testing.assert_array_equal(rph, np.arange(n + 1, dtype=np.int64) * n)
            # the symbolic phase alone: C itself would take 26 GB
        del op
        torch.cuda.synchronize()


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_one_wait_and_two_wait_symbolic_agree(dtype):
    """A product whose list bound m x (k/32 + 1) is small waits for the device
    once (every launch sized on the device); with the list limit below that
    bound the same product reads the analysis back first (two waits, exact
    sizes).  Both match the oracle, and each other bit for bit in structure."""
    A = gen.random_csr(3000, 2500, 0, 30, seed=21, dtype=dtype, empty_frac=0.1, duplicates=True)
    B = gen.random_csr(2500, 40000, 0, 40, seed=22, dtype=dtype, sorted_rows=False)
    rp1, c1, v1, op1 = run_gpu(A, B)
    assert op1.stats()["sym_waits"] == 1
    compare(A, B, rp1, c1, v1)
    rp2, c2, v2, op2 = run_gpu(A, B, list_limit_mb=1)
    assert op2.stats()["sym_waits"] == 2
    compare(A, B, rp2, c2, v2)
    np.testing.assert_array_equal(rp1, rp2)
    np.testing.assert_array_equal(c1, c2)


def test_one_wait_symbolic_global_path_and_learned_retry():
    """One-wait products whose rows reach the symbolic global path (forced)
    and whose learned sizes overflow (a constant predictor of 1 block): the
    device-sized global launch and the exact retry give the oracle's product."""
    A = gen.random_csr(700, 600, 0, 60, seed=23, empty_frac=0.2)
    B = gen.random_csr(600, 20000, 0, 80, seed=24)
    rp, c, v, op = run_gpu(A, B, force_class=9)
    assert op.stats()["sym_waits"] == 1
    compare(A, B, rp, c, v)
    import torch
    from paper_2103_11991_amd.spgemm import DeviceCsr, SpGEMM
    w = np.zeros(1217, dtype=np.float32)
    w[-1] = 1.0
    op = SpGEMM(DeviceCsr.from_host(A), DeviceCsr.from_host(B), binning=1, mlp_margin_milli=0)
    op.set_mlp(w)
    rp, _ = op.symbolic()
    col, val = op.numeric()
    torch.cuda.synchronize()
    st = op.stats()
    assert st["sym_waits"] == 1 and st["retried_rows"] > 0
    compare(A, B, rp.cpu().numpy().astype(np.int64), col.cpu().numpy(), val.cpu().numpy())


def test_large_product_waits_twice():
    A = gen.stencil27(40, seed=2)
    rp, c, v, op = run_gpu(A, A)
    assert op.stats()["sym_waits"] == 2  # 64000 rows x 2001 words > 2^25 list pairs
    assert int(rp[-1]) == (5 * 40 - 6) ** 3
    compare(A, A, rp, c, v, rows=[(0, 3000), (30000, 33000), (61000, 64000)])
