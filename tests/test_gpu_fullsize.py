"""Parity at the benchmark workloads' full sizes, in the launch configuration
bench.py times: every row of the 27-point 100^3 and R-MAT scale-18 products
compared entry by entry with the oracle (row-chunked), closed forms where they
exist, and the Galerkin chain bit-exact."""
import numpy as np
import pytest

import oracle
from paper_2103_11991_amd import gen
from gpu_util import compare_all_rows

pytestmark = pytest.mark.gpu


def setup_module(module):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _run(A, B, **opts):
    import torch
    from paper_2103_11991_amd.spgemm import DeviceCsr, SpGEMM
    dA = DeviceCsr.from_host(A)
    dB = dA if B is A else DeviceCsr.from_host(B)
    op = SpGEMM(dA, dB, **opts)
    rp, nnz = op.symbolic()
    col, val = op.numeric()
    torch.cuda.synchronize()
    return rp.cpu().numpy().astype(np.int64), col, val, op


@pytest.mark.timeout(600)
def test_stencil27_100_cubed():
    """The benchmark product (default options, as timed): every row's size
    against the closed form of the truncated {-2..2}^3 pattern, every row's
    columns bit-exact and values within 1e-12 x |A||B| of the oracle."""
    N = 100
    A = gen.stencil27(N, seed=2)
    rp, col, val, op = _run(A, A, timing=1)
    assert int(rp[-1]) == (5 * N - 6) ** 3 == 120553784
    assert op.stats()["products"] == (9 * N - 10) ** 3
    i = np.arange(N ** 3)
    c1 = lambda t: np.minimum(t, 2) + np.minimum(N - 1 - t, 2) + 1
    np.testing.assert_array_equal(np.diff(rp), c1(i % N) * c1((i // N) % N) * c1(i // (N * N)))
    compare_all_rows(A, A, rp, col, val)


@pytest.mark.timeout(900)
def test_rmat_scale18_every_row_plain_and_learned():
    """R-MAT scale 18 (FP32), seed 1: the plain product (default options, as
    timed) and the product with learned binning (the committed model when
    present, else a constant predictor) are each compared row by row with the
    FP64 oracle: columns bit-exact, values within 1e-5 x |A||B|."""
    import os
    import torch
    from paper_2103_11991_amd import learned
    from paper_2103_11991_amd.spgemm import DeviceCsr, SpGEMM
    A = gen.rmat(18, seed=1)
    rp, col, val, op = _run(A, A)
    ub = gen.products_per_row(A, A)
    assert op.stats()["products"] == int(ub.sum())
    compare_all_rows(A, A, rp, col, val, chunk_entries=1 << 26)
    del col, val
    torch.cuda.empty_cache()
    if os.path.exists(learned.DEFAULT_MODEL):
        w, margin, _ = learned.load()
    else:
        w, margin = np.zeros(1217, dtype=np.float32), 0.0
        w[-1] = 4.0
    dA = DeviceCsr.from_host(A)
    op = SpGEMM(dA, dA, binning=1, mlp_margin_milli=int(round(margin * 1000)))
    op.set_mlp(w)
    rp_l, _ = op.symbolic()
    col_l, val_l = op.numeric()
    torch.cuda.synchronize()
    rp_l = rp_l.cpu().numpy().astype(np.int64)
    np.testing.assert_array_equal(rp_l, rp)
    compare_all_rows(A, A, rp_l, col_l, val_l, chunk_entries=1 << 26)


def test_galerkin_128_cubed_five_levels_exact():
    """R A_l P = 4 L7(N/2) at every level of the 128^3 hierarchy, bit-exact."""
    import torch
    from paper_2103_11991_amd.spgemm import DeviceCsr, SpGEMM
    A = gen.laplace3d_7pt(128)
    scale = 1.0
    for N, P, R in gen.galerkin_hierarchy(128, 5):
        dA, dP, dR = DeviceCsr.from_host(A), DeviceCsr.from_host(P), DeviceCsr.from_host(R)
        op1 = SpGEMM(dA, dP)
        rp1, _ = op1.symbolic()
        c1, v1 = op1.numeric()
        AP = DeviceCsr(A.m, P.n, rp1, c1, v1)
        op2 = SpGEMM(dR, AP)
        rp2, _ = op2.symbolic()
        c2, v2 = op2.numeric()
        torch.cuda.synchronize()
        scale *= 4.0
        ref = gen.laplace3d_7pt(N // 2, scale=scale)
        np.testing.assert_array_equal(rp2.cpu().numpy(), ref.row_ptr)
        np.testing.assert_array_equal(c2.cpu().numpy(), ref.col_idx)
        np.testing.assert_array_equal(v2.cpu().numpy(), ref.values)
        A = ref


@pytest.mark.timeout(600)
def test_galerkin_level0_changed_values_every_row():
    """Symbolic once, numeric with changed values: every row of A*P and R*(AP)."""
    import torch
    from paper_2103_11991_amd.spgemm import DeviceCsr, SpGEMM
    A0 = gen.laplace3d_7pt(128)
    P = gen.aggregation_P(128)
    R = gen.transpose(P)
    dA, dP, dR = DeviceCsr.from_host(A0), DeviceCsr.from_host(P), DeviceCsr.from_host(R)
    op1 = SpGEMM(dA, dP)
    rp1, _ = op1.symbolic()
    rph = rp1.cpu().numpy().astype(np.int64)
    for t in (1, 7):
        A = A0.with_values(gen.sweep_values(A0, t))
        c1, v1 = op1.numeric(a_vals=torch.from_numpy(A.values).cuda())
        torch.cuda.synchronize()
        compare_all_rows(A, P, rph, c1, v1)
        AP = gen.Csr(A.m, P.n, rp1.cpu().numpy(), c1.cpu().numpy(), v1.cpu().numpy())
        op2 = SpGEMM(dR, DeviceCsr.from_host(AP))
        rp2, _ = op2.symbolic()
        c2, v2 = op2.numeric()
        torch.cuda.synchronize()
        compare_all_rows(R, AP, rp2.cpu().numpy().astype(np.int64), c2, v2)


@pytest.mark.timeout(900)
def test_banded_batch_1024_every_product():
    """The 1024-product banded batch in one graph launch and through the queued
    persistent kernel: every product's every row against the oracle."""
    import torch
    from paper_2103_11991_amd.spgemm import SpGEMMBatch
    pools = gen.banded_batch_pools(1024)
    dev = {k: torch.from_numpy(v).cuda() for k, v in pools.items() if k not in ("n", "a_nnz", "b_nnz")}
    n = pools["n"]
    batch = SpGEMMBatch.from_pools(n, n, n, pools["a_nnz"], pools["b_nnz"], dev["a_rp"], dev["a_ci"], dev["a_v"],
                                   dev["b_rp"], dev["b_ci"], dev["b_v"])
    nnz = batch.plan()
    batch.run()
    batch.run_queued(nnz)  # the same products through the persistent queued kernel
    torch.cuda.synchronize()
    assert (batch.q_offsets.cpu().numpy() >= 0).all()
    pairs = gen.pools_to_pairs(pools)
    for i, (A, B) in enumerate(pairs):
        rp, c, v = batch.product(i)
        compare_all_rows(A, B, rp.cpu().numpy().astype(np.int64), c, v)
        rq, cq, vq = batch.product_queued(i)
        compare_all_rows(A, B, rq.cpu().numpy(), cq, vq)
