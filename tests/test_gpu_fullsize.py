"""Parity at the benchmark workloads' full sizes, in the launch configuration
bench.py times: whole-structure checks where a closed form or the oracle's row
count covers every row, and sampled rows compared entry by entry."""
import numpy as np
import pytest

import oracle
from paper_2103_11991_amd import gen
from gpu_util import TOL

pytestmark = pytest.mark.gpu


def setup_module(module):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _sample_rows(m, rng, count=24, width=64, extra=()):
    starts = sorted(set([0, max(0, m - width)] + [int(x) for x in rng.integers(0, max(1, m - width), count)]))
    ranges = [(s, min(m, s + width)) for s in starts]
    ranges += [(int(r), int(r) + 1) for r in extra]
    return ranges


def _check_rows(A, B, rp, col, val, ranges):
    """rp: full host row pointer; col/val: device tensors (sliced per range)."""
    tol = TOL[np.dtype(A.values.dtype)]
    for r0, r1 in ranges:
        orp, ocol, oval, oabs = oracle.spgemm(A, B, r0, r1)
        g0, g1 = int(rp[r0]), int(rp[r1])
        np.testing.assert_array_equal(rp[r0:r1 + 1] - rp[r0], orp)
        np.testing.assert_array_equal(col[g0:g1].cpu().numpy(), ocol)
        v = val[g0:g1].cpu().numpy().astype(np.float64)
        bad = np.abs(v - oval) > tol * oabs
        assert not bad.any(), (r0, r1, int(bad.sum()))


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


def test_stencil27_100_cubed():
    N = 100
    A = gen.stencil27(N, seed=2)
    rp, col, val, op = _run(A, A, timing=1)
    assert int(rp[-1]) == (5 * N - 6) ** 3 == 120553784
    assert op.stats()["products"] == (9 * N - 10) ** 3
    # every row's size against the closed form of the truncated {-2..2}^3 pattern
    i = np.arange(N ** 3)
    c1 = lambda t: np.minimum(t, 2) + np.minimum(N - 1 - t, 2) + 1
    np.testing.assert_array_equal(np.diff(rp), c1(i % N) * c1((i // N) % N) * c1(i // (N * N)))
    _check_rows(A, A, rp, col, val, _sample_rows(A.m, np.random.default_rng(0)))


def test_rmat_scale18_row_sizes_and_hub_rows():
    A = gen.rmat(18, seed=1)
    rp, col, val, op = _run(A, A)
    np.testing.assert_array_equal(np.diff(rp), oracle.row_nnz(A, A))
    ub = gen.products_per_row(A, A)
    hubs = np.argsort(ub)[-6:]
    _check_rows(A, A, rp, col, val, _sample_rows(A.m, np.random.default_rng(1), count=16, width=32, extra=hubs))


def test_rmat_scale18_learned_binning_same_structure():
    """Learned binning (committed model when present, else a constant
    predictor) gives the same product as upper-bound binning."""
    import os
    from paper_2103_11991_amd import learned
    A = gen.rmat(18, seed=2)
    rp0, col0, val0, _ = _run(A, A)
    if os.path.exists(learned.DEFAULT_MODEL):
        w, margin, _ = learned.load()
    else:
        w, margin = np.zeros(1217, dtype=np.float32), 0.0
        w[-1] = 4.0
    import torch
    from paper_2103_11991_amd.spgemm import DeviceCsr, SpGEMM
    dA = DeviceCsr.from_host(A)
    op = SpGEMM(dA, dA, binning=1, mlp_margin_milli=int(round(margin * 1000)))
    op.set_mlp(w)
    rp, nnz = op.symbolic()
    col, val = op.numeric()
    torch.cuda.synchronize()
    np.testing.assert_array_equal(rp.cpu().numpy().astype(np.int64), rp0)
    assert torch.equal(col, col0)
    d = (val.double() - val0.double()).abs()
    assert float(d.max()) <= 1e-5 * float(val0.double().abs().max())


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


def test_galerkin_level0_changed_values_sampled():
    """Symbolic once, numeric with changed values: sampled rows of A*P and R*(AP)."""
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
        _check_rows(A, P, rph, c1, v1, _sample_rows(A.m, np.random.default_rng(t)))
        AP = gen.Csr(A.m, P.n, rp1.cpu().numpy(), c1.cpu().numpy(), v1.cpu().numpy())
        op2 = SpGEMM(dR, DeviceCsr.from_host(AP))
        rp2, _ = op2.symbolic()
        c2, v2 = op2.numeric()
        torch.cuda.synchronize()
        _check_rows(R, AP, rp2.cpu().numpy().astype(np.int64), c2, v2,
                    _sample_rows(R.m, np.random.default_rng(10 + t)))


def test_banded_batch_1024_sampled_products():
    import torch
    from paper_2103_11991_amd.spgemm import SpGEMMBatch
    pools = gen.banded_batch_pools(1024)
    dev = {k: torch.from_numpy(v).cuda() for k, v in pools.items() if k not in ("n", "a_nnz", "b_nnz")}
    n = pools["n"]
    batch = SpGEMMBatch.from_pools(n, n, n, pools["a_nnz"], pools["b_nnz"], dev["a_rp"], dev["a_ci"], dev["a_v"],
                                   dev["b_rp"], dev["b_ci"], dev["b_v"])
    batch.plan()
    batch.run()
    torch.cuda.synchronize()
    pairs = gen.pools_to_pairs(pools)
    rng = np.random.default_rng(5)
    for i in sorted(set([0, 1023] + [int(x) for x in rng.integers(0, 1024, 14)])):
        A, B = pairs[i]
        rp, c, v = batch.product(i)
        _check_rows(A, B, rp.cpu().numpy().astype(np.int64), c, v, [(0, A.m)])
