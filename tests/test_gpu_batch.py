"""Batched products: every C_i of one graph launch equals the oracle's
product, replays pick up changed values, numeric-only replays reuse the
planned structure, and the autotuner keeps the product unchanged."""
import numpy as np
import pytest

from paper_2103_11991_amd import gen
from gpu_util import compare

pytestmark = pytest.mark.gpu


def setup_module(module):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _products(count, seed):
    out = []
    n, bwa, bwb = gen.batch_sizes(count, seed=seed, lo=50, hi=3000)
    for i in range(count):
        if i % 7 == 3:      # an empty product and odd shapes among the banded ones
            A = gen.random_csr(40, 30, 0, 0, seed=i)
            B = gen.random_csr(30, 20, 0, 4, seed=i + 1)
        elif i % 7 == 5:
            A = gen.random_csr(300, 200, 0, 25, seed=i, empty_frac=0.2)
            B = gen.random_csr(200, 5000, 0, 40, seed=i + 1)
        else:
            A = gen.banded_random(int(n[i]), int(bwa[i]), seed, 2 * i)
            B = gen.banded_random(int(n[i]), int(bwb[i]), seed, 2 * i + 1)
        out.append((A, B))
    return out


def _check_all(batch, prods):
    import torch
    torch.cuda.synchronize()
    for i, (A, B) in enumerate(prods):
        rp, c, v = batch.product(i)
        compare(A, B, rp.cpu().numpy().astype(np.int64), c.cpu().numpy(), v.cpu().numpy())


def test_batch_matches_oracle_and_replays():
    import torch
    from paper_2103_11991_amd.spgemm import DeviceCsr, SpGEMMBatch
    prods = _products(30, 5)
    batch = SpGEMMBatch([DeviceCsr.from_host(A) for A, _ in prods], [DeviceCsr.from_host(B) for _, B in prods])
    nnz = batch.plan()
    batch.run()
    _check_all(batch, prods)
    # replay of the same graph with new values written in place
    prods2 = [(A.with_values(A.values * 2.0 - 1.0), B) for A, B in prods]
    batch.a_v.copy_(torch.from_numpy(np.concatenate([A.values for A, _ in prods2])).cuda())
    for _ in range(3):
        batch.c_val.zero_()
        batch.c_col.zero_()
        batch.run()
        _check_all(batch, prods2)
    # numeric alone on the planned structure
    batch.c_rp.zero_()
    batch.run(numeric_only=True)
    _check_all(batch, prods2)
    assert nnz == sum(int(batch.c_nnz_off[i + 1] - batch.c_nnz_off[i]) for i in range(30))


def test_batch_fp32_and_learned_binning():
    from paper_2103_11991_amd.spgemm import DeviceCsr, SpGEMMBatch
    prods = [(A.astype(np.float32), B.astype(np.float32)) for A, B in _products(12, 9)]
    w = np.zeros(1217, dtype=np.float32)
    w[-1] = 1.0  # tiny tables everywhere: hashed rows overflow and are retried
    batch = SpGEMMBatch([DeviceCsr.from_host(A) for A, _ in prods], [DeviceCsr.from_host(B) for _, B in prods],
                        binning=1, mlp_margin_milli=0)
    batch.set_mlp(w)
    batch.plan()
    batch.run()
    _check_all(batch, prods)
    batch.run()
    _check_all(batch, prods)


def test_autotuner_keeps_the_product():
    from paper_2103_11991_amd.spgemm import DeviceCsr, SpGEMMBatch
    prods = _products(10, 3)
    batch = SpGEMMBatch([DeviceCsr.from_host(A) for A, _ in prods], [DeviceCsr.from_host(B) for _, B in prods])
    chosen, best = batch.tune()
    assert chosen[0] in (8, 16, 32) and chosen[1] in (0, 2) and chosen[2] in (32, 64, 128)
    assert best > 0
    batch.run()
    _check_all(batch, prods)


def test_batch_rejects_bad_product():
    import torch
    from paper_2103_11991_amd import _lib
    from paper_2103_11991_amd.spgemm import DeviceCsr, SpGEMMBatch
    A = gen.random_csr(20, 10, 1, 4, seed=1)
    B = gen.random_csr(10, 8, 1, 4, seed=2)
    badB = gen.Csr(10, 8, B.row_ptr, np.where(B.col_idx == B.col_idx.max(), 8, B.col_idx).astype(np.int32),
                   B.values)
    with pytest.raises(_lib.SpgError):
        SpGEMMBatch([DeviceCsr.from_host(A)] * 2, [DeviceCsr.from_host(B), DeviceCsr.from_host(badB)])
    torch.cuda.synchronize()


def test_failed_tune_leaves_the_batch_unplanned_with_its_options():
    """A tuning trial that fails (here: no A values, found by the first trial's
    numeric after its symbolic ran with the trial options) returns the error,
    leaves the batch unplanned (run is a state error, no stale graph is
    replayed) and its options as they were; planning again restores it."""
    import torch
    from paper_2103_11991_amd import _lib
    from paper_2103_11991_amd.spgemm import DeviceCsr, SpGEMMBatch
    prods = _products(6, 9)
    batch = SpGEMMBatch([DeviceCsr.from_host(A) for A, _ in prods], [DeviceCsr.from_host(B) for _, B in prods],
                        work_per_lane=16)
    batch.plan()
    batch.run()
    torch.cuda.synchronize()
    _check_all(batch, prods)
    before = batch.stats()
    ptrs = list(batch._ptrs(None, None))
    ptrs[0] = 0  # no A values
    with pytest.raises(_lib.SpgError):
        _lib.spg_batch_tune(batch.b, *ptrs)
    with pytest.raises(_lib.SpgError) as e:
        _lib.spg_batch_run(batch.b, *batch._ptrs(None, None), 0)
    assert e.value.status_name == "SPG_ERR_STATE"
    batch.plan()
    batch.run()
    torch.cuda.synchronize()
    after = batch.stats()
    # same options: same classes for every row
    assert after["sym_rows"] == before["sym_rows"] and after["num_rows"] == before["num_rows"]
    _check_all(batch, prods)


def _banded_products(count, seed, lo=50, hi=3000):
    """Banded products (every row of C spans at most 257 columns), with an
    empty product and one of a single row among them."""
    n, bwa, bwb = gen.batch_sizes(count, seed=seed, lo=lo, hi=hi)
    out = []
    for i in range(count):
        if i % 9 == 4:
            A = gen.random_csr(40, 30, 0, 0, seed=i)
            B = gen.random_csr(30, 20, 0, 4, seed=i + 1)
        elif i % 9 == 7:
            A = gen.random_csr(1, 60, 1, 20, seed=i)
            B = gen.random_csr(60, 90, 0, 30, seed=i + 1)
        else:
            A = gen.banded_random(int(n[i]), int(bwa[i]), seed, 2 * i)
            B = gen.banded_random(int(n[i]), int(bwb[i]), seed, 2 * i + 1)
        out.append((A, B))
    return out


def _check_queued(batch, prods):
    import torch
    torch.cuda.synchronize()
    for i, (A, B) in enumerate(prods):
        got = batch.product_queued(i)
        assert got is not None, i
        rp, c, v = got
        compare(A, B, rp.cpu().numpy(), c.cpu().numpy(), v.cpu().numpy())


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_queued_batch_matches_oracle_and_replays(dtype):
    """One persistent kernel: every product against the oracle, on graph
    replays with new values, with per-product device time stamps."""
    import oracle
    import torch
    from paper_2103_11991_amd.spgemm import DeviceCsr, SpGEMMBatch
    prods = [(A.astype(dtype), B.astype(dtype)) for A, B in _banded_products(40, 7)]
    need = sum(int(oracle.row_nnz(A, B).sum()) for A, B in prods)
    batch = SpGEMMBatch([DeviceCsr.from_host(A) for A, _ in prods], [DeviceCsr.from_host(B) for _, B in prods])
    batch.run_queued(need)
    _check_queued(batch, prods)
    offs = batch.q_offsets.cpu().numpy()
    assert (offs >= 0).all() and len(set(offs[[A.m > 0 for A, _ in prods]].tolist())) >= 1
    st = batch.q_stamps.cpu().numpy().reshape(-1, 2)
    busy = np.array([A.m > 0 for A, _ in prods])
    assert (st[busy, 0] <= st[busy, 1]).all() and (st[busy, 0] > 0).all()
    # the pools hold exactly the products, in the order their symbolic work ended
    sizes = np.array([int(oracle.row_nnz(A, B).sum()) for A, B in prods])
    assert np.array_equal(np.sort(offs[busy] + sizes[busy])[-1:], [need])
    prods2 = [(A.with_values((A.values * 2.0 - 1.0).astype(dtype)), B) for A, B in prods]
    batch.a_v.copy_(torch.from_numpy(np.concatenate([A.values for A, _ in prods2])).cuda())
    for _ in range(3):
        batch.q_val.zero_()
        batch.q_col.zero_()
        batch.run_queued(need)
        _check_queued(batch, prods2)


def test_queued_batch_pool_too_small_skips_products():
    """A pool with room for about half the entries: products that got space
    are exact, the others report -1 and are not written."""
    import oracle
    import torch
    from paper_2103_11991_amd.spgemm import DeviceCsr, SpGEMMBatch
    prods = _banded_products(24, 11)
    sizes = [int(oracle.row_nnz(A, B).sum()) for A, B in prods]
    cap = sum(sizes) // 2
    batch = SpGEMMBatch([DeviceCsr.from_host(A) for A, _ in prods], [DeviceCsr.from_host(B) for _, B in prods])
    batch.run_queued(cap)
    torch.cuda.synchronize()
    offs = batch.q_offsets.cpu().numpy()
    fitted = [i for i in range(len(prods)) if offs[i] >= 0]
    assert 0 < len(fitted) < len(prods)
    assert sum(sizes[i] for i in fitted) <= cap
    for i in fitted:
        A, B = prods[i]
        rp, c, v = batch.product_queued(i)
        compare(A, B, rp.cpu().numpy(), c.cpu().numpy(), v.cpu().numpy())


def test_queued_batch_refuses_rows_too_wide():
    from paper_2103_11991_amd._lib import SpgError
    from paper_2103_11991_amd.spgemm import DeviceCsr, SpGEMMBatch
    A = gen.random_csr(50, 60, 1, 20, seed=1)
    B = gen.random_csr(60, 9000, 10, 40, seed=2)
    batch = SpGEMMBatch([DeviceCsr.from_host(A)], [DeviceCsr.from_host(B)])
    with pytest.raises(SpgError) as e:
        batch.run_queued(10 ** 6)
    assert e.value.status_name == "SPG_ERR_UNSUPPORTED"
