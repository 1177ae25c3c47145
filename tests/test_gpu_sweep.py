"""A seeded sweep of products against the oracle: shapes from empty to a few
thousand rows, densities from empty rows to long rows, sorted and unsorted
rows with repeated columns, FP32 and FP64, every binning, forced classes,
list limits that put the product on the two-wait path, and handles that are
reused (new matrices on an old handle) or destroyed and replaced (their
buffers taken over by the next handle).  Each case is small; together they
cover the paths' combinations rather than any one path."""
import numpy as np
import pytest
import torch

from paper_2103_11991_amd import gen
from paper_2103_11991_amd.spgemm import DeviceCsr, SpGEMM
from gpu_util import compare

pytestmark = pytest.mark.gpu


def setup_module(module):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _case(rng):
    m = int(rng.choice([0, 1, 7, 63, 64, 65, 500, 2047, 3000]))
    n = int(rng.choice([1, 33, 300, 5000]))
    k = int(rng.choice([1, 32, 31 * 32 + 5, 4096, 70000]))
    la = int(rng.integers(0, 40))
    lb = int(rng.integers(0, 60))
    dtype = np.float64 if rng.random() < 0.5 else np.float32
    A = gen.random_csr(m, n, 0, la, seed=int(rng.integers(1 << 30)), dtype=dtype,
                       empty_frac=float(rng.choice([0.0, 0.3])), duplicates=bool(rng.random() < 0.3),
                       sorted_rows=bool(rng.random() < 0.7))
    B = gen.random_csr(n, k, 0, lb, seed=int(rng.integers(1 << 30)), dtype=dtype,
                       duplicates=bool(rng.random() < 0.3), sorted_rows=bool(rng.random() < 0.7))
    opts = {}
    r = rng.random()
    if r < 0.2:
        opts["binning"] = 0
    elif r < 0.3:
        opts["force_class"] = int(rng.integers(0, 30))
    elif r < 0.45:
        opts["list_limit_mb"] = 1  # past the one-wait bound for all but tiny products
    elif r < 0.6:
        opts["binning"] = 1  # learned sizes from a random network: overflows and retries
        opts["mlp_margin_milli"] = 0
    return A, B, opts


@pytest.mark.parametrize("block", range(10))
def test_seeded_sweep(block):
    rng = np.random.default_rng(1000 + block)
    keep = None
    for it in range(12):
        A, B, opts = _case(rng)
        dA, dB = DeviceCsr.from_host(A), DeviceCsr.from_host(B)
        op = SpGEMM(dA, dB, **opts)
        if opts.get("binning") == 1:
            w = (rng.standard_normal(1217) * 0.3).astype(np.float32)
            op.set_mlp(w)
        rp, nnz = op.symbolic()
        col, val = op.numeric()
        torch.cuda.synchronize()
        rph = rp.cpu().numpy().astype(np.int64)
        compare(A, B, rph, col.cpu().numpy(), val.cpu().numpy())
        st = op.stats()
        assert st["sym_waits"] in (1, 2)
        if it % 3 == 2:
            keep = op  # some handles live on while later ones are created and dropped
        del op
    del keep


def test_handle_reused_for_new_matrices():
    """One handle, a sequence of set_matrices calls with growing and
    shrinking shapes (buffers grow, stale sizes must not leak into results)."""
    from paper_2103_11991_amd import _lib
    rng = np.random.default_rng(77)
    shapes = [(3000, 400, 5000, 30), (10, 10, 10, 3), (2047, 2000, 70000, 50), (1, 5, 5, 4), (500, 300, 300, 20)]
    op = None
    for m, n, k, ln in shapes:
        A = gen.random_csr(m, n, 0, ln, seed=int(rng.integers(1 << 30)))
        B = gen.random_csr(n, k, 0, ln, seed=int(rng.integers(1 << 30)))
        dA, dB = DeviceCsr.from_host(A), DeviceCsr.from_host(B)
        if op is None:
            op = SpGEMM(dA, dB)
        else:
            op.set_matrices(dA, dB)
        rp, nnz = op.symbolic()
        col, val = op.numeric()
        torch.cuda.synchronize()
        compare(A, B, rp.cpu().numpy().astype(np.int64), col.cpu().numpy(), val.cpu().numpy())
