"""Learned row-size predictor: data collection, GPU training, calibration, files.

Host orchestration only.  The features and targets come from the library's
symbolic phase (spg_export_rows), training runs in the library's own forward,
backward and Adam kernels (spg_mlp_train), and inference runs inside
spg_symbolic when learned binning is on.

Target: log2(1 + occupied 32-column blocks of a row of C), the quantity that
sizes a row's hashed accumulator.  The network is trained on the pinball loss
at a high quantile, so its output is an upper estimate; a margin calibrated on
the training rows adds the remaining slack.  A row whose table still
overflows is redone exactly (the retry path), so the prediction only affects
speed, never the product.
"""
from __future__ import annotations

import json
import os

import numpy as np

from . import _lib, gen

NW = 1217
MODEL_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "models")
DEFAULT_MODEL = os.path.join(MODEL_DIR, "rowsize_mlp.json")
# rows retried when 1 + blocks exceeds 1.5 x (1 + estimate): the table holds
# at least 2 x estimate slots and overflows above three-quarter occupancy
OVERFLOW_LOG2_SLACK = float(np.log2(1.5))


def init_weights(seed: int = 0) -> np.ndarray:
    """He-normal weights from counter-based draws, zero biases."""
    w = np.zeros(NW, dtype=np.float64)
    z = gen.normal(seed, gen.S_VALUES, np.arange(NW, dtype=np.uint64))
    w[0:96] = z[0:96] * np.sqrt(2.0 / 3.0)
    w[128:1152] = z[128:1152] * np.sqrt(2.0 / 32.0)
    w[1184:1216] = z[1184:1216] * np.sqrt(2.0 / 32.0)
    return w.astype(np.float32)


def collect_rows(pairs):
    """Features and targets of every non-empty row of each product A*B.

    ``pairs``: iterable of (A, B) host CSR pairs.  Returns GPU tensors
    x [N, 3] and y [N] (float32)."""
    import torch
    from .spgemm import DeviceCsr, SpGEMM
    xs, ys = [], []
    for A, B in pairs:
        dA = DeviceCsr.from_host(A)
        dB = dA if B is A else DeviceCsr.from_host(B)
        op = SpGEMM(dA, dB, keep_features=1)
        op.symbolic()
        x, y, _ = op.export_rows()
        keep = x[:, 1] > 0
        xs.append(x[keep])
        ys.append(y[keep])
        del op
    return torch.cat(xs), torch.cat(ys)


def shuffle(x, y, seed: int = 0):
    import torch
    key = gen.u64(seed, gen.S_PERM, np.arange(x.shape[0], dtype=np.uint64))
    perm = torch.from_numpy(np.argsort(key, kind="stable")).to(x.device)
    return x[perm].contiguous(), y[perm].contiguous()


def train(x, y, epochs: int = 6, batch: int = 4096, lr: float = 3e-3, quantile: float = 0.95, seed: int = 0,
          w0: np.ndarray | None = None):
    """Trains on the GPU; returns (weights float32[1217], loss per epoch)."""
    import torch
    w = torch.from_numpy(init_weights(seed) if w0 is None else np.asarray(w0, dtype=np.float32)).cuda()
    losses = torch.zeros(max(epochs, 1), dtype=torch.float32, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    _lib.spg_mlp_train(s, x.data_ptr(), y.data_ptr(), int(x.shape[0]), epochs, batch, lr, quantile, w.data_ptr(),
                       losses.data_ptr())
    torch.cuda.synchronize()
    return w.cpu().numpy(), losses.cpu().numpy()[:epochs]


def predict(w: np.ndarray, x):
    import torch
    dw = torch.from_numpy(np.ascontiguousarray(w, dtype=np.float32)).cuda()
    y = torch.empty(x.shape[0], dtype=torch.float32, device="cuda")
    _lib.spg_mlp_forward(torch.cuda.current_stream().cuda_stream, dw.data_ptr(), x.data_ptr(), int(x.shape[0]),
                         y.data_ptr(), 0)
    torch.cuda.synchronize()
    return y


def calibrate_margin(w: np.ndarray, x, y, target_overflow: float = 0.005) -> float:
    """Smallest margin m >= 0 (log2 units) with at most ``target_overflow`` of the
    rows overflowing: overflow needs y > yhat + m + log2(1.5)."""
    yh = predict(w, x)
    r = (y - yh).cpu().numpy().astype(np.float64)
    need = np.quantile(r, 1.0 - target_overflow) - OVERFLOW_LOG2_SLACK
    return float(max(0.0, need))


def evaluate(w: np.ndarray, margin: float, x, y) -> dict:
    """Predicted vs true occupancy on rows: overflow rate and mean log2 slack."""
    yh = predict(w, x).cpu().numpy().astype(np.float64) + margin
    yt = y.cpu().numpy().astype(np.float64)
    return {"rows": int(yt.size), "overflow_rate": float(np.mean(yt > yh + OVERFLOW_LOG2_SLACK)),
            "mean_slack_log2": float(np.mean(yh - yt)), "median_slack_log2": float(np.median(yh - yt))}


def save(path: str, w: np.ndarray, margin: float, meta: dict) -> None:
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as fh:
        json.dump({"weights": [float(v) for v in np.asarray(w, dtype=np.float32)], "margin_log2": margin,
                   "meta": meta}, fh)


def load(path: str = DEFAULT_MODEL):
    """Returns (weights float32[1217], margin in log2 units, meta)."""
    with open(path) as fh:
        d = json.load(fh)
    w = np.asarray(d["weights"], dtype=np.float32)
    assert w.size == NW
    return w, float(d["margin_log2"]), d.get("meta", {})


def _product_on_gpu(A, B):
    """A*B with the library, copied back as a host CSR (an input for training)."""
    import torch
    from .spgemm import DeviceCsr, spgemm
    C = spgemm(DeviceCsr.from_host(A), DeviceCsr.from_host(B))
    torch.cuda.synchronize()
    return gen.Csr(C.m, C.n, C.row_ptr.cpu().numpy(), C.col_idx.cpu().numpy(), C.values.cpu().numpy())


def training_pairs(scale_max: int = 18):
    """Training products, disjoint from every evaluation input: R-MAT graphs of
    seeds 1001-1016 at scales up to ``scale_max``, 27-point stencils, 7-point
    Galerkin products and banded random products (seed 999)."""
    pairs = []
    for i, seed in enumerate(range(1001, 1017)):
        s = max(12, scale_max - (i % 4))
        A = gen.rmat(s, seed=seed)
        pairs.append((A, A))
    for N in (18, 30, 44):
        S = gen.stencil27(N, seed=7)
        pairs.append((S, S))
    for N in (16, 32, 64):
        L = gen.laplace3d_7pt(N)
        P = gen.aggregation_P(N)
        pairs.append((L, P))
        pairs.append((gen.transpose(P), _product_on_gpu(L, P)))
    for i, (n, bwa, bwb) in enumerate(zip(*gen.batch_sizes(24, seed=999, lo=200, hi=20000))):
        pairs.append((gen.banded_random(int(n), int(bwa), 999, 2 * i),
                      gen.banded_random(int(n), int(bwb), 999, 2 * i + 1)))
    return pairs
