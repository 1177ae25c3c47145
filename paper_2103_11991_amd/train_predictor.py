"""Trains the learned row-size predictor on the GPU and writes it to a file.

    python -m paper_2103_11991_amd.train_predictor [--out PATH] [--scale-max 18]

Rows come from the symbolic phase of the training products (disjoint seeds,
see learned.training_pairs); training, inference and calibration run in the
library's kernels.  The file holds the 1217 weights, the calibrated margin
and a summary of the fit.
"""
from __future__ import annotations

import argparse
import json
import time

from . import learned


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=learned.DEFAULT_MODEL)
    ap.add_argument("--scale-max", type=int, default=18)
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--quantile", type=float, default=0.95)
    ap.add_argument("--target-overflow", type=float, default=0.005)
    args = ap.parse_args()
    t0 = time.time()
    pairs = learned.training_pairs(args.scale_max)
    x, y = learned.collect_rows(pairs)
    x, y = learned.shuffle(x, y, seed=1)
    t1 = time.time()
    w, losses = learned.train(x, y, epochs=args.epochs, batch=args.batch, lr=args.lr, quantile=args.quantile)
    margin = learned.calibrate_margin(w, x, y, args.target_overflow)
    ev = learned.evaluate(w, margin, x, y)
    meta = {"rows": int(x.shape[0]), "products": len(pairs), "epochs": args.epochs, "batch": args.batch,
            "lr": args.lr, "quantile": args.quantile, "target_overflow": args.target_overflow,
            "loss_per_epoch": [float(v) for v in losses], "train_eval": ev,
            "collect_s": round(t1 - t0, 2), "train_s": round(time.time() - t1, 2)}
    learned.save(args.out, w, margin, meta)
    print(json.dumps({"out": args.out, "margin_log2": margin, **meta}), flush=True)


if __name__ == "__main__":
    main()
