"""Throughput of the two-phase SpGEMM hot path on one MI355X.

One step = one full product C = A*A through the C ABI: symbolic (row
analysis, binning, row accumulators, row-pointer scan, the nnz(C) read-back)
then numeric (values, sorted columns) into caller-allocated C arrays.  The
workload is the 3D 27-point stencil on a 100^3 grid (1M rows, 26.46M nonzeros,
FP64 values uniform in [-1, 1], diagonal 27), synthetic and seeded.

Printed: one JSON line with GFLOP/s (2 x multiply-adds / step time), C-nnz/s,
the compulsory-byte HBM fraction, a roofline entry for the dominant kernel
(the numeric accumulator class that takes the most time, timed with HIP events
recorded by the library on its own stream) and the CPU oracle timed on a
bounded row sample on the host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "SpGEMM GFLOP/s + C-nnz/s + HBM GB/s fraction; learned/batched vs plain"


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    for f in ("spg_accum.hip", "spg_internal.h"):
        with open(os.path.join(ROOT, "paper_2103_11991_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_traffic(kernel: str):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were
    taken on the current kernel source; otherwise None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as fh:
            d = json.load(fh)
        ent = d.get(kernel)
        if not ent or ent.get("source_sha") != kernel_source_sha():
            return None
        return float(ent["hbm_bytes_per_launch"])
    except Exception:
        return None


def _pmc_rows(d: str):
    import csv
    import glob
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            yield from csv.DictReader(fh)


def summarize_counters(fetch_dir, write_dir, cfetch_dir, cwrite_dir, cls: int, command: str) -> dict:
    """HBM bytes per launch of the dominant numeric kernel from rocprofv3
    FETCH_SIZE and WRITE_SIZE runs (KiB per dispatch), each scaled by what the
    same counter reads for the plain 1 GiB copy of --copy-calibration; writes
    profiles/traffic.json keyed by the class, with the kernel source hash."""
    def per_dispatch(d, counter, want):
        vals = {}
        for r in _pmc_rows(d):
            if r["Counter_Name"] == counter and want(r["Kernel_Name"]):
                vals.setdefault((int(r["Grid_Size"]), r["Dispatch_Id"]), 0.0)
                vals[(int(r["Grid_Size"]), r["Dispatch_Id"])] += float(r["Counter_Value"])
        return vals

    is_num = lambda k: "k_num<" in k
    is_copy = lambda k: "copyBuffer" in k
    out = {}
    for counter, d, cd in (("FETCH_SIZE", fetch_dir, cfetch_dir), ("WRITE_SIZE", write_dir, cwrite_dir)):
        v = per_dispatch(d, counter, is_num)
        grid = max(g for g, _ in v)   # the dominant class launches the largest grid
        kib = [x for (g, _), x in v.items() if g == grid]
        c = [x for (g, _), x in per_dispatch(cd, counter, is_copy).items() if g == max(g2 for g2, _ in per_dispatch(cd, counter, is_copy))]
        factor = (1 << 30) / (1024.0 * float(np.mean(c)))   # true KiB per counted KiB
        out[counter] = {"kib_per_launch": float(np.mean(kib)), "launches": len(kib), "grid": grid,
                        "copy_kib_per_gib": float(np.mean(c)), "scale": round(factor, 4),
                        "bytes_per_launch": float(np.mean(kib)) * 1024.0 * factor}
    ent = {"source_sha": kernel_source_sha(), "hbm_bytes_per_launch":
           out["FETCH_SIZE"]["bytes_per_launch"] + out["WRITE_SIZE"]["bytes_per_launch"],
           "fetch": out["FETCH_SIZE"], "write": out["WRITE_SIZE"], "command": command}
    path = os.path.join(ROOT, "profiles", "traffic.json")
    d = {}
    if os.path.exists(path):
        with open(path) as fh:
            d = json.load(fh)
    d[f"num_class_{cls}"] = ent
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as fh:
        json.dump(d, fh, indent=1)
    return ent


def cpu_baseline(A, target_s: float = 12.0):
    """The oracle (symbolic + numeric) on the same product, timed on the host
    cores: whole-product passes repeated until about target_s seconds (or a
    contiguous row range when one pass would take longer); median pass as
    GFLOP/s."""
    import oracle
    from paper_2103_11991_amd import gen
    ppr = gen.products_per_row(A, A)
    probe = min(A.m, 4096)
    mid = (A.m - probe) // 2
    t0 = time.perf_counter()
    oracle.spgemm(A, A, mid, mid + probe)
    dt = max(time.perf_counter() - t0, 1e-4)
    rows = int(min(A.m, max(probe, probe * target_s / dt)))
    r0 = (A.m - rows) // 2
    times = []
    t_start = time.perf_counter()
    while True:
        t0 = time.perf_counter()
        rp, _, _, _ = oracle.spgemm(A, A, r0, r0 + rows)
        times.append(time.perf_counter() - t0)
        if time.perf_counter() - t_start > target_s or len(times) >= 50:
            break
    dt = float(np.median(times))
    prods = int(ppr[r0:r0 + rows].sum())
    what = "the whole product" if rows == A.m else f"rows {r0}..{r0 + rows - 1} ({rows} rows)"
    cores = oracle.num_threads()
    # one thread, on a row range of about 3 s
    probe1 = min(A.m, 20000)
    s1 = (A.m - probe1) // 2
    oracle.set_num_threads(1)
    try:
        t0 = time.perf_counter()
        oracle.spgemm(A, A, s1, s1 + probe1)
        d1 = max(time.perf_counter() - t0, 1e-4)
        rows1 = int(min(A.m, max(probe1, probe1 * 3.0 / d1)))
        s1 = (A.m - rows1) // 2
        t0 = time.perf_counter()
        oracle.spgemm(A, A, s1, s1 + rows1)
        d1 = time.perf_counter() - t0
    finally:
        oracle.set_num_threads(cores)
    prods1 = int(ppr[s1:s1 + rows1].sum())
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": round(2.0 * prods / dt / 1e9, 4), "unit": "GFLOP/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{what}: {prods} multiply-adds, nnz {int(rp[-1])}, symbolic+numeric, median of "
                      f"{len(times)} passes ({dt:.3f} s each, {sum(times):.1f} s total)",
            "c_nnz_per_s": round(int(rp[-1]) / dt, 1),
            "cpu_model": model,
            "value_1_thread": round(2.0 * prods1 / d1 / 1e9, 4),
            "sample_1_thread": f"rows {s1}..{s1 + rows1 - 1}: {prods1} multiply-adds, one pass ({d1:.2f} s)"}


def time_full_products(op, steps, warmup=0):
    """Wall time per full product over `steps` back-to-back products, during
    which the library times only the numeric class launches (HIP events on its
    stream, summed per class: st_timed), then the medians of the symbolic and
    numeric GPU times over three more products with every stage timed (st).
    Returns (sym_ms, num_ms, wall_ms, st_timed, st)."""
    import torch
    op.set_option("timing", 2)
    for _ in range(warmup):
        op.symbolic()
        op.numeric()
    torch.cuda.synchronize()
    op.set_option("timing", 2)  # the sums cover the timed products only
    t0 = time.perf_counter()
    for _ in range(steps):
        op.symbolic()
        op.numeric()
    torch.cuda.synchronize()
    wall = 1e3 * (time.perf_counter() - t0) / steps
    st_timed = op.stats()
    op.set_option("timing", 1)
    sym, num = [], []
    for _ in range(3):
        op.symbolic()
        op.numeric()
        st = op.stats()
        sym.append(st["sym_ms"])
        num.append(st["num_ms"])
    op.set_option("timing", 0)
    return float(np.median(sym)), float(np.median(num)), wall, st_timed, st


def small_product_latency(steps):
    """C = A*A for the 2D 5-point Laplacian on 64^2 (4096 rows, FP64): the
    latency of one whole product (symbolic with its host synchronisation,
    then numeric) over back-to-back products, and the graph-replayed and
    queued batch forms of the same product as a one-product batch."""
    import torch
    from paper_2103_11991_amd import gen
    from paper_2103_11991_amd.spgemm import DeviceCsr, SpGEMM, SpGEMMBatch
    A = gen.laplace2d_5pt(64)
    dA = DeviceCsr.from_host(A)
    op = SpGEMM(dA, dA)
    rp, nnz = op.symbolic()
    col, val = op.numeric()
    torch.cuda.synchronize()
    reps = max(50, steps * 10)
    t0 = time.perf_counter()
    for _ in range(reps):
        op.symbolic()
        op.numeric(out_col=col, out_val=val)
    torch.cuda.synchronize()
    t_full = 1e3 * (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        op.numeric(out_col=col, out_val=val)
    torch.cuda.synchronize()
    t_num = 1e3 * (time.perf_counter() - t0) / reps
    prods = int(op.stats()["products"])
    batch = SpGEMMBatch([dA], [dA])
    nb = batch.plan()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t = []
        for _ in range(reps):
            ev[0].record(batch.stream)
            fn()
            ev[1].record(batch.stream)
            ev[1].synchronize()
            t.append(ev[0].elapsed_time(ev[1]))
        return float(np.median(t))

    t_graph = timed(lambda: batch.run())
    t_queued = timed(lambda: batch.run_queued(nb))
    return {"workload": "C=A*A, A = 2D 5-point Laplacian on 64^2 (FP64)", "rows": A.m, "nnz_c": int(nnz),
            "multiply_adds": prods, "full_product_ms": round(t_full, 4), "numeric_reuse_ms": round(t_num, 4),
            "one_product_graph_ms": round(t_graph, 4), "one_product_queued_ms": round(t_queued, 4),
            "note": "full product = host-synchronised symbolic (nnz(C) returned) + numeric, wall time per "
                    "back-to-back product; graph / queued: HIP events around one replay"}


def learned_vs_plain(dA, steps, plain):
    """The same product with the symbolic tables sized three ways: the upper
    bound from each row's products, the default upper bound from the
    compressed-B runs it reads (the headline run, ``plain``), and the learned
    row-size predictor (committed model)."""
    from paper_2103_11991_amd import learned
    from paper_2103_11991_amd.spgemm import SpGEMM
    out = {"t_sym_runs_bound_ms": round(plain["sym"], 4), "t_full_runs_bound_ms": round(plain["wall"], 4)}
    op = SpGEMM(dA, dA, timing=1, binning=0)
    for _ in range(2):
        op.symbolic()
        op.numeric()
    sym0, _, wall0, _, st0 = time_full_products(op, steps)
    rows = st0["m"] - st0["empty_rows"]
    out.update({"t_sym_products_bound_ms": round(sym0, 4), "t_full_products_bound_ms": round(wall0, 4),
                "products_bound_mispredict_rate": round(st0["mispredicted_rows"] / max(rows, 1), 5),
                "runs_bound_mispredict_rate": round(plain["mispredicted"] / max(rows, 1), 5)})
    del op
    if not os.path.exists(learned.DEFAULT_MODEL):
        return out
    w, margin, meta = learned.load()
    op = SpGEMM(dA, dA, timing=1, binning=1, mlp_margin_milli=int(round(margin * 1000)))
    op.set_mlp(w)
    for _ in range(2):
        op.symbolic()
        op.numeric()
    sym, num, wall, _, st = time_full_products(op, steps)
    # the ideal estimate: each row's exact occupied blocks (from the run just made)
    opi = SpGEMM(dA, dA, timing=1, binning=2)
    opi.symbolic()
    opi.set_option("binning", 3)
    for _ in range(2):
        opi.symbolic()
        opi.numeric()
    sym_i, _, wall_i, _, _ = time_full_products(opi, steps)
    del opi
    out.update({"t_sym_ideal_ms": round(sym_i, 4), "t_full_ideal_ms": round(wall_i, 4),
                "speedup_sym_ideal_vs_runs_bound": round(plain["sym"] / sym_i, 3)})
    out.update({"t_sym_learned_ms": round(sym, 4), "t_full_learned_ms": round(wall, 4),
                "speedup_sym_vs_products_bound": round(sym0 / sym, 3),
                "speedup_full_vs_products_bound": round(wall0 / wall, 3),
                "speedup_sym_vs_runs_bound": round(plain["sym"] / sym, 3),
                "speedup_full_vs_runs_bound": round(plain["wall"] / wall, 3),
                "retry_rate": round(st["retried_rows"] / max(rows, 1), 5),
                "mispredict_rate": round(st["mispredicted_rows"] / max(rows, 1), 5),
                "mlp_ms": round(st["mlp_ms"], 4), "model_rows": meta.get("rows"),
                "model_quantile": meta.get("quantile"), "margin_log2": round(margin, 3)})
    return out


def _learned_opts():
    from paper_2103_11991_amd import learned
    if not os.path.exists(learned.DEFAULT_MODEL):
        return None, None
    w, margin, _ = learned.load()
    return w, {"binning": 1, "mlp_margin_milli": int(round(margin * 1000))}


def rmat_learned_vs_plain(steps, scale=18, seeds=(1, 2, 3)):
    """R-MAT scale 18 (FP32) A*A with the products bound, the compressed-run
    bound, learned binning and the ideal estimate (each row's exact count),
    on each test seed; the per-seed figures and their mean."""
    import torch
    from paper_2103_11991_amd import gen
    from paper_2103_11991_amd.spgemm import DeviceCsr, SpGEMM
    out = {"workload": f"C=A*A, A = R-MAT scale {scale} edge factor 16 (a=0.57, b=c=0.19), FP32, test seeds {list(seeds)}"}
    w, lopts = _learned_opts()
    per_seed = []
    for seed in seeds:
        A = gen.rmat(scale, seed=seed)
        dA = DeviceCsr.from_host(A)
        ent = {"seed": seed, "rows": A.m, "nnz_a": A.nnz}
        for label, opts in (("products_bound", {"binning": 0}), ("runs_bound", {"binning": 2}), ("learned", lopts),
                            ("ideal", {"binning": 2, "ideal": 1})):
            if opts is None:
                ent[label] = None
                continue
            opts = dict(opts)
            ideal = opts.pop("ideal", 0)
            op = SpGEMM(dA, dA, timing=1, **opts)
            if opts.get("binning") == 1:
                op.set_mlp(w)
            op.symbolic()
            if ideal:
                op.set_option("binning", 3)
            for _ in range(2):
                op.symbolic()
                op.numeric()
            sym, num, wall, st_t, st = time_full_products(op, steps)
            rows = st["m"] - st["empty_rows"]
            rows_c = st["sym_rows"]
            lds_mb = sum(rows_c[c] * (256 << (c % 10)) for c in range(30) if c % 10 != 9) / 2 ** 20
            ent[label] = {"t_sym_ms": round(sym, 3), "t_num_ms": round(num, 3), "t_full_ms": round(wall, 3),
                          "sym_table_bytes_summed_over_rows_mib": round(lds_mb, 2),
                          "sym_rows_per_class": {c: rows_c[c] for c in range(30) if rows_c[c]},
                          "gflops": round(2.0 * st["products"] / (wall * 1e-3) / 1e9, 2),
                          "c_nnz_per_s": round(st["nnz_c"] / (wall * 1e-3), 1),
                          "retry_rate": round(st["retried_rows"] / max(rows, 1), 5),
                          "mispredict_rate": round(st["mispredicted_rows"] / max(rows, 1), 5)}
            if label == "runs_bound":
                # the dominant numeric launch (the global class: tile build,
                # tiled kernel and segment-path rest) against HBM, priced with
                # FP32 values: 8 B per A entry of its rows, per C entry it
                # writes and per B entry (its share of products), 12 B per row
                dom = {c: st_t["num_class_ms_total"][c] / st_t["num_class_launches"][c]
                       for c in range(30) if st_t["num_class_launches"][c]}
                dc = max(dom, key=lambda c: dom[c])
                alg = (st["num_a_nnz"][dc] * 8 + st["num_c_nnz"][dc] * 8
                       + st["num_products"][dc] / max(st["products"], 1) * A.nnz * 8 + st["num_rows"][dc] * 12)
                ach = alg / (dom[dc] * 1e-3) / 1e9
                ent[label]["roofline"] = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                                          "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                                          "kernel": f"numeric class {dc}", "launch_ms": round(dom[dc], 3),
                                          "algorithmic_bytes": int(alg), "products_share": round(
                                              st["num_products"][dc] / max(st["products"], 1), 4)}
            ent["multiply_adds"] = int(st["products"])
            ent["nnz_c"] = int(st["nnz_c"])
            del op
            torch.cuda.synchronize()
        per_seed.append(ent)
        del dA
        torch.cuda.synchronize()
    out["seeds"] = per_seed
    labels = [k for k in ("products_bound", "runs_bound", "learned", "ideal") if all(e.get(k) for e in per_seed)]
    mean = {k: {f: round(float(np.mean([e[k][f] for e in per_seed])), 4)
                for f in ("t_sym_ms", "t_num_ms", "t_full_ms", "gflops", "retry_rate", "mispredict_rate")}
            for k in labels}
    out["mean"] = mean
    if "learned" in mean:
        for ref in ("products_bound", "runs_bound"):
            out[f"learned_speedup_full_vs_{ref}"] = round(mean[ref]["t_full_ms"] / mean["learned"]["t_full_ms"], 3)
            out[f"learned_speedup_sym_vs_{ref}"] = round(mean[ref]["t_sym_ms"] / mean["learned"]["t_sym_ms"], 3)
    if "ideal" in mean:
        out["ideal_speedup_sym_vs_runs_bound"] = round(mean["runs_bound"]["t_sym_ms"] / mean["ideal"]["t_sym_ms"], 3)
    return out


def galerkin_chain(sweeps=10, n0=128, levels=5):
    """R*(A*P) over 5 aggregation levels from a 7-point Laplacian on 128^3:
    the whole chain with both phases, then `sweeps` numeric-only passes with
    changed fine-level values (symbolic reused), for the products bound, the
    compressed-run bound and learned binning."""
    import torch
    from paper_2103_11991_amd import gen
    from paper_2103_11991_amd.spgemm import DeviceCsr, SpGEMM
    A0 = gen.laplace3d_7pt(n0)
    hier = [(N, DeviceCsr.from_host(P), DeviceCsr.from_host(R)) for N, P, R in gen.galerkin_hierarchy(n0, levels)]
    sweep_vals = [torch.from_numpy(gen.sweep_values(A0, t)).cuda() for t in range(1, sweeps + 1)]
    out = {"workload": f"Galerkin R*(A*P), 7-point Laplacian {n0}^3, 2x2x2 aggregation, {levels} levels, FP64, "
                       f"{sweeps} changed-value numeric sweeps"}
    w, lopts = _learned_opts()
    for label, opts in (("products_bound", {"binning": 0}), ("runs_bound", {"binning": 2}), ("learned", lopts)):
        if opts is None:
            out[label] = None
            continue
        times, ops = [], None
        for rep in range(3):
            dA = DeviceCsr.from_host(A0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            cur, ops, products = dA, [], 0
            for N, dP, dR in hier:
                for X, Y in ((None, dP), (dR, None)):
                    left, right = (cur, Y) if X is None else (X, cur)
                    op = SpGEMM(left, right, **opts)
                    if opts.get("binning") == 1:
                        op.set_mlp(w)
                    rp, nnz = op.symbolic()
                    col, val = op.numeric()
                    nxt = DeviceCsr(left.m, right.n, rp, col, val)
                    ops.append((op, left, right, nxt))
                    products += op.stats()["products"]
                    cur = nxt
            torch.cuda.synchronize()
            times.append(1e3 * (time.perf_counter() - t0))
        # numeric sweeps: new fine-level values flow through the whole chain
        t0 = time.perf_counter()
        for sv in sweep_vals:
            ops[0][1].values.copy_(sv)
            for op, left, right, nxt in ops:
                op.numeric(a_vals=left.values, b_vals=right.values, out_col=nxt.col_idx, out_val=nxt.values)
        torch.cuda.synchronize()
        t_sweeps = 1e3 * (time.perf_counter() - t0)
        out[label] = {"t_chain_full_ms": round(float(np.median(times)), 3),
                      "t_sweep_numeric_ms": round(t_sweeps / sweeps, 3),
                      "reuse_speedup": round(float(np.median(times)) / (t_sweeps / sweeps), 2),
                      "products": 2 * len(hier)}
        out["multiply_adds"] = int(products)
        del ops
        torch.cuda.synchronize()
    if out.get("learned"):
        for ref in ("products_bound", "runs_bound"):
            out[f"learned_speedup_chain_vs_{ref}"] = round(
                out[ref]["t_chain_full_ms"] / out["learned"]["t_chain_full_ms"], 3)
    return out


def single_leg(name, steps, warmup):
    """One workload alone, for a profiler run: `steps` timed repetitions
    after `warmup` untimed ones."""
    import torch
    from paper_2103_11991_amd import gen
    from paper_2103_11991_amd.spgemm import DeviceCsr, SpGEMM, SpGEMMBatch
    if name == "rmat":
        A = gen.rmat(18, seed=1)
        dA = DeviceCsr.from_host(A)
        op = SpGEMM(dA, dA)
        for _ in range(warmup):
            op.symbolic()
            op.numeric()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            op.symbolic()
            op.numeric()
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / max(steps, 1)
        return {"leg": "C=A*A, A = R-MAT scale 18 seed 1 (FP32), plain two-phase", "steps": steps,
                "ms_per_product": round(ms, 3), "nnz_c": int(op.nnz)}
    pools = gen.banded_batch_pools(1024)
    dev = {k: torch.from_numpy(v).cuda() for k, v in pools.items() if k not in ("n", "a_nnz", "b_nnz")}
    n = pools["n"]
    batch = SpGEMMBatch.from_pools(n, n, n, pools["a_nnz"], pools["b_nnz"], dev["a_rp"], dev["a_ci"], dev["a_v"],
                                   dev["b_rp"], dev["b_ci"], dev["b_v"])
    cap = int(batch.plan())
    run = (lambda: batch.run_queued(cap)) if name == "queued" else batch.run
    for _ in range(warmup):
        run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        run()
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / max(steps, 1)
    return {"leg": f"1024 banded products (seed 12345), {'queued persistent kernel' if name == 'queued' else 'graph'}",
            "steps": steps, "ms_per_batch": round(ms, 3)}


def batched_vs_loop(count, steps):
    """The banded batch: one graph launch (autotuned) against a loop of plain
    two-phase products, each with its own handle."""
    import torch
    from paper_2103_11991_amd import gen
    from paper_2103_11991_amd.spgemm import DeviceCsr, SpGEMM, SpGEMMBatch
    t0 = time.perf_counter()
    pools = gen.banded_batch_pools(count)
    gen_s = time.perf_counter() - t0
    dev = {k: torch.from_numpy(v).cuda() for k, v in pools.items() if k not in ("n", "a_nnz", "b_nnz")}
    n = pools["n"]
    batch = SpGEMMBatch.from_pools(n, n, n, pools["a_nnz"], pools["b_nnz"], dev["a_rp"], dev["a_ci"], dev["a_v"],
                                   dev["b_rp"], dev["b_ci"], dev["b_v"])
    batch.plan()
    chosen, tuned_ms = batch.tune()
    for _ in range(2):
        batch.run()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    times = []
    for _ in range(steps):
        ev[0].record(batch.stream)
        batch.run()
        ev[1].record(batch.stream)
        ev[1].synchronize()
        times.append(ev[0].elapsed_time(ev[1]))
    t_batch = float(np.median(times))
    numeric_times = []
    for _ in range(steps):
        ev[0].record(batch.stream)
        batch.run(numeric_only=True)
        ev[1].record(batch.stream)
        ev[1].synchronize()
        numeric_times.append(ev[0].elapsed_time(ev[1]))
    # the persistent queued kernel: both phases of every product, C space from
    # the device bump allocator, per-product device time stamps (100 MHz clock)
    batch.run_queued(int(batch.nnz))
    torch.cuda.synchronize()
    q_times, spans, from_launch = [], [], []
    for _ in range(steps):
        ev[0].record(batch.stream)
        batch.run_queued(int(batch.nnz))
        ev[1].record(batch.stream)
        ev[1].synchronize()
        q_times.append(ev[0].elapsed_time(ev[1]))
        st_ = batch.q_stamps.cpu().numpy().reshape(-1, 2).astype(np.float64)
        busy = st_[:, 1] > 0
        spans.append((st_[busy, 1] - st_[busy, 0]) / 1e5)
        from_launch.append((st_[busy, 1] - st_[busy, 0].min()) / 1e5)
    q_ok = bool((batch.q_offsets.cpu().numpy() >= 0).all())
    t_queued = float(np.median(q_times))
    spans = np.concatenate(spans)
    from_launch = np.concatenate(from_launch)
    st = batch.stats()
    products = st["products"]
    # loop of plain launches: every product symbolic + numeric + synchronise
    pairs = gen.pools_to_pairs(pools)
    ops = []
    for A, B in pairs:
        dA, dB = DeviceCsr.from_host(A), DeviceCsr.from_host(B)
        ops.append((SpGEMM(dA, dB), dA, dB))
    outs = []
    for op, _, _ in ops:  # warm-up pass that also allocates every C once
        op.symbolic()
        outs.append(op.numeric())
    torch.cuda.synchronize()
    lat = []
    t0 = time.perf_counter()
    for (op, _, _), (col, val) in zip(ops, outs):
        t1 = time.perf_counter()
        op.symbolic()
        op.numeric(out_col=col, out_val=val)
        torch.cuda.synchronize()
        lat.append(1e3 * (time.perf_counter() - t1))
    t_loop = 1e3 * (time.perf_counter() - t0)
    return {"products": count, "rows": int(n.sum()), "multiply_adds": int(products), "nnz_c": int(batch.nnz),
            "batched_ms": round(t_batch, 3), "batched_numeric_only_ms": round(float(np.median(numeric_times)), 3),
            "loop_ms": round(t_loop, 3),
            "batched_gflops": round(2.0 * products / (t_batch * 1e-3) / 1e9, 2),
            "loop_gflops": round(2.0 * products / (t_loop * 1e-3) / 1e9, 2),
            "speedup": round(t_loop / t_batch, 2),
            "loop_latency_p50_ms": round(float(np.percentile(lat, 50)), 4),
            "loop_latency_p99_ms": round(float(np.percentile(lat, 99)), 4),
            "batched_latency_ms": round(t_batch, 3),
            "batched_latency_note": "all products complete with the single graph launch: each product's "
                                    "latency from launch is the batch time",
            "queued_ms": round(t_queued, 3),
            "queued_gflops": round(2.0 * products / (t_queued * 1e-3) / 1e9, 2),
            "queued_speedup_vs_graph": round(t_batch / t_queued, 3),
            "queued_speedup_vs_loop": round(t_loop / t_queued, 2),
            "queued_all_fitted": q_ok,
            "queued_product_span_p50_ms": round(float(np.percentile(spans, 50)), 4),
            "queued_product_span_p99_ms": round(float(np.percentile(spans, 99)), 4),
            "queued_product_done_from_first_start_p50_ms": round(float(np.percentile(from_launch, 50)), 4),
            "queued_product_done_from_first_start_p99_ms": round(float(np.percentile(from_launch, 99)), 4),
            "queued_latency_note": "device clock per product: span = first work item start to last work item "
                                   "end; done-from-first-start = last item end minus the earliest item start "
                                   "of the run",
            "autotuned": {"work_per_lane": chosen[0], "binning": chosen[1], "hash_max_blocks": chosen[2],
                          "best_full_run_ms": round(tuned_ms, 3)},
            "generation_s": round(gen_s, 1)}


def jacobi_fused_vs_unfused(steps, n0=128, omega=2.0 / 3.0):
    """Prolongator smoothing C = (I - omega D^-1 A) P: A the 7-point Laplacian
    on n0^3 (FP64), P the 2x2x2 aggregation, D^-1 = 1/6.  Fused: one
    Jacobi-fused numeric call on the symbolic result of A*P.  Unfused (the
    three kernels of the paper's comparison): E = A*P, F = D^-1 E (row scaling
    of E's values), C = P - omega F (sparse addition)."""
    import torch
    from paper_2103_11991_amd import gen
    from paper_2103_11991_amd.spgemm import DeviceCsr, SpAdd, SpGEMM
    A = gen.laplace3d_7pt(n0)
    P = gen.aggregation_P(n0)
    dA, dP = DeviceCsr.from_host(A), DeviceCsr.from_host(P)
    dinv = torch.full((A.m,), 1.0 / 6.0, dtype=torch.float64, device="cuda")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        t = []
        for _ in range(reps):
            ev[0].record()
            fn()
            ev[1].record()
            ev[1].synchronize()
            t.append(ev[0].elapsed_time(ev[1]))
        return float(np.median(t))

    op = SpGEMM(dA, dP)
    rp, nnz = op.symbolic()
    col, val = op.numeric_jacobi(omega, dinv)

    def fused_full():
        op.symbolic()
        op.numeric_jacobi(omega, dinv, out_col=col, out_val=val)

    t_fused_num = timed(lambda: op.numeric_jacobi(omega, dinv, out_col=col, out_val=val), steps)
    t_fused_full = timed(fused_full, steps)
    # unfused: SpGEMM, row scaling, addition
    opE = SpGEMM(dA, dP)
    rpE, nnzE = opE.symbolic()
    colE, valE = opE.numeric()
    rowsE = torch.repeat_interleave(torch.arange(A.m, device="cuda"), torch.diff(rpE.long()))
    F = DeviceCsr(A.m, P.n, rpE, colE, valE.clone())
    add = SpAdd(dP, F)
    add.symbolic()
    colC, valC = add.numeric(1.0, -omega)

    def unfused_num():
        opE.numeric(out_col=colE, out_val=valE)
        torch.mul(valE, dinv[rowsE], out=F.values)
        add.numeric(1.0, -omega, out_col=colC, out_val=valC)

    def unfused_full():
        opE.symbolic()
        opE.numeric(out_col=colE, out_val=valE)
        torch.mul(valE, dinv[rowsE], out=F.values)
        add.symbolic()
        add.numeric(1.0, -omega, out_col=colC, out_val=valC)

    t_unf_num = timed(unfused_num, steps)
    t_unf_full = timed(unfused_full, steps)
    torch.cuda.synchronize()
    same = bool(torch.equal(col, colC)) and float((val - valC).abs().max()) <= 1e-12 * 2
    return {"workload": f"C = (I - {omega:.4g} D^-1 A) P, A = 7-point Laplacian {n0}^3 (FP64), P = 2x2x2 "
                        f"aggregation ({P.n} columns), D^-1 = 1/6",
            "rows": A.m, "nnz_c": int(nnz), "multiply_adds": int(op.stats()["products"]),
            "fused_numeric_ms": round(t_fused_num, 4), "fused_full_ms": round(t_fused_full, 4),
            "unfused_numeric_ms": round(t_unf_num, 4), "unfused_full_ms": round(t_unf_full, 4),
            "speedup_numeric": round(t_unf_num / t_fused_num, 3), "speedup_full": round(t_unf_full / t_fused_full, 3),
            "unfused_kernels": "SpGEMM (this library), row scaling (torch elementwise), SpAdd (this library)",
            "same_result": same}


def spadd_bench(steps, m=1 << 20, per_row=30):
    """C = A + B for square m x m matrices with `per_row` random columns per
    row (the paper's SpAdd input), sorted and unsorted rows, FP64: symbolic and
    numeric times, and the numeric phase's compulsory-byte bandwidth."""
    import torch
    from paper_2103_11991_amd import gen
    from paper_2103_11991_amd.spgemm import DeviceCsr, SpAdd
    out = {"workload": f"C = A + B, {m} x {m}, {per_row} random columns per row of A and of B, FP64"}
    for label, srt in (("sorted", True), ("unsorted", False)):
        A = gen.random_csr(m, m, per_row, per_row, seed=21, sorted_rows=srt)
        B = gen.random_csr(m, m, per_row, per_row, seed=22, sorted_rows=srt)
        add = SpAdd(DeviceCsr.from_host(A), DeviceCsr.from_host(B))
        rp, nnz = add.symbolic()
        col, val = add.numeric(1.0, 1.0)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ts, tn = [], []
        for _ in range(steps):
            ev[0].record()
            add.symbolic()
            ev[1].record()
            ev[1].synchronize()
            ts.append(ev[0].elapsed_time(ev[1]))
            ev[0].record()
            add.numeric(1.0, 1.0, out_col=col, out_val=val)
            ev[1].record()
            ev[1].synchronize()
            tn.append(ev[0].elapsed_time(ev[1]))
        sym, num = float(np.median(ts)), float(np.median(tn))
        # numeric compulsory bytes: A and B structure, values and positions read, C columns and values written
        nbytes = (A.nnz + B.nnz) * (4 + 8 + 4) + 2 * (m + 1) * 4 * 2 + (m + 1) * 4 + int(nnz) * 12
        out[label] = {"nnz_c": int(nnz), "symbolic_ms": round(sym, 4), "numeric_ms": round(num, 4),
                      "numeric_gbs": round(nbytes / (num * 1e-3) / 1e9, 1),
                      "numeric_hbm_frac": round(nbytes / (num * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    return out


def paper_method_ablation(steps):
    """The paper's design (one method for the whole matrix, two-level hash
    maps whose global level a row uses once its LDS level fills;
    SPG_OPT_METHOD 2 = a 16-lane group per row, 3 = a 256-lane team per row,
    1 = picked from the products per row) against this library's per-row
    classes (method 0) on the same products: full product (symbolic +
    numeric) and numeric alone, median over `steps` after one warm-up (one
    timed run for the paper's design on R-MAT, which takes seconds).  The
    paper's numeric leaves rows in hash order; ours emits them sorted."""
    import torch
    from paper_2103_11991_amd import gen
    from paper_2103_11991_amd.spgemm import DeviceCsr, SpGEMM
    cases = [("2D 5-point 64^2 A*A (FP64)", lambda: (gen.laplace2d_5pt(64),) * 2, steps),
             ("3D 27-point 100^3 A*A (FP64)", lambda: (gen.stencil27(100, seed=2),) * 2, steps),
             ("R-MAT scale 18 A*A (FP32, seed 1)", lambda: (gen.rmat(18, seed=1),) * 2, 1),
             ("7-point 128^3 A*P, 2x2x2 aggregation (FP64)", lambda: (gen.laplace3d_7pt(128), gen.aggregation_P(128)),
              steps)]
    out = {}
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    for name, make, paper_steps in cases:
        A, B = make()
        dA = DeviceCsr.from_host(A)
        dB = dA if B is A else DeviceCsr.from_host(B)
        rows = int((gen.products_per_row(A, B) > 0).sum())
        ent = {}
        for label, method, reps in (("classes", 0, steps), ("paper_group", 2, paper_steps),
                                    ("paper_team", 3, paper_steps)):
            op = SpGEMM(dA, dB, method=method)
            op.symbolic()
            col, val = op.numeric()
            torch.cuda.synchronize()
            full, num = [], []
            for _ in range(reps):
                ev[0].record()
                op.symbolic()
                op.numeric(out_col=col, out_val=val)
                ev[1].record()
                ev[1].synchronize()
                full.append(ev[0].elapsed_time(ev[1]))
                ev[0].record()
                op.numeric(out_col=col, out_val=val)
                ev[1].record()
                ev[1].synchronize()
                num.append(ev[0].elapsed_time(ev[1]))
            ent[label] = {"full_ms": round(float(np.median(full)), 4), "numeric_ms": round(float(np.median(num)), 4)}
            if label == "classes":
                ent["products_per_row"] = round(op.stats()["products"] / max(rows, 1), 1)
            del op, col, val
            torch.cuda.synchronize()
        auto = "paper_team" if ent["products_per_row"] >= 256 else "paper_group"
        ent["paper_auto"] = auto
        for lab in ("paper_group", "paper_team"):
            ent[f"{lab}_slowdown_full"] = round(ent[lab]["full_ms"] / ent["classes"]["full_ms"], 3)
        out[name] = ent
        del dA, dB
        torch.cuda.synchronize()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--grid", type=int, default=100, help="stencil grid edge (100 = the 1M-row workload)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--verbose", action="store_true", help="per-class rows and times on stderr")
    ap.add_argument("--batch", type=int, default=1024, help="products in the batched comparison (0 = skip)")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-binning comparison")
    ap.add_argument("--no-rmat", action="store_true", help="skip the R-MAT plain/learned comparison")
    ap.add_argument("--no-galerkin", action="store_true", help="skip the Galerkin chain")
    ap.add_argument("--no-jacobi", action="store_true", help="skip the Jacobi-fused vs unfused comparison")
    ap.add_argument("--no-spadd", action="store_true", help="skip the sparse-addition leg")
    ap.add_argument("--no-ablation", action="store_true", help="skip the paper-design ablation")
    ap.add_argument("--no-small", action="store_true", help="skip the 2D 5-point 64^2 latency leg")
    ap.add_argument("--leg", choices=("rmat", "queued", "graph"), default=None,
                    help="run only one workload (for profiling): R-MAT scale 18 seed 1 plain products, or the "
                         "1024-product banded batch through the queued kernel or its graph; prints its own line")
    ap.add_argument("--opt", action="append", default=[], metavar="NAME=VALUE",
                    help="library option for the timed product (e.g. work_per_lane=32); repeatable")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy 5 times (HBM counter calibration) and exit")
    ap.add_argument("--counters", nargs=4, metavar=("FETCH", "WRITE", "COPY_FETCH", "COPY_WRITE"),
                    help="rocprofv3 output folders of FETCH_SIZE and WRITE_SIZE runs of this bench and of "
                         "--copy-calibration: write profiles/traffic.json for --counters-class and exit (no GPU)")
    ap.add_argument("--counters-class", type=int, default=23)
    ap.add_argument("--counters-command", default="", help="the rocprofv3 command recorded beside the figures")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(1)
    if args.counters:
        ent = summarize_counters(*args.counters, cls=args.counters_class, command=args.counters_command)
        print(json.dumps(ent), flush=True)
        return

    import torch
    from paper_2103_11991_amd import gen
    from paper_2103_11991_amd.spgemm import DeviceCsr, SpGEMM

    torch.cuda.set_device(0)
    if args.leg:
        print(json.dumps(single_leg(args.leg, args.steps, args.warmup)), flush=True)
        return
    if args.copy_calibration:
        # a plain copy of known size: 2^27 doubles read and written (1 GiB each way)
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": src.numel() * 8, "launches": 5}), flush=True)
        return
    N = args.grid
    A = gen.stencil27(N, seed=2)
    products = int(gen.products_per_row(A, A).sum())
    dA = DeviceCsr.from_host(A)
    opts = dict(kv.split("=", 1) for kv in args.opt)
    op = SpGEMM(dA, dA, **{k: int(v) for k, v in opts.items()})
    # the timed region: args.steps back-to-back products (symbolic, then
    # numeric), bracketed by device synchronisation; the numeric class
    # launches carry HIP events on the library's stream throughout
    sym_med, num_med, ms_step, st_t, st = time_full_products(op, args.steps, args.warmup)
    nnz = op.nnz
    dom = {c: st_t["num_class_ms_total"][c] / st_t["num_class_launches"][c]
           for c in range(len(st_t["num_class_launches"])) if st_t["num_class_launches"][c]}

    # numeric alone (symbolic reused), the repeated-product path
    col, val = op.numeric()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        op.numeric(out_col=col, out_val=val)
    torch.cuda.synchronize()
    ms_num_only = 1e3 * (time.perf_counter() - t0) / args.steps

    st = op.stats()
    nnz_a = A.nnz
    eb = 8
    # compulsory bytes of one full product: A and B structure + values read
    # once, C written once, row pointers and per-row bookkeeping
    comp = (nnz_a * (4 + eb)) * 2 + nnz * (4 + eb) + (A.m + 1) * 4 * 3 + A.m * 4 * 4
    gflops = 2.0 * products / (ms_step * 1e-3) / 1e9

    dcls = max(dom, key=lambda c: dom[c])
    dom_ms = float(dom[dcls])
    rows_c = st["num_rows"][dcls]
    frac_prod = st["num_products"][dcls] / max(st["products"], 1)
    alg_bytes = (st["num_a_nnz"][dcls] * (4 + eb) + st["num_c_nnz"][dcls] * (4 + eb)
                 + frac_prod * A.nnz * (4 + eb) + rows_c * 12)
    achieved = alg_bytes / (dom_ms * 1e-3) / 1e9
    kname = f"numeric class {dcls} (mode {('direct', 'hashed', 'two-level')[dcls // 10]}, tier {dcls % 10})"
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": stored_traffic(f"num_class_{dcls}"),
            "kernel": kname, "launch_ms": round(dom_ms, 4), "launches_averaged": int(st_t["num_class_launches"][dcls]),
            "algorithmic_bytes": int(alg_bytes)}

    out = {
        "metric": METRIC, "value": round(gflops, 2), "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"C=A*A, A = 3D 27-point stencil on {N}^3 (FP64 U[-1,1], diagonal 27), "
                               "plain two-phase (upper-bound binning from compressed-B runs)",
                   "rows": A.m, "nnz_a": nnz_a, "nnz_c": int(nnz), "multiply_adds": products,
                   **({"options": opts} if opts else {})},
        "c_nnz_per_s": round(nnz / (ms_step * 1e-3), 1),
        "hbm_frac_compulsory": round(comp / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "t_sym_ms": round(sym_med, 4), "t_num_ms": round(num_med, 4),
        "t_num_reuse_ms": round(ms_num_only, 4),
        "gflops_numeric_reuse": round(2.0 * products / (ms_num_only * 1e-3) / 1e9, 2),
        "roofline": roof,
    }
    if args.verbose:
        detail = {"sym_rows": {c: st["sym_rows"][c] for c in range(len(st["sym_rows"])) if st["sym_rows"][c]},
                  "sym_class_ms": {c: round(st["sym_class_ms"][c], 4) for c in range(len(st["sym_rows"])) if st["sym_rows"][c]},
                  "num_rows": {c: st["num_rows"][c] for c in range(len(st["num_rows"])) if st["num_rows"][c]},
                  "num_class_ms": {c: round(st["num_class_ms"][c], 4) for c in range(len(st["num_rows"])) if st["num_rows"][c]},
                  "analysis_ms": st["analysis_ms"], "scan_ms": st["scan_ms"], "sym_ms": st["sym_ms"],
                  "num_ms": st["num_ms"]}
        print(json.dumps(detail), file=sys.stderr, flush=True)
    plain = {"sym": out["t_sym_ms"], "wall": ms_step, "mispredicted": st["mispredicted_rows"]}
    if not args.no_small:
        out["laplace2d_64"] = small_product_latency(args.steps)
    if not args.no_learned:
        out["learned_vs_plain"] = learned_vs_plain(dA, args.steps, plain)
    if args.batch > 0:
        out["batched_vs_loop"] = batched_vs_loop(args.batch, max(3, args.steps // 2))
    if not args.no_rmat:
        out["rmat_s18"] = rmat_learned_vs_plain(max(3, args.steps // 2))
    if not args.no_galerkin:
        out["galerkin"] = galerkin_chain()
    if not args.no_jacobi:
        out["jacobi_fused_vs_unfused"] = jacobi_fused_vs_unfused(max(3, args.steps // 2))
    if not args.no_spadd:
        out["spadd"] = spadd_bench(max(3, args.steps // 2))
    if not args.no_ablation:
        out["paper_design_ablation"] = paper_method_ablation(3)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(A)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
