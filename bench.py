#!/usr/bin/env python3
"""Throughput of the Vietoris-Rips persistence hot path on one MI355X.

One step = one full barcode (distances, threshold, H0, enumeration /
apparent-pair filter, column sort and Z/p reduction in every dimension) of
the so3-1000 workload: 1000 Haar-random rotations of R^3 flattened to R^9,
float32, threshold 1.4, dimensions 0-2, Z/2 (the shape of the paper's o3
data set). The input is resident in HBM before the timed region.

value = simplices/s = (|K_0| + |K_1| + |K_2| + |K_3|) at the threshold, the size
of the explicit filtration the method avoids building, divided by the time
per step. Also reported: the roofline of the dominant kernel (HIP events
over the timed region), and the CPU oracle timed on this host.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


def kernel_bytes(name: str, n: int, m: int, counts, stats, info) -> float | None:
    """Algorithmic HBM bytes of one launch of a kernel class (the data the
    method must move once): candidate records in, surviving records out, the
    distance matrix and neighbour lists read once."""
    sparse = info["sparse"]
    edges = counts[1] if len(counts) > 1 else 0
    nnz = 2 * edges if sparse else 0
    dmat = 4.0 * n * n
    if name == "distances":
        return 4.0 * n * n + 4.0 * n * m
    if name == "edges":
        return dmat + 20.0 * edges
    if name.startswith("filter_d"):
        k = int(name[-1])
        cand = counts[k]
        surv = stats[k]["columns"]
        return 12.0 * cand + 17.0 * surv + dmat + 4.0 * nnz
    if name.startswith("expand_d"):
        k = int(name[-1])
        return 12.0 * counts[k - 1] + 12.0 * counts[k] + dmat + 4.0 * nnz
    if name.startswith("sort_d"):
        k = int(name[-1])
        return 2.0 * 17.0 * stats[k]["columns"]
    if name.startswith("reduce_d"):
        k = int(name[-1])
        return 17.0 * stats[k]["columns"]
    if name == "h0":
        return 20.0 * edges + 24.0 * n
    return None


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="bound on the CPU-oracle sample (seconds)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(batched clouds would shard by clouds across GPUs; see DESIGN.md).",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_1908_02518_amd as rips
    import workloads

    cfg = workloads.config(2)
    x = cfg["clouds"][0]
    n, m = x.shape
    t, p, max_dim = cfg["threshold"], cfg["p"], cfg["max_dim"]
    dev = torch.device("cuda:0")
    xt = torch.from_numpy(x).to(dev)
    torch.cuda.synchronize()

    # size of the explicit filtration (numerator), outside the timed region
    counts = rips.simplex_counts(xt, max_dim + 1, threshold=t)
    n_simplices = int(sum(counts))

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    log(f"workload {cfg['name']}: n={n}, |K_0..K_{max_dim + 1}| = {counts}")
    for i in range(args.warmup):
        c0 = time.perf_counter()
        bars, info = rips.barcode_device(xt, max_dim=max_dim, threshold=t, p=p)
        torch.cuda.synchronize()
        log(f"warmup {i}: {1e3 * (time.perf_counter() - c0):.2f} ms")

    rips.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        bars, info = rips.barcode_device(xt, max_dim=max_dim, threshold=t, p=p)
        if i % 5 == 4:
            log(f"step {i + 1}/{args.steps}")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    log(f"timed: {1e3 * (t1 - t0) / args.steps:.2f} ms/step")
    rips.profile_enable(False)
    prof = rips.profile_read()

    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = n_simplices / ((t1 - t0) / args.steps)
    stats = info["stats"]

    # dominant kernel and its roofline
    dom = max(prof.items(), key=lambda kv: kv[1][0])
    dname, (dms, dcalls) = dom
    per_launch_ms = dms / dcalls
    dbytes = kernel_bytes(dname, n, m, counts, stats, info)
    achieved = (dbytes / (per_launch_ms * 1e-3) / 1e9) if dbytes else None
    roofline = {
        "kernel": dname,
        "bound": "hbm",
        "achieved": round(achieved, 3) if achieved is not None else None,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 6) if achieved is not None else None,
        "traffic": None,
        "bytes_per_launch": dbytes,
        "avg_launch_us": round(per_launch_ms * 1e3, 3),
    }
    # the enumeration / apparent-pair pass of the top dimension, reported beside it
    fname = f"filter_d{max_dim}"
    enum_pass = None
    if fname in prof:
        fms, fc = prof[fname]
        fb = kernel_bytes(fname, n, m, counts, stats, info)
        fa = fb / (fms / fc * 1e-3) / 1e9
        cand = counts[max_dim]
        enum_pass = {"kernel": fname, "achieved_GBs": round(fa, 3),
                     "frac_hbm": round(fa / HBM_PEAK_GBS, 6),
                     "avg_launch_us": round(fms / fc * 1e3, 3),
                     "candidates_per_s": round(cand / (fms / fc * 1e-3), 1)}

    eliminated = {}
    for k in range(1, max_dim + 1):
        s = stats[k]
        c = max(1, s["candidates"])
        eliminated[f"d{k}"] = {
            "candidates": s["candidates"],
            "cleared": s["cleared"], "apparent_col": s["apparent_col"],
            "apparent_pivot": s["apparent_pivot"],
            "fraction_eliminated": round(
                (s["cleared"] + s["apparent_col"] + s["apparent_pivot"]) / c, 6),
            "columns": s["columns"], "emergent": s["emergent"], "reduced": s["reduced"],
            "additions": s["additions"],
        }

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        oracle.build(force=False)
        reps, el = 0, 0.0
        while reps == 0 or el < args.cpu_seconds:
            c0 = time.perf_counter()
            oracle.barcode(x, max_dim=max_dim, threshold=t, p=p)
            el += time.perf_counter() - c0
            reps += 1
            log(f"cpu oracle run {reps}: {el / reps:.2f} s")
            if el > args.cpu_seconds:
                break
        cpu = {"value": round(n_simplices / (el / reps), 1), "unit": "simplices/s", "cores": 1,
               "kind": "oracle",
               "sample": f"the full so3-1000 cloud (same input), {reps} run(s), "
                         f"{el / reps:.3f} s each, single thread"}

    line = {
        "metric": "simplices/s (one barcode of the so3-1000 workload per step)",
        "value": round(value, 1),
        "unit": "simplices/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "so3-1000: 1000 Haar SO(3) rotations in R^9, float32, "
                               "threshold 1.4, dims 0-2, Z/2",
                   "n": n, "dims": max_dim, "threshold": t, "p": p,
                   "simplex_counts": counts},
        "roofline": roofline,
        "enumeration_pass": enum_pass,
        "kernels_ms_per_step": {k: round(v[0] / args.steps, 4) for k, v in sorted(prof.items())},
        "eliminated": eliminated,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))
    return 0


if __name__ == "__main__":
    sys.exit(main())
