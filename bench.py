#!/usr/bin/env python3
"""Throughput of the Vietoris-Rips persistence hot path on one MI355X.

One step = the barcodes of the circles-64x400 batch, the largest of the five
workloads: 64 clouds of 400 points in R^2 (360 on the unit circle with
Gaussian noise 0.1, 40 uniform outliers in [-2, 2]^2), float32, full Rips (the
enclosing radius), dimensions 0-1, Z/2, all in one persistent launch replayed
from a hipGraph (distances, threshold, H0, enumeration / apparent-pair
filter, column sort and Z/p reduction for every cloud). The input is
resident in HBM before the timed region.

value = simplices/s = the sum over the 64 clouds of |K_0| + |K_1| + |K_2| at
each cloud's threshold (the size of the explicit filtrations the method
avoids building) divided by the time per step. Also reported:
  roofline          the dominant kernel (the batched launch): its algorithmic
                    bytes per launch over its mean launch time (HIP events on
                    the stream it runs on), against the HBM peak; traffic =
                    HBM bytes per launch from rocprofv3 FETCH_SIZE /
                    WRITE_SIZE counters (committed summary under profiles/,
                    scaled by a plain copy of known size), null when the
                    kernel sources changed since
  configs           every workload: sphere-100, so3-1000 and torus4-2000 one
                    cloud per call (simplices/s), mixture-512 in one launch
                    (barcodes/s and simplices/s) against one cloud at a time,
                    and the headline batch
  enumeration_pass  the enumeration / apparent-pair filter of so3-1000
                    (dimension 2): candidates, survivors and neighbour lists
                    in bytes over its launch time, with the vector-ALU issue
                    rate beside it
  shortcuts         the ablation of the paper's Table 3 on so3-1000: explicit
                    matrix, implicit storing / discarding R, emergent and
                    apparent shortcuts, with time and entries held
  cocycles          representative cocycles of dimension 1 on so3-1000
  homology          the homology variant on so3-1000 in dims 0-1
  paper_scale       the paper's o3 runs (1024 matrices, t = 1.8, and 4096,
                    t = 1.4, dims 0-3) and its torus4 run (50,000 points,
                    t = 0.15, dims 0-2), one barcode each; the 1024 one also
                    on the CPU implementation of the paper's algorithm
  cpu_baseline      the CPU oracle on this host (a bounded sample of the
                    headline batch: its first clouds), single thread
  cpu_paper_algorithm  the single-threaded CPU implementation of the paper's
                    algorithm (cpu_baseline/) on all 64 clouds, and the same
                    over one process per core

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
       python bench.py --pmc-run            (counter runs under rocprofv3)
       python bench.py --summarize-pmc FETCH_DIR WRITE_DIR   (profiles helpers)
       python bench.py --summarize-trace TRACE_DIR
       python bench.py --summarize-valu PMC_DIR
"""

from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
PMC_SUMMARY = os.path.join(ROOT, "profiles", "pmc_traffic_so3-1000.txt")
PMC_SUMMARY_BATCH = os.path.join(ROOT, "profiles", "pmc_traffic_circles-64x400.txt")
PMC_VALU_SUMMARY = os.path.join(ROOT, "profiles", "pmc_valu_so3-1000.txt")
COPY_BYTES = 1 << 29   # plain copy used to calibrate the counters (512 MiB read + written)


def _code_only(text: str) -> str:
    """The source without comments and whitespace (string and character
    literals kept), so that a comment edit leaves the hash alone."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
        elif c in "\"'":
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        else:
            if not c.isspace():
                out.append(c)
            i += 1
    return "".join(out)


def source_hash() -> str:
    """Hash of the code of the HIP sources (comments and whitespace left out):
    counter summaries are valid for this code only."""
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_1908_02518_amd", "csrc", "*"))):
        if f.endswith((".hip", ".hpp")):
            h.update(os.path.basename(f).encode())
            with open(f, encoding="utf-8") as fh:
                h.update(_code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def read_pmc_summary(path: str):
    """{class: (fetch_bytes, write_bytes) per launch} scaled by the copy
    calibration, or None when absent or stale."""
    if not os.path.exists(path):
        return None
    vals, rows = {}, {}
    for ln in open(path):
        ln = ln.strip()
        if not ln or ln.startswith("#"):
            continue
        parts = ln.split()
        if parts[0] == "kernel":
            rows[parts[1]] = (float(parts[3]), float(parts[5]))
        else:
            vals[parts[0]] = parts[1]
    if vals.get("source_sha256") != source_hash():
        return None
    ff = float(vals["copy_bytes"]) / (float(vals["copy_fetch_kib"]) * 1024.0)
    fw = float(vals["copy_bytes"]) / (float(vals["copy_write_kib"]) * 1024.0)
    return {k: (f * 1024.0 * ff, w * 1024.0 * fw) for k, (f, w) in rows.items()}


def _load_counter(d: str, counter: str):
    """{kernel name: [(dispatch id, value)]} for one counter of a rocprofv3
    --pmc run (csv output)."""
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    per = {}
    for fpath in files:
        with open(fpath) as fh:
            for r in csv.DictReader(fh):
                if r.get("Counter_Name") != counter:
                    continue
                name = r.get("Kernel_Name", "")
                per.setdefault(name, []).append((int(r.get("Dispatch_Id", 0)),
                                                 float(r["Counter_Value"])))
    return per


def _classify(per):
    """Mean value per dispatch of each kernel class. A reduction belongs to
    the dimension of the filter dispatched before it; filters alternate d1,
    d2 in every barcode."""
    allr = sorted((d, name, v) for name, lst in per.items() for d, v in lst)
    out, nfilter, dim, copies = {}, 0, 0, []
    for _, name, v in allr:
        if "k_filter" in name:
            dim = 1 + nfilter % 2
            nfilter += 1
            out.setdefault(f"filter_d{dim}", []).append(v)
        elif "k_reduce" in name:
            out.setdefault(f"reduce_d{dim}", []).append(v)
        elif "k_batched" in name:
            out.setdefault("batched", []).append(v)
        elif "copy" in name.lower() or "elementwise" in name.lower():
            copies.append(v)
    if copies:
        out["copy"] = [max(copies)]
    return {k: sum(v) / len(v) for k, v in out.items()}


# Instruction counters of the vector-ALU pass (one rocprofv3 --pmc run)
VALU_COUNTERS = ("SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_VMEM_RD",
                 "SQ_INSTS_LDS", "SQ_WAVE_CYCLES", "SQ_BUSY_CYCLES", "SQ_WAIT_INST_ANY")
# Vector-ALU issue peak: 256 CUs x 2.4 GHz x one wave64 instruction per CU
# per cycle (four SIMD16 units, four cycles per wave64 instruction each)
VALU_PEAK_GIPS = 256 * 2.4 * 1.0


def summarize_valu(d: str) -> int:
    """Print the profiles/ summary of a rocprofv3 --pmc run of
    `bench.py --pmc-run` with VALU_COUNTERS: mean per dispatch per class."""
    per = {c: _classify(_load_counter(d, c)) for c in VALU_COUNTERS}
    print("# instruction counters per dispatch, rocprofv3 --pmc: bench.py --pmc-run "
          "(circles-64x400 batch and so3-1000 barcode)")
    print(f"source_sha256 {source_hash()}")
    kinds = sorted({k for v in per.values() for k in v if k != "copy"})
    for k in kinds:
        print(f"kernel {k} " + " ".join(f"{c} {per[c].get(k, 0.0):.0f}" for c in VALU_COUNTERS))
    return 0


def read_valu_summary():
    """{class: {counter: value per dispatch}} or None when absent or stale."""
    if not os.path.exists(PMC_VALU_SUMMARY):
        return None
    out, sha = {}, None
    for ln in open(PMC_VALU_SUMMARY):
        parts = ln.split()
        if not parts or parts[0].startswith("#"):
            continue
        if parts[0] == "source_sha256":
            sha = parts[1]
        elif parts[0] == "kernel":
            out[parts[1]] = {parts[q]: float(parts[q + 1]) for q in range(2, len(parts) - 1, 2)}
    return out if sha == source_hash() else None


def alu_rate(prof, name):
    """Vector-ALU issue rate of a kernel class: VALU wave instructions per
    dispatch (committed counter summary) over the live launch time, with its
    LDS and vector-memory instructions; None when the summary is stale."""
    valu = read_valu_summary()
    row = valu.get(name) if valu else None
    if not row or name not in prof:
        return None
    ms, calls = prof[name]
    sec = ms / calls * 1e-3
    ach = row["SQ_INSTS_VALU"] / sec / 1e9
    return {"bound": "alu", "achieved": round(ach, 3), "peak": VALU_PEAK_GIPS,
            "unit": "G wave64 VALU instructions/s", "frac": round(ach / VALU_PEAK_GIPS, 5),
            "lds_instructions": row.get("SQ_INSTS_LDS"),
            "vmem_read_instructions": row.get("SQ_INSTS_VMEM_RD")}


def summarize_pmc(fetch_dir: str, write_dir: str) -> int:
    """Print the profiles/ summary from two rocprofv3 --pmc runs of
    `bench.py --pmc-run` (FETCH_SIZE, then WRITE_SIZE): mean KiB per
    dispatch for each kernel class, and the copy kernel's reading."""
    f = _classify(_load_counter(fetch_dir, "FETCH_SIZE"))
    w = _classify(_load_counter(write_dir, "WRITE_SIZE"))
    print("# HBM traffic per dispatch, rocprofv3 counters (KiB): bench.py --pmc-run "
          "(circles-64x400 batch and so3-1000 barcode)")
    print(f"source_sha256 {source_hash()}")
    print(f"copy_bytes {COPY_BYTES}")
    print(f"copy_fetch_kib {f.get('copy', 0.0):.1f}")
    print(f"copy_write_kib {w.get('copy', 0.0):.1f}")
    for k in sorted(set(f) & set(w)):
        if k != "copy":
            print(f"kernel {k} fetch_kib {f[k]:.1f} write_kib {w[k]:.1f}")
    return 0


def summarize_trace(trace_dir: str) -> int:
    """Print the profiles/ summary of a `rocprofv3 --kernel-trace --stats`
    run of bench.py: calls and mean duration per kernel, with the filter and
    reduction dispatches split by dimension (they alternate d1, d2 in every
    barcode)."""
    files = glob.glob(os.path.join(trace_dir, "**", "*kernel_trace.csv"), recursive=True)
    rows = []
    for fpath in files:
        with open(fpath) as fh:
            for r in csv.DictReader(fh):
                rows.append((int(r["Dispatch_Id"]), r["Kernel_Name"],
                             int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
    rows.sort()
    # a reduction belongs to the dimension of the filter dispatched before it
    # (a reduction relaunched after a scratch overflow has no filter of its own)
    per, nfilter, dim = {}, 0, 0
    for _, name, ns in rows:
        short = name.split("(")[0].replace("void ", "")
        if "k_filter" in name:
            dim = 1 + nfilter % 2
            nfilter += 1
            short = f"{short} [filter_d{dim}]"
        elif "k_reduce" in name:
            short = f"{short} [reduce_d{dim}]"
        per.setdefault(short, []).append(ns)
    # last3_us: mean of the last three dispatches (the timed steps of a
    # `--steps 3` run; earlier ones include warm-up and scratch growth)
    print("# kernel                                                   calls   mean_us  last3_us    total_ms")
    for k, v in sorted(per.items(), key=lambda kv: -sum(kv[1])):
        tail = v[-3:]
        print(f"{k:58s} {len(v):5d} {sum(v) / len(v) / 1e3:9.1f} {sum(tail) / len(tail) / 1e3:9.1f}"
              f" {sum(v) / 1e6:10.2f}")
    return 0


def host_cpu() -> dict:
    """CPU model and core counts of this host."""
    model = None
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for ln in out.splitlines():
            if ln.startswith("Model name:"):
                model = ln.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    if model is None and os.path.exists("/proc/cpuinfo"):
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cores": usable}


def batched_bytes(clouds, counts, stats) -> float:
    """Algorithmic HBM bytes of one batched launch: per cloud the distances
    (points read once, 4 B per pair written), one read of them by the
    threshold / H0 / enumeration passes (4 B per pair), the surviving columns
    written (12 B each) and sorted (2 x 17 B), the reduction's columns
    (17 B) and entries added or stored (16 B each), and the bars (24 B)."""
    total = 0.0
    for b, x in enumerate(clouds):
        n, m = x.shape
        pairs = n * (n - 1) / 2
        s = stats[b]
        cols = s[1]["columns"]
        bars = s[0]["bars_nonzero"] + s[0]["essential"] + s[1]["bars_nonzero"] + s[1]["essential"]
        total += (4.0 * n * m + 4.0 * pairs + 4.0 * pairs + 12.0 * cols + 34.0 * cols
                  + 17.0 * cols + 16.0 * (s[1]["entries_added"] + s[1]["entries_stored"])
                  + 24.0 * bars)
    return total


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="bound on the CPU-oracle sample (seconds)")
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the CPU legs (oracle and the paper's algorithm)")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the legs of the other four workloads")
    ap.add_argument("--no-shortcuts", action="store_true",
                    help="skip the ablation leg (Table 3 of the paper, on so3-1000)")
    ap.add_argument("--no-cocycles", action="store_true",
                    help="skip the representative-cocycle leg (so3-1000, dimension 1)")
    ap.add_argument("--no-homology", action="store_true",
                    help="skip the homology-variant leg (so3-1000, dims 0-1, about 15 s)")
    ap.add_argument("--no-paper-scale", action="store_true",
                    help="skip the paper-scale legs (o3 1024 and 4096, torus4 50,000)")
    ap.add_argument("--pmc-run", action="store_true",
                    help="counter runs: a few steps of the headline batch and of so3-1000, "
                         "plus one plain copy of known size")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"))
    ap.add_argument("--summarize-trace", metavar="TRACE_DIR")
    ap.add_argument("--summarize-valu", metavar="PMC_DIR")
    args = ap.parse_args()
    if args.summarize_pmc:
        return summarize_pmc(*args.summarize_pmc)
    if args.summarize_valu:
        return summarize_valu(args.summarize_valu)
    if args.summarize_trace:
        return summarize_trace(args.summarize_trace)
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: there is no multi-GPU path "
              "(a batch of clouds would shard by clouds across GPUs).",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_1908_02518_amd as rips
    import workloads

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    dev = torch.device("cuda:0")
    c5 = workloads.config(5)
    clouds5 = c5["clouds"]
    kw5 = dict(max_dim=c5["max_dim"], threshold=c5["threshold"], p=c5["p"])
    xb5, off5, nmax5 = rips.pack_clouds(clouds5)
    c2 = workloads.config(2)
    x2 = c2["clouds"][0]
    x2t = torch.from_numpy(x2).to(dev)
    kw2 = dict(max_dim=c2["max_dim"], threshold=c2["threshold"], p=c2["p"])
    torch.cuda.synchronize()

    if args.pmc_run:
        a = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        for i in range(args.steps):
            rips.barcode_batched(xb5, off5, nmax5, **kw5)
            torch.cuda.synchronize()
            rips.barcode_device(x2t, **kw2)
            torch.cuda.synchronize()
            log(f"pmc step {i + 1}/{args.steps}")
        return 0

    def ev_pair():
        return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    # ---- headline: the circles-64x400 batch in one launch
    counts5 = [rips.simplex_counts(torch.from_numpy(x).to(dev), kw5["max_dim"] + 1,
                                   threshold=kw5["threshold"]) for x in clouds5]
    n_simplices = int(sum(sum(c) for c in counts5))
    log(f"workload {c5['name']}: {len(clouds5)} clouds, {n_simplices} simplices of dims 0-2")
    # the launch configuration the autotuner picks on this batch (every
    # configuration's bars agree; it keeps the fastest for the timed steps)
    tuned = rips.batched_autotune(xb5, off5, nmax5, reps=2, **kw5)
    log(f"autotune: delta slots {tuned[0]}, workgroups per CU {tuned[1]}, {tuned[2]:.2f} ms")
    for i in range(args.warmup):
        c0 = time.perf_counter()
        bb = rips.barcode_batched(xb5, off5, nmax5, **kw5)
        torch.cuda.synchronize()
        log(f"warmup {i}: {1e3 * (time.perf_counter() - c0):.2f} ms")
    rips.profile_enable(True)
    evs = [ev_pair() for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        evs[i][0].record()
        bb = rips.barcode_batched(xb5, off5, nmax5, **kw5)
        evs[i][1].record()
        if i % 5 == 4:
            log(f"step {i + 1}/{args.steps}")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rips.profile_enable(False)
    prof5 = rips.profile_read()
    step_ms = sorted(a.elapsed_time(b) for a, b in evs)
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = n_simplices / ((t1 - t0) / args.steps)
    log(f"timed: {ms_per_step:.2f} ms/step (event median {step_ms[len(step_ms) // 2]:.2f} ms)")
    stats5 = bb.stats.cpu().numpy()
    fields = rips.STAT_FIELDS
    st5 = [[{f: int(stats5[b, d, q]) for q, f in enumerate(fields)} for d in range(2)]
           for b in range(len(clouds5))]
    pmc = read_pmc_summary(PMC_SUMMARY_BATCH)
    gms, gcalls = prof5["batched_graph"]
    glaunch = gms / gcalls
    gbytes = batched_bytes(clouds5, counts5, st5)
    gach = gbytes / (glaunch * 1e-3) / 1e9
    tr = pmc.get("batched") if pmc else None
    roofline = {
        "kernel": "k_batched (the batched launch: one hipGraph of the LPT order, the persistent "
                  "kernel and the bar layout)",
        "bound": "hbm",
        "achieved": round(gach, 4),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(gach / HBM_PEAK_GBS, 7),
        "traffic": round(tr[0] + tr[1], 1) if tr else None,
        "bytes_per_launch": gbytes,
        "avg_launch_us": round(glaunch * 1e3, 3),
        "note": "latency-bound: each cloud's dimension-1 reduction is a chain of dependent "
                "column additions in one workgroup; the HBM roof is far away",
    }
    elim5 = {}
    for key in ("candidates", "cleared", "apparent_col", "columns", "emergent", "reduced",
                "additions", "entries_added", "entries_stored"):
        elim5[key] = int(sum(s[1][key] for s in st5))
    elim5["fraction_eliminated"] = round(
        (elim5["cleared"] + elim5["apparent_col"]) / max(1, elim5["candidates"]), 6)

    # ---- the other four workloads
    configs = {"circles-64x400": {
        "ms_per_batch": round(ms_per_step, 3), "simplices_per_s": round(value, 1),
        "barcodes_per_s": round(len(clouds5) / (ms_per_step * 1e-3), 1),
        "simplices": n_simplices, "eliminated_d1": elim5}}
    enum_pass = None
    prof2 = None
    info2 = None
    counts2 = rips.simplex_counts(x2t, kw2["max_dim"] + 1, threshold=kw2["threshold"])
    if not args.no_configs:
        for cid in (1, 2, 3):
            c = workloads.config(cid)
            xt = torch.from_numpy(c["clouds"][0]).to(dev)
            kw = dict(max_dim=c["max_dim"], threshold=c["threshold"], p=c["p"])
            cnt = rips.simplex_counts(xt, kw["max_dim"] + 1, threshold=kw["threshold"])
            rips.barcode_device(xt, **kw)
            torch.cuda.synchronize()
            reps = 10
            ev = [ev_pair() for _ in range(reps)]
            if cid == 2:
                rips.profile_enable(True)
            torch.cuda.synchronize()
            c0 = time.perf_counter()
            for q in range(reps):
                ev[q][0].record()
                _, info = rips.barcode_device(xt, **kw)
                ev[q][1].record()
            torch.cuda.synchronize()
            wall = (time.perf_counter() - c0) / reps
            if cid == 2:
                rips.profile_enable(False)
                prof2 = rips.profile_read()
                info2 = info
            med = sorted(a.elapsed_time(b) for a, b in ev)[reps // 2]
            configs[c["name"]] = {
                "ms_per_barcode": round(wall * 1e3, 3), "event_median_ms": round(med, 3),
                "simplices": cnt, "simplices_per_s": round(sum(cnt) / wall, 1),
                "columns": [info["stats"][k]["columns"] for k in range(1, kw["max_dim"] + 1)],
                "additions": [info["stats"][k]["additions"] for k in range(1, kw["max_dim"] + 1)]}
            log(f"{c['name']}: {wall * 1e3:.2f} ms per barcode")
        # mixture-512 in one launch against one cloud at a time
        c4 = workloads.config(4)
        clouds4 = c4["clouds"]
        kw4 = dict(max_dim=c4["max_dim"], threshold=c4["threshold"], p=c4["p"])
        xb4, off4, nmax4 = rips.pack_clouds(clouds4)
        cnt4 = int(sum(sum(rips.simplex_counts(torch.from_numpy(x).to(dev), 2)) for x in clouds4))
        rips.barcode_batched(xb4, off4, nmax4, **kw4)
        torch.cuda.synchronize()
        reps = 10
        c0 = time.perf_counter()
        for _ in range(reps):
            rips.barcode_batched(xb4, off4, nmax4, **kw4)
        torch.cuda.synchronize()
        tb = (time.perf_counter() - c0) / reps
        xs = [torch.from_numpy(a).to(dev) for a in clouds4]
        torch.cuda.synchronize()
        c0 = time.perf_counter()
        for q, a in enumerate(xs):
            rips.barcode_device(a, **kw4)
        torch.cuda.synchronize()
        ts = time.perf_counter() - c0
        configs[c4["name"]] = {
            "ms_per_batch": round(tb * 1e3, 3), "simplices": cnt4,
            "simplices_per_s": round(cnt4 / tb, 1),
            "barcodes_per_s_batched": round(len(clouds4) / tb, 1),
            "barcodes_per_s_single": round(len(clouds4) / ts, 1),
            "batched_over_single": round(ts / tb, 2),
            "config": list(rips.batched_get_config())}
        log(f"mixture-512: {tb * 1e3:.1f} ms per batch, {ts:.2f} s one at a time")

    if prof2 is not None and "filter_d2" in prof2:
        # the enumeration / apparent-pair pass of so3-1000, dimension 2: the
        # candidates read (12 B), the survivors written (12 B) and the
        # neighbour lists read (8 B per edge); the apparent-pair table the
        # reduction reads afterwards is an implementation choice, reported
        # apart
        fms, fc = prof2["filter_d2"]
        sec = fms / fc * 1e-3
        s2 = info2["stats"][2]
        by = 12.0 * counts2[2] + 12.0 * s2["columns"] + 8.0 * counts2[1]
        ach = by / sec / 1e9
        pmc2 = read_pmc_summary(PMC_SUMMARY)
        tr2 = pmc2.get("filter_d2") if pmc2 else None
        enum_pass = {
            "kernel": "filter_d2 (so3-1000)", "bound": "hbm", "achieved": round(ach, 4),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 7),
            "traffic": round(tr2[0] + tr2[1], 1) if tr2 else None,
            "bytes_per_launch": by, "avg_launch_us": round(sec * 1e6, 3),
            "table_bytes_per_launch": 32.0 * s2["apparent_col"],
            "candidates_per_s": round(counts2[2] / sec, 1),
            "valu": alu_rate(prof2, "filter_d2")}

    shortcuts = None
    if not args.no_shortcuts:
        # the ablation of the paper's Table 3 on so3-1000, its five columns in
        # order (every one with clearing and cohomology): explicit matrix
        # reduction, implicit reduction storing R, discarding R, the emergent
        # shortcut, the apparent one; then this library's default (R kept
        # where cheaper to add) and all shortcuts but clearing. "memory" is
        # the entries the reduction holds (coboundary matrix and stored
        # columns), 16 bytes each.
        C, E, A = rips.SHORTCUT_CLEARING, rips.SHORTCUT_EMERGENT, rips.SHORTCUT_APPARENT
        rows = [("explicit", rips.R_EXPLICIT, C), ("implicit, storing R", rips.R_STORE, C),
                ("discarding R", rips.R_DISCARD, C), ("emergent", rips.R_DISCARD, C | E),
                ("apparent", rips.R_DISCARD, C | E | A),
                ("default (R kept where cheaper)", rips.R_AUTO, C | E | A),
                ("no clearing", rips.R_AUTO, E | A)]
        shortcuts = []
        try:
            for name, mode, flags in rows:
                rips.set_reduced_storage(mode)
                rips.set_shortcuts(flags)
                rips.barcode_device(x2t, **kw2)  # warm-up
                torch.cuda.synchronize()
                tt = []
                for _ in range(3):
                    c0 = time.perf_counter()
                    _, inf_s = rips.barcode_device(x2t, **kw2)
                    torch.cuda.synchronize()
                    tt.append(time.perf_counter() - c0)
                st_s = inf_s["stats"]
                stored = sum(st_s[k]["entries_stored"] for k in range(1, 3))
                shortcuts.append({
                    "column": name,
                    "ms_per_barcode": round(1e3 * sorted(tt)[1], 3),
                    "columns": [st_s[k]["columns"] for k in range(1, 3)],
                    "emergent": [st_s[k]["emergent"] for k in range(1, 3)],
                    "additions": [st_s[k]["additions"] for k in range(1, 3)],
                    "entries_held": [st_s[k]["entries_stored"] for k in range(1, 3)],
                    "memory_mb": round(16 * stored / 1e6, 2),
                })
                log(f"table 3 {name}: {1e3 * sorted(tt)[1]:.1f} ms, {16 * stored / 1e6:.1f} MB")
        finally:
            rips.set_shortcuts()
            rips.set_reduced_storage()

    cocycles = None
    if not args.no_cocycles:
        rips.cocycles(x2, dim=1, threshold=kw2["threshold"], p=kw2["p"])
        tc, tbc = [], []
        for _ in range(3):
            c0 = time.perf_counter()
            cc = rips.cocycles(x2, dim=1, threshold=kw2["threshold"], p=kw2["p"])
            tc.append(time.perf_counter() - c0)
            c0 = time.perf_counter()
            rips.barcode(x2, max_dim=1, threshold=kw2["threshold"], p=kw2["p"])
            tbc.append(time.perf_counter() - c0)
        sizes = [len(sc) for sc, _ in cc.cocycles]
        cocycles = {
            "workload": "so3-1000, t = 1.4, cocycles of dimension 1, Z/2 (host input)",
            "ms_cocycles": round(1e3 * sorted(tc)[1], 2),
            "ms_barcode_dims_0_1": round(1e3 * sorted(tbc)[1], 2),
            "bars": len(sizes), "entries": int(sum(sizes)),
            "max_entries": int(max(sizes)) if sizes else 0,
        }
        log(f"cocycles: {cocycles['ms_cocycles']} ms for {len(sizes)} bars")

    homology = None
    if not args.no_homology:
        c0 = time.perf_counter()
        hom = rips.barcode_homology(x2, max_dim=1, threshold=kw2["threshold"], p=kw2["p"])
        t_hom = time.perf_counter() - c0
        rips.barcode(x2, max_dim=1, threshold=kw2["threshold"], p=kw2["p"])  # warm-up
        c0 = time.perf_counter()
        coh = rips.barcode(x2, max_dim=1, threshold=kw2["threshold"], p=kw2["p"])
        t_coh = time.perf_counter() - c0
        same = all(np.array_equal(getattr(hom.bars[d], f), getattr(coh.bars[d], f))
                   for d in range(2) for f in ("birth", "death", "birth_simplex", "death_simplex"))
        homology = {
            "workload": "so3-1000, t = 1.4, dims 0-1, Z/2 (host input, one call each)",
            "seconds_homology": round(t_hom, 3), "seconds_cohomology": round(t_coh, 4),
            "columns_homology": [hom.stats[d]["columns"] for d in range(2)],
            "cleared_homology": [hom.stats[d]["cleared"] for d in range(2)],
            "additions_homology": [hom.stats[d]["additions"] for d in range(2)],
            "columns_cohomology": [coh.stats[d]["columns"] for d in range(2)],
            "additions_cohomology": [coh.stats[d]["additions"] for d in range(2)],
            "bars_equal": bool(same),
        }
        log(f"homology variant: {t_hom:.2f} s against {1e3 * t_coh:.1f} ms, bars equal {same}")

    paper_scale = None
    if not args.no_paper_scale:
        # the paper's o3 and torus4 runs (Tables 1 and 2): o3 on 1024 and on
        # 4096 orthogonal matrices, torus4 on 50,000 points; one barcode per
        # call, input resident in HBM, median of 3 after a warm-up call
        ripser_s = {6: 2.1, 8: 43.1, 9: 117.0}
        paper_scale = {}
        bars6 = None
        for cfg in (6, 8, 9):
            cp = workloads.config(cfg)
            xp = cp["clouds"][0]
            xpt = torch.from_numpy(xp).to(dev)
            kp = dict(max_dim=cp["max_dim"], threshold=cp["threshold"], p=cp["p"])
            counts_p = rips.simplex_counts(xpt, cp["max_dim"] + 1, threshold=cp["threshold"])
            bars_p, info_p = rips.barcode_device(xpt, **kp)  # warm-up: scratch sizes
            torch.cuda.synchronize()
            tsp = []
            for _ in range(3):
                c0 = time.perf_counter()
                bars_p, info_p = rips.barcode_device(xpt, **kp)
                torch.cuda.synchronize()
                tsp.append(time.perf_counter() - c0)
            tp = sorted(tsp)[1]
            if cfg == 6:
                bars6 = bars_p
            log(f"paper scale {cp['name']}: {tp:.3f} s per barcode (median of 3)")
            paper_scale[cp["name"]] = {
                "points": int(xp.shape[0]),
                "threshold": cp["threshold"],
                "dims": f"0-{cp['max_dim']}",
                "simplex_counts": counts_p,
                "seconds_per_barcode": round(tp, 4),
                "simplices_per_s": round(sum(counts_p) / tp, 1),
                "bars": [int(bars_p[d][0].shape[0]) for d in range(cp["max_dim"] + 1)],
                "context": f"the paper reports {ripser_s[cfg]} s for Ripser on its own data of "
                           "this shape (4 GHz Core i7): other data, other machine, not a target",
            }
            del xpt
            torch.cuda.empty_cache()
        if not args.no_cpu_baseline:
            import cpu_baseline
            import oracle
            c6 = workloads.config(6)
            x6 = c6["clouds"][0]
            k6 = dict(max_dim=c6["max_dim"], threshold=c6["threshold"], p=c6["p"])
            cpu_baseline.build(force=False)
            dl6 = oracle.distances(x6)  # not timed
            c0 = time.perf_counter()
            cb6 = cpu_baseline.barcode(dl6, x6.shape[0], **k6)
            tc6 = time.perf_counter() - c0
            log(f"paper scale, cpu paper algorithm: {tc6:.2f} s")
            e6 = paper_scale[c6["name"]]
            e6["cpu_paper_algorithm_seconds"] = round(tc6, 3)
            e6["bars_equal_cpu_paper_algorithm"] = bool(all(
                np.array_equal(getattr(cb6.bars[d], f), g.cpu().numpy())
                for d in range(c6["max_dim"] + 1)
                for f, g in zip(("birth", "death", "birth_simplex", "death_simplex"), bars6[d])))

    cpu = None
    cpu_paper = None
    if not args.no_cpu_baseline:
        import cpu_baseline
        import oracle
        hc = host_cpu()
        oracle.build(force=False)
        # the oracle on the first clouds of the headline batch, one thread,
        # until the bound on CPU seconds is reached
        el, done, simp = 0.0, 0, 0
        while done < len(clouds5) and (done == 0 or el < args.cpu_seconds):
            c0 = time.perf_counter()
            oracle.barcode(clouds5[done], **kw5)
            el += time.perf_counter() - c0
            simp += sum(counts5[done])
            done += 1
            log(f"cpu oracle cloud {done}: {el / done:.2f} s per cloud")
        cpu = {"value": round(simp / el, 1), "unit": "simplices/s", "cores": 1, "kind": "oracle",
               "sample": f"the first {done} clouds of the circles-64x400 batch (same inputs), "
                         f"{el / done:.3f} s per cloud, single thread",
               **hc}
        # the paper's algorithm on every cloud of the batch, one thread; then
        # one process per usable core (at most 16)
        cpu_baseline.build(force=False)
        dls = [oracle.distances(x) for x in clouds5]  # the same float32 distances (not timed)
        c0 = time.perf_counter()
        res = [cpu_baseline.barcode(dl, x.shape[0], **kw5) for dl, x in zip(dls, clouds5)]
        tcpu = time.perf_counter() - c0
        same = True
        for b, r in enumerate(res):
            for d in range(kw5["max_dim"] + 1):
                seg = [t.cpu().numpy() for t in bb.segment(b, d)]
                for f, g in zip(("birth", "death", "birth_simplex", "death_simplex"), seg):
                    same = same and np.array_equal(getattr(r.bars[d], f), g)
        workers = max(1, min(16, hc["usable_cores"] or 1))
        tpar = cpu_baseline.timed_pool(dls, [x.shape[0] for x in clouds5], workers, **kw5)
        log(f"cpu paper algorithm: {tcpu:.2f} s for the batch on one thread, {tpar:.2f} s on "
            f"{workers} processes")
        cpu_paper = {"value": round(n_simplices / tcpu, 1), "unit": "simplices/s", "cores": 1,
                     "kind": "paper algorithm, single thread (cpu_baseline/)",
                     "sample": f"all {len(clouds5)} clouds of the circles-64x400 batch, "
                               f"{tcpu:.3f} s; distances precomputed",
                     "bars_equal_gpu": bool(same),
                     "all_cores": {"value": round(n_simplices / tpar, 1), "cores": workers,
                                   "seconds": round(tpar, 3),
                                   "kind": "the same, one process per core over the clouds"},
                     **hc}

    line = {
        "metric": "simplices/s (the circles-64x400 batch of barcodes per step)",
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
        "config": {"workload": "circles-64x400: 64 clouds of 400 points in R^2 (360 on the unit "
                               "circle, noise 0.1, 40 uniform outliers in [-2, 2]^2), float32, "
                               "full Rips, dims 0-1, Z/2, one persistent launch",
                   "clouds": len(clouds5), "n": 400, "dims": 1, "p": 2,
                   "simplices": n_simplices,
                   "launch": {"delta_slots": tuned[0], "workgroups_per_cu": tuned[1],
                              "chosen_by": "rips_batched_autotune on this batch",
                              "autotune_ms": round(tuned[2], 3)}},
        "event_ms_per_step": {"median": round(step_ms[len(step_ms) // 2], 4),
                              "min": round(step_ms[0], 4), "max": round(step_ms[-1], 4)},
        "barcodes_per_s": round(len(clouds5) / (ms_per_step * 1e-3), 1),
        "roofline": roofline,
        "enumeration_pass": enum_pass,
        "configs": configs,
        "kernels_ms_per_barcode_so3_1000": (
            {k: round(v[0] / v[1], 4) for k, v in sorted(prof2.items())} if prof2 else None),
        "shortcuts": shortcuts,
        "homology": homology,
        "cocycles": cocycles,
        "paper_scale": paper_scale,
        "cpu_baseline": cpu,
        "cpu_paper_algorithm": cpu_paper,
    }
    print(json.dumps(line))
    return 0


if __name__ == "__main__":
    sys.exit(main())
