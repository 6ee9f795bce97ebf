#!/usr/bin/env python3
"""Throughput of the Vietoris-Rips persistence hot path on one MI355X.

One step = one full barcode (distances, threshold, H0, enumeration /
apparent-pair filter, column sort and Z/p reduction in every dimension) of
the so3-1000 workload: 1000 Haar-random rotations of R^3 flattened to R^9,
float32, threshold 1.4, dimensions 0-2, Z/2 (the shape of the paper's o3
data set). The input is resident in HBM before the timed region.

value = simplices/s = (|K_0| + |K_1| + |K_2| + |K_3|) at the threshold, the size
of the explicit filtration the method avoids building, divided by the time
per step. Also reported:
  roofline          the dominant kernel's algorithmic bytes per launch over
                    its mean launch time (HIP events on the library's
                    stream), against the HBM peak; traffic = HBM bytes per
                    launch from rocprofv3 FETCH_SIZE / WRITE_SIZE counters
                    (committed summary under profiles/, scaled by a plain copy
                    of known size), null when the kernel sources changed since
  enumeration_pass  the same for the enumeration / apparent-pair filter
  valu              (in both) the kernel's vector-ALU issue rate: VALU wave
                    instructions per dispatch from a committed rocprofv3
                    counter summary over the live launch time, against
                    256 CUs x 2.4 GHz x one wave64 instruction per CU-cycle
  batched           barcodes/s of the 512-cloud mixture batch in one
                    persistent launch vs one cloud at a time
  shortcuts         the shortcut ablation of the paper's Table 3 on the same
                    cloud: ms per barcode with clearing and no other
                    shortcut, clearing + emergent, all three (the default),
                    clearing + apparent; and cohomology without clearing
  cocycles          representative cocycles of dimension 1 on the bench
                    cloud: ms per call against the plain barcode, entries
  homology          the homology variant (boundary matrices with clearing,
                    top dimension first) on the bench cloud in dims 0-1,
                    against cohomology: seconds, columns and additions
  paper_scale       one barcode of a paper-scale workload (o3 shape, 1024
                    points, threshold 1.8, dims 0-3), against the CPU
                    implementation of the paper's algorithm
  cpu_baseline      the CPU oracle on this host (a bounded sample)
  cpu_paper_algorithm  the single-threaded CPU implementation of the paper's
                    algorithm (cpu_baseline/) on the same cloud, same host

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
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
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
PMC_SUMMARY = os.path.join(ROOT, "profiles", "pmc_traffic_so3-1000.txt")
PMC_VALU_SUMMARY = os.path.join(ROOT, "profiles", "pmc_valu_so3-1000.txt")
COPY_BYTES = 1 << 29   # plain copy used to calibrate the counters (512 MiB read + written)


def source_hash() -> str:
    """Hash of the HIP sources: counter summaries are valid for these only."""
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_1908_02518_amd", "csrc", "*"))):
        if f.endswith((".hip", ".hpp")):
            h.update(os.path.basename(f).encode())
            with open(f, "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def kernel_bytes(name: str, n: int, counts, stats, sparse: bool) -> float | None:
    """Algorithmic HBM bytes of one launch of a kernel class: what the method
    must move once. Records: simplex (index 8 B + diameter 4 B), column
    (+ zero pivot cofacet 4 B + flag 1 B), apparent-pair table record (4 x
    8 B), reduction entry (index 8 B + diameter 4 B + coefficient 4 B)."""
    edges = counts[1] if len(counts) > 1 else 0
    dmat = 4.0 * n * n
    if name == "distances":
        return dmat
    if name == "edges":
        return dmat + 12.0 * edges
    if name.startswith("filter_d"):
        # + one apparent-pair table record per zero apparent pair (tau key,
        # rho value, rho's vertices, its neighbour-list span: 4 x 8 B)
        k = int(name[-1])
        return (12.0 * counts[k] + 17.0 * stats[k]["columns"] + 32.0 * stats[k]["apparent_col"]
                + (8.0 * edges if sparse else dmat))
    if name.startswith("expand_d"):
        k = int(name[-1])
        return 12.0 * counts[k - 1] + 12.0 * counts[k] + (8.0 * edges if sparse else dmat)
    if name.startswith("sort_d"):
        k = int(name[-1])
        return 2.0 * 17.0 * stats[k]["columns"]
    if name.startswith("reduce_d"):
        k = int(name[-1])
        s = stats[k]
        return 17.0 * s["columns"] + 16.0 * (s["entries_added"] + s["entries_stored"])
    if name == "h0":
        return 12.0 * edges + 16.0 * n
    return None


def read_pmc_summary():
    """{class: (fetch_bytes, write_bytes) per launch} scaled by the copy
    calibration, or None when absent or stale."""
    if not os.path.exists(PMC_SUMMARY):
        return None
    vals, rows = {}, {}
    for ln in open(PMC_SUMMARY):
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
    print("# instruction counters per dispatch, rocprofv3 --pmc, so3-1000 barcode")
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


def summarize_pmc(fetch_dir: str, write_dir: str) -> int:
    """Print the profiles/ summary from two rocprofv3 --pmc runs of
    `bench.py --pmc-run` (FETCH_SIZE, then WRITE_SIZE): mean KiB per
    dispatch for each kernel class, and the copy kernel's reading."""
    f = _classify(_load_counter(fetch_dir, "FETCH_SIZE"))
    w = _classify(_load_counter(write_dir, "WRITE_SIZE"))
    print("# HBM traffic per dispatch, rocprofv3 counters (KiB), so3-1000 barcode")
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


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="bound on the CPU-oracle sample (seconds)")
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip both CPU legs (oracle and the paper's algorithm)")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-shortcuts", action="store_true",
                    help="skip the shortcut ablation leg (Table 3 of the paper, on so3-1000)")
    ap.add_argument("--no-cocycles", action="store_true",
                    help="skip the representative-cocycle leg (so3-1000, dimension 1)")
    ap.add_argument("--no-homology", action="store_true",
                    help="skip the homology-variant leg (so3-1000, dims 0-1, about 15 s)")
    ap.add_argument("--no-paper-scale", action="store_true",
                    help="skip the paper-scale o3-1024 (t = 1.8, dims 0-3) leg")
    ap.add_argument("--pmc-run", action="store_true",
                    help="counter runs: a few steps plus one plain copy of known size")
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

    cfg = workloads.config(2)
    x = cfg["clouds"][0]
    n, m = x.shape
    t, p, max_dim = cfg["threshold"], cfg["p"], cfg["max_dim"]
    dev = torch.device("cuda:0")
    xt = torch.from_numpy(x).to(dev)
    torch.cuda.synchronize()

    if args.pmc_run:
        a = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        for i in range(args.steps):
            rips.barcode_device(xt, max_dim=max_dim, threshold=t, p=p)
            torch.cuda.synchronize()
            log(f"pmc step {i + 1}/{args.steps}")
        return 0

    # size of the explicit filtration (numerator), outside the timed region
    counts = rips.simplex_counts(xt, max_dim + 1, threshold=t)
    n_simplices = int(sum(counts))
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
    sparse = info["sparse"]
    pmc = read_pmc_summary()
    valu = read_valu_summary()

    def roof(name):
        ms, calls = prof[name]
        per_launch_ms = ms / calls
        by = kernel_bytes(name, n, counts, stats, sparse)
        ach = by / (per_launch_ms * 1e-3) / 1e9 if by else None
        tr = pmc.get(name) if pmc else None
        return {
            "kernel": name,
            "bound": "hbm",
            "achieved": round(ach, 4) if ach is not None else None,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 7) if ach is not None else None,
            "traffic": round(tr[0] + tr[1], 1) if tr else None,
            "bytes_per_launch": by,
            "avg_launch_us": round(per_launch_ms * 1e3, 3),
        }

    def alu(name):
        """Vector-ALU issue rate of a kernel class: VALU wave instructions
        per dispatch (committed counter summary) over the live launch time;
        LDS instructions alongside. None when the summary is stale."""
        row = valu.get(name) if valu else None
        if not row:
            return None
        ms, calls = prof[name]
        sec = ms / calls * 1e-3
        ach = row["SQ_INSTS_VALU"] / sec / 1e9
        return {"bound": "alu", "achieved": round(ach, 3), "peak": VALU_PEAK_GIPS,
                "unit": "G wave64 VALU instructions/s", "frac": round(ach / VALU_PEAK_GIPS, 5),
                "lds_instructions": row.get("SQ_INSTS_LDS"),
                "vmem_read_instructions": row.get("SQ_INSTS_VMEM_RD")}

    dname = max(prof.items(), key=lambda kv: kv[1][0])[0]
    roofline = roof(dname)
    roofline["valu"] = alu(dname)
    if dname.startswith("reduce_d"):
        k = int(dname[-1])
        s = stats[k]
        roofline["note"] = ("column reduction spread over one workgroup per CU, bound by the "
                            "latency of the longest chain of dependent additions: "
                            f"{s['columns']} columns, {s['additions']} additions, "
                            f"{s['entries_added']} entries added, {s['entries_stored']} stored")
        roofline["columns_per_s"] = round(s["columns"] / (roofline["avg_launch_us"] * 1e-6), 1)
    fname = f"filter_d{max_dim}"
    enum_pass = None
    if fname in prof:
        enum_pass = roof(fname)
        fms, fc = prof[fname]
        enum_pass["candidates_per_s"] = round(counts[max_dim] / (fms / fc * 1e-3), 1)
        enum_pass["valu"] = alu(fname)

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

    batched = None
    if not args.no_batched:
        c4 = workloads.config(4)
        clouds = c4["clouds"]
        xb, off, nmax = rips.pack_clouds(clouds)
        rips.barcode_batched(xb, off, nmax, max_dim=c4["max_dim"], p=c4["p"])  # graph + scratch
        torch.cuda.synchronize()
        reps = 5
        c0 = time.perf_counter()
        for _ in range(reps):
            rips.barcode_batched(xb, off, nmax, max_dim=c4["max_dim"], p=c4["p"])
        torch.cuda.synchronize()
        tb = (time.perf_counter() - c0) / reps
        log(f"batched mixture-512: {1e3 * tb:.1f} ms per batch")
        xs = [torch.from_numpy(a).to(dev) for a in clouds]
        torch.cuda.synchronize()
        c0 = time.perf_counter()
        for q, a in enumerate(xs):
            rips.barcode_device(a, max_dim=c4["max_dim"], p=c4["p"])
            if q % 128 == 127:
                log(f"one at a time: {q + 1}/{len(xs)}")
        torch.cuda.synchronize()
        ts = time.perf_counter() - c0
        batched = {
            "workload": "mixture-512: 512 clouds of 32-256 points in R^3 (1-3 noisy circles "
                        "and blobs), full Rips, dims 0-1, Z/2",
            "barcodes_per_s_batched": round(len(clouds) / tb, 1),
            "barcodes_per_s_single": round(len(clouds) / ts, 1),
            "ratio": round(ts / tb, 2),
            "config": list(rips.batched_get_config()),
        }

    shortcuts = None
    if not args.no_shortcuts:
        # the ablation of the paper's Table 3 on the bench cloud, every row
        # with clearing: no other shortcut ("discarded"), the emergent
        # shortcut, both ("apparent"); the apparent one alone; and all but
        # clearing (cohomology without clearing)
        C, E, A = rips.SHORTCUT_CLEARING, rips.SHORTCUT_EMERGENT, rips.SHORTCUT_APPARENT
        names = {C: "clearing", C | E: "clearing + emergent",
                 C | E | A: "clearing + emergent + apparent (default)",
                 C | A: "clearing + apparent", E | A: "emergent + apparent, no clearing"}
        shortcuts = []
        try:
            for flags in names:
                rips.set_shortcuts(flags)
                rips.barcode_device(xt, max_dim=max_dim, threshold=t, p=p)  # warm-up
                torch.cuda.synchronize()
                tt = []
                for _ in range(3):
                    c0 = time.perf_counter()
                    _, inf_s = rips.barcode_device(xt, max_dim=max_dim, threshold=t, p=p)
                    torch.cuda.synchronize()
                    tt.append(time.perf_counter() - c0)
                st_s = inf_s["stats"]
                shortcuts.append({
                    "shortcuts": names[flags],
                    "ms_per_barcode": round(1e3 * sorted(tt)[1], 3),
                    "columns": [st_s[k]["columns"] for k in range(1, max_dim + 1)],
                    "emergent": [st_s[k]["emergent"] for k in range(1, max_dim + 1)],
                    "additions": [st_s[k]["additions"] for k in range(1, max_dim + 1)],
                })
                log(f"shortcuts {names[flags]}: {1e3 * sorted(tt)[1]:.1f} ms")
        finally:
            rips.set_shortcuts()

    cocycles = None
    if not args.no_cocycles:
        # representative cocycles of dimension 1 on the bench cloud (V_j of
        # every bar, essential columns included), against the plain barcode
        # of the same dimensions; host input, median of three after a warm-up
        rips.cocycles(x, dim=1, threshold=t, p=p)
        tc, tb = [], []
        for _ in range(3):
            c0 = time.perf_counter()
            cc = rips.cocycles(x, dim=1, threshold=t, p=p)
            tc.append(time.perf_counter() - c0)
            c0 = time.perf_counter()
            rips.barcode(x, max_dim=1, threshold=t, p=p)
            tb.append(time.perf_counter() - c0)
        sizes = [len(sc) for sc, _ in cc.cocycles]
        cocycles = {
            "workload": "so3-1000, t = 1.4, cocycles of dimension 1, Z/2 (host input)",
            "ms_cocycles": round(1e3 * sorted(tc)[1], 2),
            "ms_barcode_dims_0_1": round(1e3 * sorted(tb)[1], 2),
            "bars": len(sizes),
            "entries": int(sum(sizes)),
            "max_entries": int(max(sizes)) if sizes else 0,
        }
        log(f"cocycles: {cocycles['ms_cocycles']} ms for {len(sizes)} bars")

    homology = None
    if not args.no_homology:
        # the homology variant on the bench cloud, dims 0-1: boundary matrices
        # with clearing from the top down, against cohomology with clearing
        # (sections "Clearing inessential birth columns" and "Cohomology")
        c0 = time.perf_counter()
        hom = rips.barcode_homology(x, max_dim=1, threshold=t, p=p)
        t_hom = time.perf_counter() - c0
        rips.barcode(x, max_dim=1, threshold=t, p=p)  # warm-up
        c0 = time.perf_counter()
        coh = rips.barcode(x, max_dim=1, threshold=t, p=p)
        t_coh = time.perf_counter() - c0
        same = all(np.array_equal(getattr(hom.bars[d], f), getattr(coh.bars[d], f))
                   for d in range(2) for f in ("birth", "death", "birth_simplex", "death_simplex"))
        homology = {
            "workload": "so3-1000, t = 1.4, dims 0-1, Z/2 (host input, one call each)",
            "seconds_homology": round(t_hom, 3),
            "seconds_cohomology": round(t_coh, 4),
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
        c6 = workloads.config(6)
        x6 = c6["clouds"][0]
        x6t = torch.from_numpy(x6).to(dev)
        k6 = dict(max_dim=c6["max_dim"], threshold=c6["threshold"], p=c6["p"])
        counts6 = rips.simplex_counts(x6t, c6["max_dim"] + 1, threshold=c6["threshold"])
        bars6, _ = rips.barcode_device(x6t, **k6)  # warm-up: scratch sizes
        torch.cuda.synchronize()
        ts6 = []
        for _ in range(3):
            c0 = time.perf_counter()
            bars6, _ = rips.barcode_device(x6t, **k6)
            torch.cuda.synchronize()
            ts6.append(time.perf_counter() - c0)
        t6 = sorted(ts6)[1]
        log(f"paper scale {c6['name']}: {t6:.3f} s per barcode (median of 3)")
        paper_scale = {
            "workload": "o3-1024-t1.8: 1024 Haar SO(3) rotations in R^9, float32, threshold 1.8, "
                        "dims 0-3, Z/2 (the shape of the paper's o3 1024 run)",
            "simplex_counts": counts6,
            "seconds_per_barcode": round(t6, 4),
            "simplices_per_s": round(sum(counts6) / t6, 1),
            "context": "the paper reports 2.1 s for Ripser on its own o3 1024 data (t = 1.8, "
                       "4 GHz Core i7): other data, other machine, not a target",
        }
        if not args.no_cpu_baseline:
            import cpu_baseline
            import oracle
            cpu_baseline.build(force=False)
            dl6 = oracle.distances(x6)  # not timed
            c0 = time.perf_counter()
            cb6 = cpu_baseline.barcode(dl6, x6.shape[0], **k6)
            tc6 = time.perf_counter() - c0
            log(f"paper scale, cpu paper algorithm: {tc6:.2f} s")
            paper_scale["cpu_paper_algorithm_seconds"] = round(tc6, 3)
            paper_scale["bars_equal_cpu_paper_algorithm"] = bool(all(
                np.array_equal(getattr(cb6.bars[d], f), g.cpu().numpy())
                for d in range(c6["max_dim"] + 1)
                for f, g in zip(("birth", "death", "birth_simplex", "death_simplex"), bars6[d])))

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
        cpu = {"value": round(n_simplices / (el / reps), 1), "unit": "simplices/s", "cores": 1,
               "kind": "oracle",
               "sample": f"the full so3-1000 cloud (same input), {reps} run(s), "
                         f"{el / reps:.3f} s each, single thread"}

    cpu_paper = None
    if not args.no_cpu_baseline:
        import cpu_baseline
        import oracle
        cpu_baseline.build(force=False)
        dl = oracle.distances(x)  # the same float32 distances (not timed)
        reps, el = 0, 0.0
        while reps == 0 or el < 5.0:
            c0 = time.perf_counter()
            cb = cpu_baseline.barcode(dl, n, max_dim=max_dim, threshold=t, p=p)
            el += time.perf_counter() - c0
            reps += 1
        log(f"cpu paper algorithm: {el / reps:.3f} s per barcode ({reps} runs)")
        same = all(np.array_equal(getattr(cb.bars[d], f), g.cpu().numpy())
                   for d in range(max_dim + 1)
                   for f, g in zip(("birth", "death", "birth_simplex", "death_simplex"), bars[d]))
        cpu_paper = {"value": round(n_simplices / (el / reps), 1), "unit": "simplices/s", "cores": 1,
                     "kind": "paper algorithm, single thread (cpu_baseline/)",
                     "sample": f"the full so3-1000 cloud, {reps} run(s), {el / reps:.3f} s each; "
                               f"distances precomputed",
                     "bars_equal_gpu": bool(same)}

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
        "batched": batched,
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
