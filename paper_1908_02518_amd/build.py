"""Build of the gfx950 HIP library (librips.so), in-tree.

hipcc cross-compiles for gfx950 without a GPU. Flags: -ffp-contract=off keeps
every float32 product and sum rounded separately (the distance formula must
match the CPU bit for bit); packed-fp32 instructions are disabled.
"""

from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librips.so")
SOURCES = ["rips_kernels.hip", "rips_batched.hip", "rips_homology.hip", "rips_explicit.hip", "rips_api.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-function",
]


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]


def _compile(src: str, extra) -> tuple:
    obj = os.path.join(CSRC, os.path.basename(src) + ".o")
    cmd = [HIPCC, *FLAGS, *extra, "-I", os.path.join(ROOT, "include"), "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(ln for ln in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in ln)
    return src, obj, r.returncode, out


def build(verbose: bool = False) -> str:
    """Compile every source into librips.so (always recompiles; the sources
    compile in parallel)."""
    from concurrent.futures import ThreadPoolExecutor
    # RIPS_PHASE_TIMERS=1 compiles the reduction's phase timers in (profiling only)
    extra = ["-DRIPS_PHASE_TIMERS=1"] if os.environ.get("RIPS_PHASE_TIMERS") == "1" else []
    # RIPS_COLUMN_TRACE=1 records per-column clocks of the spread-out
    # reduction into the file named by RIPS_COLUMN_TRACE_OUT (profiling only)
    if os.environ.get("RIPS_COLUMN_TRACE") == "1":
        extra.append("-DRIPS_COLUMN_TRACE=1")
    srcs = sources()
    with ThreadPoolExecutor(max_workers=max(1, min(len(srcs), os.cpu_count() or 1))) as ex:
        results = list(ex.map(lambda s: _compile(s, extra), srcs))
    objs = []
    for src, obj, rc, out in results:
        if rc != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{out}")
        if verbose and out.strip():
            print(out)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}{r.stderr}")
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
