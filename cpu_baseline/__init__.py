"""A plain single-threaded CPU implementation of the paper's algorithm -- a
PERFORMANCE BASELINE, timed beside the GPU library and the oracle.

``paper_cpu.c`` follows the paper (Bauer, arXiv:1908.02518): implicit
coboundary columns in the combinatorial number system, cohomology with
clearing, a binary heap with lazy cancellation for the working column, the
stored reduction matrix V, and the shortcuts for zero-persistence apparent
and emergent pairs. It shares no code with the GPU library or the oracle;
only ``bench.py`` and the tests call it.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "paper_cpu.c")
_LIB = os.path.join(_HERE, "libpaper_cpu.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile with gcc (-O2, -ffp-contract=off: float32 comparisons only)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                        "-shared", "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    f32p = ctypes.POINTER(ctypes.c_float)
    i64p = ctypes.POINTER(ctypes.c_int64)
    lib.pc_run.argtypes = [f32p, ctypes.c_int32, ctypes.c_int32, ctypes.c_float, ctypes.c_uint32]
    lib.pc_run.restype = P
    lib.pc_free.argtypes = [P]
    lib.pc_threshold.argtypes = [P]
    lib.pc_threshold.restype = ctypes.c_float
    for name in ("pc_num_bars", "pc_num_columns", "pc_num_additions"):
        fn = getattr(lib, name)
        fn.argtypes = [P, ctypes.c_int]
        fn.restype = ctypes.c_int64
    lib.pc_get_bars.argtypes = [P, ctypes.c_int, f32p, f32p, i64p, i64p]
    _lib = lib
    return lib


@dataclass
class Bars:
    birth: np.ndarray
    death: np.ndarray
    birth_simplex: np.ndarray
    death_simplex: np.ndarray


@dataclass
class Result:
    threshold: float
    bars: list
    columns: list
    additions: list


def barcode(dist_lower: np.ndarray, n: int, *, max_dim: int = 1,
            threshold: float = float("inf"), p: int = 2) -> Result:
    """Barcode from the lower triangle (i > j, row-major) of a float32
    distance matrix on n points; bars in the canonical order (birth
    ascending, then birth simplex index descending)."""
    lib = _load()
    dl = np.ascontiguousarray(dist_lower, dtype=np.float32)
    if dl.shape[0] == 0:
        dl = np.zeros(1, np.float32)
    h = lib.pc_run(dl.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), n, max_dim,
                   ctypes.c_float(threshold), p)
    if not h:
        raise ValueError("paper_cpu: invalid arguments")
    try:
        bars, cols, adds = [], [], []
        for k in range(max_dim + 1):
            nb = lib.pc_num_bars(h, k)
            b = np.empty(nb, np.float32)
            d = np.empty(nb, np.float32)
            bs = np.empty(nb, np.int64)
            ds = np.empty(nb, np.int64)
            if nb:
                lib.pc_get_bars(h, k, b.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                d.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                bs.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                ds.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
            bars.append(Bars(b, d, bs, ds))
            cols.append(int(lib.pc_num_columns(h, k)))
            adds.append(int(lib.pc_num_additions(h, k)))
        return Result(float(lib.pc_threshold(h)), bars, cols, adds)
    finally:
        lib.pc_free(h)


def _pool_one(args):
    dl, n, kw = args
    barcode(dl, n, **kw)
    return 0


def timed_pool(dist_lowers, ns, workers: int, **kw) -> float:
    """Wall seconds of barcode() over many clouds in `workers` processes (one
    cloud per task, largest first), with the workers started and warmed up
    before the clock starts. The processes are spawned, so none inherits a
    process that uses the GPU."""
    import multiprocessing as mp
    import time
    order = sorted(range(len(ns)), key=lambda b: -ns[b])
    ctx = mp.get_context("spawn")
    with ctx.Pool(workers) as pool:
        warm = np.zeros(3, np.float32) + 1.0
        pool.map(_pool_one, [(warm, 3, dict(max_dim=1))] * workers)
        t0 = time.perf_counter()
        pool.map(_pool_one, [(dist_lowers[b], ns[b], kw) for b in order], chunksize=1)
        return time.perf_counter() - t0
