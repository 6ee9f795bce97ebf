"""MI355X (gfx950) Vietoris-Rips persistence barcodes -- Python binding.

A thin ctypes binding of the C ABI declared in include/rips.h (librips.so,
built in-tree by ``paper_1908_02518_amd.build``). It only marshals
arguments: every step of the method runs in the library's HIP kernels. If
the library is missing this module raises at import; there is no other
implementation behind it.

Functions take and return torch tensors (device-resident inputs) or numpy
arrays (host inputs):

* ``barcode(points, ...)``        host arrays in, host results out (C ABI rips_barcode)
* ``barcode_device(x, ...)``      torch.cuda tensor in, torch.cuda bars out
* ``simplex_counts(x, top, ...)`` |K_d| for d <= top on the GPU
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librips.so")

RIPS_MAX_DIM = 3
RIPS_MAX_POINTS = 65535

STATUS = {
    0: "RIPS_OK",
    -1: "RIPS_E_INVALID_ARG",
    -2: "RIPS_E_NOT_PRIME",
    -3: "RIPS_E_INDEX_OVERFLOW",
    -4: "RIPS_E_NONFINITE",
    -5: "RIPS_E_OOM",
    -6: "RIPS_E_CAPACITY",
    -7: "RIPS_E_HIP",
}

# exported symbols, in include/rips.h order
EXPORTS = (
    "rips_barcode",
    "rips_result_free",
    "rips_barcode_cocycles",
    "rips_barcode_homology",
    "rips_set_working_column",
    "rips_get_working_column",
    "rips_set_reduced_storage",
    "rips_get_reduced_storage",
    "rips_cocycles_free",
    "rips_status_string",
    "rips_last_error",
    "rips_barcode_device",
    "rips_barcode_device_noalloc",
    "rips_simplex_counts_device",
    "rips_barcode_batched_device",
    "rips_backward_device",
    "rips_set_reduce_workgroups",
    "rips_get_reduce_workgroups",
    "rips_set_shortcuts",
    "rips_get_shortcuts",
    "rips_batched_set_config",
    "rips_batched_set_spread",
    "rips_batched_get_config",
    "rips_batched_autotune",
    "rips_profile_enable",
    "rips_profile_count",
    "rips_profile_name",
    "rips_profile_ms",
    "rips_profile_calls",
)


class RipsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class rips_bars(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int64),
                ("birth", ctypes.POINTER(ctypes.c_float)),
                ("death", ctypes.POINTER(ctypes.c_float)),
                ("birth_simplex", ctypes.POINTER(ctypes.c_int64)),
                ("death_simplex", ctypes.POINTER(ctypes.c_int64))]


STAT_FIELDS = ("candidates", "cleared", "apparent_col", "apparent_pivot", "columns", "emergent",
               "reduced", "additions", "bars_nonzero", "essential", "entries_added",
               "entries_stored")


class rips_dim_stats(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int64) for f in STAT_FIELDS]


class rips_result(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32),
                ("max_dim", ctypes.c_int32),
                ("p", ctypes.c_uint32),
                ("sparse", ctypes.c_int32),
                ("threshold_used", ctypes.c_float),
                ("enclosing_radius", ctypes.c_float),
                ("dims", ctypes.POINTER(rips_bars)),
                ("stats", ctypes.POINTER(rips_dim_stats)),
                ("simplex_count", ctypes.POINTER(ctypes.c_int64)),
                ("column_count", ctypes.POINTER(ctypes.c_int64)),
                ("column_index", ctypes.POINTER(ctypes.POINTER(ctypes.c_int64))),
                ("column_diam", ctypes.POINTER(ctypes.POINTER(ctypes.c_float)))]


class rips_cocycles(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32),
                ("count", ctypes.c_int64),
                ("birth", ctypes.POINTER(ctypes.c_float)),
                ("death", ctypes.POINTER(ctypes.c_float)),
                ("birth_simplex", ctypes.POINTER(ctypes.c_int64)),
                ("death_simplex", ctypes.POINTER(ctypes.c_int64)),
                ("offsets", ctypes.POINTER(ctypes.c_int64)),
                ("simplex", ctypes.POINTER(ctypes.c_int64)),
                ("coef", ctypes.POINTER(ctypes.c_uint32))]


_D1 = RIPS_MAX_DIM + 1


class rips_device_out(ctypes.Structure):
    _fields_ = [("cap", ctypes.c_int64),
                ("birth", ctypes.c_void_p),
                ("death", ctypes.c_void_p),
                ("birth_simplex", ctypes.c_void_p),
                ("death_simplex", ctypes.c_void_p),
                ("count", ctypes.c_int64 * _D1),
                ("stats", rips_dim_stats * _D1),
                ("simplex_count", ctypes.c_int64 * _D1),
                ("threshold_used", ctypes.c_float),
                ("sparse", ctypes.c_int32),
                ("needed_cap", ctypes.c_int64)]


class rips_batch_out(ctypes.Structure):
    _fields_ = [("cap", ctypes.c_int64),
                ("birth", ctypes.c_void_p),
                ("death", ctypes.c_void_p),
                ("birth_simplex", ctypes.c_void_p),
                ("death_simplex", ctypes.c_void_p),
                ("bar_offsets", ctypes.c_void_p),
                ("stats", ctypes.c_void_p),
                ("threshold_used", ctypes.c_void_p),
                ("needed", ctypes.c_int64)]


def _load():
    # One HIP runtime per process: torch ships its own libamdhip64 (SONAME
    # libamdhip64.so.7) and resolves it through its RPATH. Importing torch
    # first lets librips.so bind to that same, already loaded runtime instead
    # of a second copy from /opt/rocm, which would make torch see no GPU.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python paper_1908_02518_amd/build.py` "
            "(hipcc, gfx950). There is no fallback implementation.")
    lib = ctypes.CDLL(LIB_PATH)
    f32p = ctypes.POINTER(ctypes.c_float)
    lib.rips_barcode.argtypes = [f32p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                 ctypes.c_float, ctypes.c_uint32,
                                 ctypes.POINTER(ctypes.POINTER(rips_result))]
    lib.rips_barcode.restype = ctypes.c_int
    lib.rips_barcode_homology.argtypes = lib.rips_barcode.argtypes
    lib.rips_barcode_homology.restype = ctypes.c_int
    lib.rips_result_free.argtypes = [ctypes.POINTER(rips_result)]
    lib.rips_result_free.restype = None
    lib.rips_barcode_cocycles.argtypes = [f32p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                          ctypes.c_float, ctypes.c_uint32,
                                          ctypes.POINTER(ctypes.POINTER(rips_cocycles))]
    lib.rips_barcode_cocycles.restype = ctypes.c_int
    lib.rips_cocycles_free.argtypes = [ctypes.POINTER(rips_cocycles)]
    lib.rips_cocycles_free.restype = None
    lib.rips_status_string.argtypes = [ctypes.c_int]
    lib.rips_status_string.restype = ctypes.c_char_p
    lib.rips_last_error.argtypes = []
    lib.rips_last_error.restype = ctypes.c_char_p
    lib.rips_barcode_device.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                        ctypes.c_int32, ctypes.c_float, ctypes.c_uint32,
                                        ctypes.POINTER(rips_device_out), ctypes.c_void_p]
    lib.rips_barcode_device.restype = ctypes.c_int
    lib.rips_barcode_device_noalloc.argtypes = lib.rips_barcode_device.argtypes
    lib.rips_barcode_device_noalloc.restype = ctypes.c_int
    lib.rips_simplex_counts_device.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                               ctypes.c_int32, ctypes.c_float,
                                               ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p]
    lib.rips_simplex_counts_device.restype = ctypes.c_int
    lib.rips_barcode_batched_device.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                                ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                                ctypes.c_float, ctypes.c_uint32,
                                                ctypes.POINTER(rips_batch_out), ctypes.c_void_p]
    lib.rips_barcode_batched_device.restype = ctypes.c_int
    lib.rips_backward_device.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                         ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    lib.rips_backward_device.restype = ctypes.c_int
    lib.rips_set_reduce_workgroups.argtypes = [ctypes.c_int32]
    lib.rips_set_reduce_workgroups.restype = ctypes.c_int
    lib.rips_get_reduce_workgroups.argtypes = [ctypes.POINTER(ctypes.c_int32)]
    lib.rips_get_reduce_workgroups.restype = ctypes.c_int
    lib.rips_set_shortcuts.argtypes = [ctypes.c_int32]
    lib.rips_set_shortcuts.restype = ctypes.c_int
    lib.rips_get_shortcuts.argtypes = [ctypes.POINTER(ctypes.c_int32)]
    lib.rips_get_shortcuts.restype = ctypes.c_int
    lib.rips_set_working_column.argtypes = [ctypes.c_int32]
    lib.rips_set_working_column.restype = ctypes.c_int
    lib.rips_get_working_column.argtypes = [ctypes.POINTER(ctypes.c_int32)]
    lib.rips_get_working_column.restype = ctypes.c_int
    lib.rips_set_reduced_storage.argtypes = [ctypes.c_int32]
    lib.rips_set_reduced_storage.restype = ctypes.c_int
    lib.rips_get_reduced_storage.argtypes = [ctypes.POINTER(ctypes.c_int32)]
    lib.rips_get_reduced_storage.restype = ctypes.c_int
    lib.rips_batched_set_config.argtypes = [ctypes.c_int32, ctypes.c_int32]
    lib.rips_batched_set_config.restype = ctypes.c_int
    lib.rips_batched_set_spread.argtypes = [ctypes.c_int32]
    lib.rips_batched_set_spread.restype = ctypes.c_int
    lib.rips_batched_get_config.argtypes = [ctypes.POINTER(ctypes.c_int32),
                                            ctypes.POINTER(ctypes.c_int32)]
    lib.rips_batched_get_config.restype = ctypes.c_int
    lib.rips_batched_autotune.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                          ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                          ctypes.c_float, ctypes.c_uint32,
                                          ctypes.POINTER(rips_batch_out), ctypes.c_void_p,
                                          ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                          ctypes.POINTER(ctypes.c_int32),
                                          ctypes.POINTER(ctypes.c_float)]
    lib.rips_batched_autotune.restype = ctypes.c_int
    lib.rips_profile_enable.argtypes = [ctypes.c_int]
    lib.rips_profile_enable.restype = None
    lib.rips_profile_count.argtypes = []
    lib.rips_profile_count.restype = ctypes.c_int
    lib.rips_profile_name.argtypes = [ctypes.c_int]
    lib.rips_profile_name.restype = ctypes.c_char_p
    lib.rips_profile_ms.argtypes = [ctypes.c_int]
    lib.rips_profile_ms.restype = ctypes.c_double
    lib.rips_profile_calls.argtypes = [ctypes.c_int]
    lib.rips_profile_calls.restype = ctypes.c_int64
    return lib


_lib = _load()


def lib():
    return _lib


def _check(status: int):
    if status != 0:
        raise RipsError(status, _lib.rips_last_error().decode())


@dataclass
class Bars:
    birth: np.ndarray
    death: np.ndarray
    birth_simplex: np.ndarray
    death_simplex: np.ndarray

    def __len__(self):
        return int(self.birth.shape[0])


@dataclass
class Result:
    n: int
    max_dim: int
    p: int
    sparse: bool
    threshold: float
    enclosing_radius: float
    bars: list
    stats: list
    simplex_count: list
    columns: list = field(default_factory=list)


def _stats_dict(s) -> dict:
    return {f: int(getattr(s, f)) for f in STAT_FIELDS}


def barcode(points: np.ndarray | None = None, *, dist: np.ndarray | None = None,
            max_dim: int = 1, threshold: float = float("inf"), p: int = 2) -> Result:
    """Barcode of a host point cloud (float32 (n, m)) or full distance matrix
    (float32 (n, n), entries i > j read) via the C ABI rips_barcode."""
    return _run_result(_lib.rips_barcode, points, dist, max_dim, threshold, p)


def barcode_homology(points: np.ndarray | None = None, *, dist: np.ndarray | None = None,
                     max_dim: int = 1, threshold: float = float("inf"), p: int = 2) -> Result:
    """The same barcode by the homology variant (rips_barcode_homology):
    boundary matrices reduced with clearing from the top dimension down, for
    the ablation against cohomology; max_dim <= 2. stats[d] counts the
    columns of the boundary of the (d+1)-simplices."""
    return _run_result(_lib.rips_barcode_homology, points, dist, max_dim, threshold, p)


def _run_result(entry, points, dist, max_dim, threshold, p) -> Result:
    if (points is None) == (dist is None):
        raise ValueError("give exactly one of points, dist")
    if points is not None:
        x = np.ascontiguousarray(points, dtype=np.float32)
        if x.ndim != 2:
            raise ValueError("points must be (n, m)")
        n, m = x.shape
    else:
        x = np.ascontiguousarray(dist, dtype=np.float32)
        if x.ndim != 2 or x.shape[0] != x.shape[1]:
            raise ValueError("dist must be (n, n)")
        n, m = x.shape[0], 0
    out = ctypes.POINTER(rips_result)()
    _check(entry(x.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), n, m, max_dim,
                 ctypes.c_float(threshold), p, ctypes.byref(out)))
    try:
        r = out.contents
        bars, stats, counts, cols = [], [], [], []
        for d in range(r.max_dim + 1):
            b = r.dims[d]
            c = int(b.count)

            def arr(ptr, dt):
                return np.ctypeslib.as_array(ptr, shape=(c,)).astype(dt, copy=True) if c else \
                    np.empty(0, dt)
            bars.append(Bars(arr(b.birth, np.float32), arr(b.death, np.float32),
                             arr(b.birth_simplex, np.int64), arr(b.death_simplex, np.int64)))
            stats.append(_stats_dict(r.stats[d]))
            counts.append(int(r.simplex_count[d]))
            nc = int(r.column_count[d])
            if nc:
                ci = np.ctypeslib.as_array(r.column_index[d], shape=(nc,)).copy()
                cd = np.ctypeslib.as_array(r.column_diam[d], shape=(nc,)).copy()
            else:
                ci, cd = np.empty(0, np.int64), np.empty(0, np.float32)
            cols.append((ci, cd))
        return Result(n=int(r.n), max_dim=int(r.max_dim), p=int(r.p), sparse=bool(r.sparse),
                      threshold=float(r.threshold_used),
                      enclosing_radius=float(r.enclosing_radius), bars=bars, stats=stats,
                      simplex_count=counts, columns=cols)
    finally:
        _lib.rips_result_free(out)


@dataclass
class Cocycles:
    bars: Bars
    cocycles: list  # per bar: (CNS indices of its simplices, coefficients in Z/p)


def cocycles(points: np.ndarray | None = None, *, dist: np.ndarray | None = None, dim: int = 1,
             threshold: float = float("inf"), p: int = 2) -> Cocycles:
    """Bars of dimension `dim` >= 1 with a representative cocycle each, via
    the C ABI rips_barcode_cocycles: `cocycles[b]` = (CNS indices of
    dim-simplices, coefficients in Z/p) of bar b."""
    if (points is None) == (dist is None):
        raise ValueError("give exactly one of points, dist")
    if points is not None:
        x = np.ascontiguousarray(points, dtype=np.float32)
        if x.ndim != 2:
            raise ValueError("points must be (n, m)")
        n, m = x.shape
    else:
        x = np.ascontiguousarray(dist, dtype=np.float32)
        if x.ndim != 2 or x.shape[0] != x.shape[1]:
            raise ValueError("dist must be (n, n)")
        n, m = x.shape[0], 0
    out = ctypes.POINTER(rips_cocycles)()
    _check(_lib.rips_barcode_cocycles(x.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), n, m, dim,
                                      ctypes.c_float(threshold), p, ctypes.byref(out)))
    try:
        r = out.contents
        c = int(r.count)

        def arr(ptr, k, dt):
            return np.ctypeslib.as_array(ptr, shape=(k,)).astype(dt, copy=True) if k else np.empty(0, dt)
        bars = Bars(arr(r.birth, c, np.float32), arr(r.death, c, np.float32),
                    arr(r.birth_simplex, c, np.int64), arr(r.death_simplex, c, np.int64))
        off = arr(r.offsets, c + 1, np.int64)
        ne = int(off[-1]) if c else 0
        simp, coef = arr(r.simplex, ne, np.int64), arr(r.coef, ne, np.uint32)
        cc = [(simp[off[b]:off[b + 1]], coef[off[b]:off[b + 1]]) for b in range(c)]
        return Cocycles(bars, cc)
    finally:
        _lib.rips_cocycles_free(out)


def _stream_ptr(torch, device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def barcode_device(x, *, max_dim: int = 1, threshold: float = float("inf"), p: int = 2,
                   is_distance: bool = False, cap: int | None = None, noalloc: bool = False):
    """Barcode of a device-resident float32 tensor (points (n, m), or a full
    (n, n) distance matrix with is_distance=True). Returns (bars, info):
    bars[d] = (birth, death, birth_simplex, death_simplex) torch.cuda tensors;
    info holds stats, simplex counts and the threshold used. noalloc=True
    calls rips_barcode_device_noalloc (the library allocates nothing; the
    output tensors are still allocated here, by the caller)."""
    import torch
    entry = _lib.rips_barcode_device_noalloc if noalloc else _lib.rips_barcode_device
    if not x.is_cuda or x.dtype != torch.float32 or not x.is_contiguous() or x.dim() != 2:
        raise ValueError("x must be a contiguous float32 CUDA tensor of rank 2")
    n = x.shape[0]
    m = 0 if is_distance else x.shape[1]
    dev = x.device
    cap = cap if cap is not None else max(64, n)
    while True:
        birth = torch.empty((max_dim + 1) * cap, dtype=torch.float32, device=dev)
        death = torch.empty_like(birth)
        bs = torch.empty((max_dim + 1) * cap, dtype=torch.int64, device=dev)
        ds = torch.empty_like(bs)
        o = rips_device_out()
        o.cap = cap
        o.birth, o.death = birth.data_ptr(), death.data_ptr()
        o.birth_simplex, o.death_simplex = bs.data_ptr(), ds.data_ptr()
        st = entry(ctypes.c_void_p(x.data_ptr()), n, m, max_dim, ctypes.c_float(threshold), p,
                   ctypes.byref(o), _stream_ptr(torch, dev))
        if st == -6 and o.needed_cap > cap:
            cap = int(o.needed_cap)
            continue
        _check(st)
        break
    bars = []
    for d in range(max_dim + 1):
        c = int(o.count[d])
        sl = slice(d * cap, d * cap + c)
        bars.append((birth[sl], death[sl], bs[sl], ds[sl]))
    info = dict(stats=[_stats_dict(o.stats[d]) for d in range(max_dim + 1)],
                simplex_count=[int(o.simplex_count[d]) for d in range(max_dim + 1)],
                threshold=float(o.threshold_used), sparse=bool(o.sparse))
    return bars, info


def simplex_counts(x, top: int, *, threshold: float = float("inf"), is_distance: bool = False):
    """|K_d| for d = 0..top at min(threshold, enclosing radius), on the GPU."""
    import torch
    if not x.is_cuda or x.dtype != torch.float32 or not x.is_contiguous():
        raise ValueError("x must be a contiguous float32 CUDA tensor")
    n = x.shape[0]
    m = 0 if is_distance else x.shape[1]
    counts = (ctypes.c_int64 * (top + 1))()
    _check(_lib.rips_simplex_counts_device(ctypes.c_void_p(x.data_ptr()), n, m, top,
                                           ctypes.c_float(threshold), counts,
                                           _stream_ptr(torch, x.device)))
    return [int(c) for c in counts]


def profile_enable(on: bool = True):
    """Start (clearing the totals) or stop per-kernel-class GPU timing."""
    _lib.rips_profile_enable(1 if on else 0)


def profile_read() -> dict:
    """{kernel class: (total ms, launches)} for the classes that ran."""
    out = {}
    for i in range(_lib.rips_profile_count()):
        c = int(_lib.rips_profile_calls(i))
        if c:
            out[_lib.rips_profile_name(i).decode()] = (float(_lib.rips_profile_ms(i)), c)
    return out


class BatchedBars:
    """Bars of a batch: flat device tensors plus offsets[(b, d)] segments."""

    def __init__(self, birth, death, birth_simplex, death_simplex, offsets, stats, thresholds,
                 B, max_dim):
        self.birth, self.death = birth, death
        self.birth_simplex, self.death_simplex = birth_simplex, death_simplex
        self.offsets, self.stats, self.thresholds = offsets, stats, thresholds
        self.B, self.max_dim = B, max_dim

    def segment(self, b: int, d: int):
        i = b * (self.max_dim + 1) + d
        lo, hi = int(self.offsets_host[i]), int(self.offsets_host[i + 1])
        return (self.birth[lo:hi], self.death[lo:hi], self.birth_simplex[lo:hi],
                self.death_simplex[lo:hi])

    @property
    def offsets_host(self):
        if not hasattr(self, "_off_host"):
            self._off_host = self.offsets.cpu().numpy()
        return self._off_host


def pack_clouds(clouds, device="cuda"):
    """Concatenate a list of (n_b, m) float32 arrays / tensors into the
    (points, offsets, n_max) triple the batched entry point takes."""
    import torch
    ts = [torch.as_tensor(c, dtype=torch.float32) for c in clouds]
    sizes = [int(t.shape[0]) for t in ts]
    offsets = torch.zeros(len(ts) + 1, dtype=torch.int64)
    offsets[1:] = torch.cumsum(torch.tensor(sizes, dtype=torch.int64), 0)
    x = torch.cat(ts, 0).contiguous().to(device)
    return x, offsets.to(device), max(sizes)


STATS_DTYPE = np.dtype([(f, np.int64) for f in STAT_FIELDS])


def barcode_batched(x, offsets, n_max: int, *, max_dim: int = 1,
                    threshold: float = float("inf"), p: int = 2, cap: int | None = None):
    """Barcodes of a batch of point clouds in one persistent launch (a cached
    hipGraph). x: (N, m) float32 CUDA tensor of all points; offsets: (B+1,)
    int64 CUDA tensor; n_max: bound on cloud sizes. Returns BatchedBars."""
    import torch
    if not x.is_cuda or x.dtype != torch.float32 or not x.is_contiguous() or x.dim() != 2:
        raise ValueError("x must be a contiguous float32 CUDA tensor of rank 2")
    if not offsets.is_cuda or offsets.dtype != torch.int64 or offsets.dim() != 1:
        raise ValueError("offsets must be an int64 CUDA tensor")
    B = offsets.shape[0] - 1
    D1 = max_dim + 1
    dev = x.device
    cap = cap if cap is not None else max(1024, 4 * int(n_max) * B)
    off = torch.empty(B * D1 + 1, dtype=torch.int64, device=dev)
    stats = torch.empty(B * D1 * len(STAT_FIELDS), dtype=torch.int64, device=dev)
    thr = torch.empty(B, dtype=torch.float32, device=dev)
    while True:
        birth = torch.empty(cap, dtype=torch.float32, device=dev)
        death = torch.empty_like(birth)
        bs = torch.empty(cap, dtype=torch.int64, device=dev)
        ds = torch.empty_like(bs)
        o = rips_batch_out()
        o.cap = cap
        o.birth, o.death = birth.data_ptr(), death.data_ptr()
        o.birth_simplex, o.death_simplex = bs.data_ptr(), ds.data_ptr()
        o.bar_offsets, o.stats, o.threshold_used = off.data_ptr(), stats.data_ptr(), thr.data_ptr()
        st = _lib.rips_barcode_batched_device(ctypes.c_void_p(x.data_ptr()),
                                              ctypes.c_void_p(offsets.data_ptr()), B,
                                              x.shape[1], int(n_max), max_dim,
                                              ctypes.c_float(threshold), p, ctypes.byref(o),
                                              _stream_ptr(torch, dev))
        if st == -6 and o.needed > cap:
            cap = int(o.needed)
            continue
        _check(st)
        break
    return BatchedBars(birth, death, bs, ds, off, stats.view(B, D1, len(STAT_FIELDS)), thr, B,
                       max_dim)


def set_reduce_workgroups(workgroups: int = 0):
    """Workgroups of the single-cloud reduction: 0 = one per compute unit,
    1 = one workgroup, columns one after another (same bars either way)."""
    _check(_lib.rips_set_reduce_workgroups(int(workgroups)))


def get_reduce_workgroups() -> int:
    a = ctypes.c_int32()
    _check(_lib.rips_get_reduce_workgroups(ctypes.byref(a)))
    return int(a.value)


SHORTCUT_APPARENT = 1
SHORTCUT_EMERGENT = 2
SHORTCUT_CLEARING = 4


def set_shortcuts(flags: int = SHORTCUT_APPARENT | SHORTCUT_EMERGENT | SHORTCUT_CLEARING):
    """Shortcuts of the single-cloud path (the ablation switches of the
    paper's Table 3): SHORTCUT_APPARENT skips zero apparent pairs,
    SHORTCUT_EMERGENT pairs emergent columns at once, SHORTCUT_CLEARING
    gives no column to a pivot of the dimension below. The bars are the same
    with any of them off."""
    _check(_lib.rips_set_shortcuts(int(flags)))


R_AUTO = 0
R_DISCARD = 1
R_STORE = 2
R_EXPLICIT = 3


def set_reduced_storage(mode: int = R_AUTO):
    """When the single-cloud path keeps R_j beside V_j (Table 3's "storing R"
    and "discarding R" rows): R_AUTO when cheaper to add, R_DISCARD never,
    R_STORE whenever it fits; R_EXPLICIT: explicit matrix reduction (the
    "explicit" column: every coboundary column built before the reduction,
    every reduced column stored and added). The bars are the same in every
    mode."""
    _check(_lib.rips_set_reduced_storage(int(mode)))


WORKING_COLUMN_AUTO = 0
WORKING_COLUMN_GENERAL = 1


def set_working_column(mode: int = WORKING_COLUMN_AUTO):
    """Working column of the dimension-1 reduction: WORKING_COLUMN_AUTO uses
    the direct-mapped one (one bit per longest edge and third vertex) where
    it applies (Z/2, every shortcut on) and fits; WORKING_COLUMN_GENERAL
    always the general one. The bars are the same either way."""
    _check(_lib.rips_set_working_column(int(mode)))


def get_working_column() -> int:
    a = ctypes.c_int32()
    _check(_lib.rips_get_working_column(ctypes.byref(a)))
    return int(a.value)


def get_reduced_storage() -> int:
    a = ctypes.c_int32()
    _check(_lib.rips_get_reduced_storage(ctypes.byref(a)))
    return int(a.value)


def get_shortcuts() -> int:
    a = ctypes.c_int32()
    _check(_lib.rips_get_shortcuts(ctypes.byref(a)))
    return int(a.value)


def batched_set_config(delta_slots: int = 0, workgroups_per_cu: int = 0):
    """Launch configuration of the batched path (0 = defaults)."""
    _check(_lib.rips_batched_set_config(int(delta_slots), int(workgroups_per_cu)))


def batched_set_spread(mode: int = 0):
    """Workgroups per cloud of the batched path: 0 (auto) spreads each cloud
    of a batch smaller than the chip over several workgroups, 1 keeps one
    workgroup per cloud. The bars are the same either way."""
    _check(_lib.rips_batched_set_spread(int(mode)))


def batched_get_config():
    a, b = ctypes.c_int32(), ctypes.c_int32()
    _check(_lib.rips_batched_get_config(ctypes.byref(a), ctypes.byref(b)))
    return int(a.value), int(b.value)


def batched_autotune(x, offsets, n_max: int, *, max_dim: int = 1,
                     threshold: float = float("inf"), p: int = 2, reps: int = 2,
                     cap: int | None = None):
    """Time every batched launch configuration on this batch and keep the
    fastest (rips_batched_autotune). Returns (delta_slots, workgroups_per_cu,
    ms per launch)."""
    import torch
    bb = barcode_batched(x, offsets, n_max, max_dim=max_dim, threshold=threshold, p=p, cap=cap)
    B = offsets.shape[0] - 1
    o = rips_batch_out()
    o.cap = bb.birth.shape[0]
    o.birth, o.death = bb.birth.data_ptr(), bb.death.data_ptr()
    o.birth_simplex, o.death_simplex = bb.birth_simplex.data_ptr(), bb.death_simplex.data_ptr()
    o.bar_offsets = bb.offsets.data_ptr()
    o.stats, o.threshold_used = None, None
    a, w, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_float()
    _check(_lib.rips_batched_autotune(ctypes.c_void_p(x.data_ptr()),
                                      ctypes.c_void_p(offsets.data_ptr()), B, x.shape[1],
                                      int(n_max), max_dim, ctypes.c_float(threshold), p,
                                      ctypes.byref(o), _stream_ptr(torch, x.device), int(reps),
                                      ctypes.byref(a), ctypes.byref(w), ctypes.byref(ms)))
    return int(a.value), int(w.value), float(ms.value)


def backward_scatter(x, n: int, dim: int, k_birth: int, birth_simplex, death_simplex,
                     grad_birth, grad_death, grad_out, row0=None):
    """rips_backward_device: grad_out += d(loss)/d(input) through the critical
    edges of the bars' birth and death simplices (device tensors)."""
    import torch
    nb = int(birth_simplex.shape[0])
    if nb == 0:
        return grad_out
    for t, dt in ((birth_simplex, torch.int64), (death_simplex, torch.int64),
                  (grad_birth, torch.float32), (grad_death, torch.float32)):
        if not t.is_cuda or t.dtype != dt or not t.is_contiguous() or t.shape[0] != nb:
            raise ValueError("bar tensors must be contiguous CUDA tensors of one length")
    if row0 is not None and (row0.dtype != torch.int64 or not row0.is_contiguous()):
        raise ValueError("row0 must be a contiguous int64 CUDA tensor")
    _check(_lib.rips_backward_device(
        ctypes.c_void_p(x.data_ptr()), int(n), int(dim), nb, int(k_birth),
        ctypes.c_void_p(row0.data_ptr() if row0 is not None else 0),
        ctypes.c_void_p(birth_simplex.data_ptr()), ctypes.c_void_p(death_simplex.data_ptr()),
        ctypes.c_void_p(grad_birth.data_ptr()), ctypes.c_void_p(grad_death.data_ptr()),
        ctypes.c_void_p(grad_out.data_ptr()), _stream_ptr(torch, x.device)))
    return grad_out


from .autograd import Bars, diagram, batched_diagram, top_persistence_loss  # noqa: E402,F401
