"""The oracle -- TEST INFRASTRUCTURE ONLY.

A plain, slow, explicit CPU computation of Vietoris-Rips persistence barcodes
(Bauer, arXiv:1908.02518), written from the paper and used only by the tests,
the smoke check and the CPU-baseline leg of the benchmark. The GPU library
never imports, links or calls anything in this package, and this package
never touches the GPU library.

* ``rips_oracle.c``  -- explicit simplex lists, explicit coboundary matrices,
  Algorithm 2 (clearing) over Z/p in increasing dimension (cohomology), the
  apparent pairs from their definition, and a homology cross-check
  (Algorithm 1 on the explicit boundary matrices).
* ``bruteforce.py`` -- persistence pairs from ranks of lower-left submatrices
  (pairing-uniqueness), for inputs of at most ~10 points.
* ``gradient.py``   -- float64 chain rule of a bar loss through critical edges.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rips_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2 -ffp-contract=off, IEEE float32)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
               "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
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
    lib.oracle_distances.argtypes = [f32p, ctypes.c_int64, ctypes.c_int64, f32p]
    lib.oracle_distances.restype = None
    lib.oracle_run.argtypes = [f32p, ctypes.c_int32, ctypes.c_int32, ctypes.c_float,
                               ctypes.c_uint32, ctypes.c_int32, ctypes.c_int32]
    lib.oracle_run.restype = P
    lib.oracle_free.argtypes = [P]
    lib.oracle_error.argtypes = [P]
    lib.oracle_error.restype = ctypes.c_char_p
    lib.oracle_threshold.argtypes = [P]
    lib.oracle_threshold.restype = ctypes.c_float
    lib.oracle_enclosing_radius.argtypes = [P]
    lib.oracle_enclosing_radius.restype = ctypes.c_float
    for name in ("oracle_simplex_count", "oracle_num_bars", "oracle_num_columns",
                 "oracle_num_pairs", "oracle_num_essential", "oracle_num_hom_pairs",
                 "oracle_num_hom_essential", "oracle_num_apparent"):
        fn = getattr(lib, name)
        fn.argtypes = [P, ctypes.c_int]
        fn.restype = ctypes.c_int64
    lib.oracle_counters.argtypes = [P, ctypes.c_int, i64p]
    lib.oracle_get_bars.argtypes = [P, ctypes.c_int, f32p, f32p, i64p, i64p]
    lib.oracle_get_columns.argtypes = [P, ctypes.c_int, i64p, f32p]
    lib.oracle_get_pairs.argtypes = [P, ctypes.c_int, i64p, i64p, i64p]
    lib.oracle_get_hom_pairs.argtypes = [P, ctypes.c_int, i64p, i64p, i64p]
    lib.oracle_get_apparent.argtypes = [P, ctypes.c_int, i64p, i64p]
    i32p = ctypes.POINTER(ctypes.c_int32)
    lib.oracle_cns_index.argtypes = [i32p, ctypes.c_int32]
    lib.oracle_cns_index.restype = ctypes.c_int64
    lib.oracle_filtration.argtypes = [f32p, ctypes.c_int32, ctypes.c_int32, ctypes.c_float,
                                      i32p, i64p, f32p, ctypes.c_int64]
    lib.oracle_filtration.restype = ctypes.c_int64
    _lib = lib
    return lib


def _f32p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def _i64p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def distances(points: np.ndarray) -> np.ndarray:
    """Lower triangle (i > j, row-major) of the float32 Euclidean distance matrix."""
    lib = _load()
    x = np.ascontiguousarray(points, dtype=np.float32)
    n, m = x.shape
    out = np.empty(n * (n - 1) // 2, dtype=np.float32)
    lib.oracle_distances(_f32p(x), n, m, _f32p(out))
    return out


def lower_from_full(dist: np.ndarray) -> np.ndarray:
    """Lower triangle (i > j) of a full square float32 matrix."""
    d = np.asarray(dist, dtype=np.float32)
    n = d.shape[0]
    ii, jj = np.tril_indices(n, -1)
    return np.ascontiguousarray(d[ii, jj])


def cns_index(vertices) -> int:
    """CNS index the oracle assigns to a simplex (vertices in any order)."""
    lib = _load()
    v = np.ascontiguousarray(sorted(vertices, reverse=True), dtype=np.int32)
    return int(lib.oracle_cns_index(v.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                    len(v) - 1))


def filtration(points: np.ndarray, top: int, threshold: float = float("inf")):
    """All simplices of dims <= top with diam <= threshold (no clamp), in the
    refined order. Returns (dims, cns indices, diameters)."""
    lib = _load()
    dl = distances(points)
    n = int(points.shape[0])
    if dl.shape[0] == 0:
        dl = np.zeros(1, dtype=np.float32)
    total = lib.oracle_filtration(_f32p(dl), n, top, ctypes.c_float(threshold), None, None,
                                  None, 0)
    dims = np.empty(total, np.int32)
    idx = np.empty(total, np.int64)
    diam = np.empty(total, np.float32)
    lib.oracle_filtration(_f32p(dl), n, top, ctypes.c_float(threshold),
                          dims.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _i64p(idx),
                          _f32p(diam), total)
    return dims, idx, diam


@dataclass
class Bars:
    birth: np.ndarray
    death: np.ndarray
    birth_simplex: np.ndarray
    death_simplex: np.ndarray

    def __len__(self):
        return int(self.birth.shape[0])


@dataclass
class OracleResult:
    n: int
    max_dim: int
    p: int
    threshold: float
    enclosing_radius: float
    counts: list            # |K_k|, k = 0..max_dim+1
    bars: list              # Bars per dimension
    columns: list           # (idx, diam) per dimension, reduction order
    counters: list          # dict per dimension
    pairs: list             # (lo, hi, essential) per dimension, CNS indices
    apparent: list = field(default_factory=list)   # (lo, hi) per dimension, any persistence
    hom_pairs: list = field(default_factory=list)


def barcode(points: np.ndarray | None = None, *, dist_lower: np.ndarray | None = None,
            max_dim: int = 1, threshold: float = float("inf"), p: int = 2,
            clamp: bool = True, homology: bool = False) -> OracleResult:
    """Run the oracle on a point cloud (float32, (n, m)) or a lower-triangle
    distance vector. Returns bars in canonical order (birth asc, then birth
    simplex CNS index desc)."""
    lib = _load()
    if dist_lower is None:
        dl = distances(points)
        n = int(np.asarray(points).shape[0])
    else:
        dl = np.ascontiguousarray(dist_lower, dtype=np.float32)
        n = int(round((1 + np.sqrt(1 + 8 * dl.shape[0])) / 2)) if dl.shape[0] else 1
        if n * (n - 1) // 2 != dl.shape[0]:
            raise ValueError("dist_lower has no triangular length")
    if dl.shape[0] == 0:
        dl = np.zeros(1, dtype=np.float32)
    h = lib.oracle_run(_f32p(dl), n, max_dim, ctypes.c_float(threshold), p,
                       1 if clamp else 0, 1 if homology else 0)
    if not h:
        raise MemoryError("oracle_run")
    try:
        err = lib.oracle_error(h).decode()
        if err:
            raise ValueError(err)
        counts = [int(lib.oracle_simplex_count(h, k)) for k in range(max_dim + 2)]
        bars, cols, ctrs, pairs, hom, app = [], [], [], [], [], []
        for k in range(max_dim + 1):
            nb = lib.oracle_num_bars(h, k)
            b = np.empty(nb, np.float32)
            d = np.empty(nb, np.float32)
            bs = np.empty(nb, np.int64)
            ds = np.empty(nb, np.int64)
            if nb:
                lib.oracle_get_bars(h, k, _f32p(b), _f32p(d), _i64p(bs), _i64p(ds))
            bars.append(Bars(b, d, bs, ds))
            nc = lib.oracle_num_columns(h, k)
            ci = np.empty(nc, np.int64)
            cd = np.empty(nc, np.float32)
            if nc:
                lib.oracle_get_columns(h, k, _i64p(ci), _f32p(cd))
            cols.append((ci, cd))
            c6 = np.zeros(6, np.int64)
            lib.oracle_counters(h, k, _i64p(c6))
            ctrs.append(dict(cleared=int(c6[0]), zero_apparent_col=int(c6[1]),
                             zero_apparent_piv=int(c6[2]), reduced_columns=int(c6[3]),
                             pairs=int(c6[4]), essential=int(c6[5])))
            npr = lib.oracle_num_pairs(h, k)
            ne = lib.oracle_num_essential(h, k)
            lo = np.empty(npr, np.int64)
            hi = np.empty(npr, np.int64)
            es = np.empty(ne, np.int64)
            lib.oracle_get_pairs(h, k, _i64p(lo), _i64p(hi), _i64p(es))
            pairs.append((lo, hi, es))
            na = lib.oracle_num_apparent(h, k)
            alo = np.empty(na, np.int64)
            ahi = np.empty(na, np.int64)
            if na:
                lib.oracle_get_apparent(h, k, _i64p(alo), _i64p(ahi))
            app.append((alo, ahi))
            if homology:
                hp = lib.oracle_num_hom_pairs(h, k)
                he = lib.oracle_num_hom_essential(h, k)
                hlo = np.empty(hp, np.int64)
                hhi = np.empty(hp, np.int64)
                hes = np.empty(he, np.int64)
                lib.oracle_get_hom_pairs(h, k, _i64p(hlo), _i64p(hhi), _i64p(hes))
                hom.append((hlo, hhi, hes))
        return OracleResult(n=n, max_dim=max_dim, p=p,
                            threshold=float(lib.oracle_threshold(h)),
                            enclosing_radius=float(lib.oracle_enclosing_radius(h)),
                            counts=counts, bars=bars, columns=cols, counters=ctrs,
                            pairs=pairs, apparent=app, hom_pairs=hom)
    finally:
        lib.oracle_free(h)
