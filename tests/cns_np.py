"""Host-side helpers for checks at sizes the oracle cannot take whole:
vectorised decoding of combinatorial-number-system indices (section
"Vertices and simplices"), float32 distances between given vertex pairs
written out from their definition, and the restriction of a barcode to a
prefix of the filtration. Test infrastructure only; numpy, no GPU."""

from __future__ import annotations

import math

import numpy as np


def binom_table(n: int, r: int) -> np.ndarray:
    return np.array([math.comb(i, r) for i in range(n + 1)], dtype=np.int64)


def decode(idx, k: int, n: int) -> np.ndarray:
    """Vertices (decreasing) of the k-simplices with CNS indices idx: the
    largest vertex of an r-vertex simplex is the largest i with C(i, r) <=
    index; then the rest recursively. Shape (len(idx), k + 1)."""
    rem = np.array(idx, dtype=np.int64).reshape(-1)
    verts = []
    for r in range(k + 1, 0, -1):
        tab = binom_table(n, r)
        v = np.searchsorted(tab, rem, side="right") - 1
        verts.append(v)
        rem = rem - tab[v]
    return np.stack(verts, axis=1) if verts else np.zeros((len(rem), 0), np.int64)


def index_of(verts: np.ndarray, n: int) -> np.ndarray:
    """CNS indices of simplices given by decreasing vertex rows."""
    k = verts.shape[1] - 1
    s = np.zeros(verts.shape[0], dtype=np.int64)
    for m in range(k + 1):
        s += binom_table(n, k - m + 1)[verts[:, m]]
    return s


def pair_dist(x: np.ndarray, a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """float32 distances between rows a and b of x: the squared differences
    summed in coordinate order, each step rounded to float32, then the
    correctly rounded square root."""
    x = np.asarray(x, dtype=np.float32)
    s = np.zeros(len(a), dtype=np.float32)
    for c in range(x.shape[1]):
        t = x[a, c] - x[b, c]
        s = s + t * t
    return np.sqrt(s)


def diameters(x: np.ndarray, verts: np.ndarray) -> np.ndarray:
    """Largest pairwise float32 distance of each vertex row (0 for a vertex)."""
    out = np.zeros(verts.shape[0], dtype=np.float32)
    for i in range(verts.shape[1]):
        for j in range(i + 1, verts.shape[1]):
            out = np.maximum(out, pair_dist(x, verts[:, i], verts[:, j]))
    return out


def restrict_to_prefix(birth, death, bs, ds, r: float):
    """The bars of the filtration cut at diameter r (the simplices of
    diameter <= r form a prefix of the refined order, so the pairs inside it
    are the pairs of the cut filtration): bars born after r vanish, bars
    alive at r become essential. Returned in the canonical order (birth
    ascending, then birth simplex index descending)."""
    birth, death = np.asarray(birth, np.float32), np.asarray(death, np.float32)
    bs, ds = np.asarray(bs, np.int64), np.asarray(ds, np.int64)
    r32 = np.float32(r)
    keep = birth <= r32
    b, d, s, t = birth[keep], death[keep].copy(), bs[keep], ds[keep].copy()
    alive = d > r32
    d[alive] = np.inf
    t[alive] = -1
    order = np.lexsort((-s, b))
    return b[order], d[order], s[order], t[order]
