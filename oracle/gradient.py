"""Reference gradient of a bar loss -- TEST INFRASTRUCTURE ONLY (part of the oracle).

The paper does not differentiate barcodes. The reading used here: each bar
endpoint equals the length of one edge of its simplex, the *critical edge*,
i.e. the edge of maximal float32 length, ties broken by the smallest CNS
edge index (the youngest such edge in the refined order, the one whose
arrival gives the simplex its diameter). With d(u, v) = ||x_u - x_v||,
d d / d x_u = (x_u - x_v) / d and d d / d x_v = -(x_u - x_v) / d. Vertex
(H0) births and infinite deaths contribute nothing.

Everything here is float64 numpy, applied to the pairing computed by the
oracle.
"""

from __future__ import annotations

import math

import numpy as np


def decode(idx: int, k: int, n: int):
    """Vertices (decreasing) of the k-simplex with CNS index idx: the largest
    vertex is the largest i with C(i, k+1) <= idx (Lemma of the 'Vertices and
    simplices' paragraph), then recurse on idx - C(i, k+1)."""
    out = []
    hi = n - 1
    for l in range(k, -1, -1):
        i = hi
        while math.comb(i, l + 1) > idx:
            i -= 1
        out.append(i)
        idx -= math.comb(i, l + 1)
        hi = i - 1
    return out


def critical_edge(points32: np.ndarray, idx: int, k: int):
    """(u, v), u > v: the edge of the k-simplex with the largest float32
    length, ties to the smallest CNS edge index."""
    from . import distances  # float32 distances, same arithmetic as the oracle
    n = points32.shape[0]
    vs = decode(int(idx), k, n)
    best = None
    for a in range(len(vs)):
        for b in range(a + 1, len(vs)):
            u, v = vs[a], vs[b]  # u > v
            x = points32[[u, v]]
            d = distances(x)[0]
            key = (-float(d), math.comb(u, 2) + v)
            if best is None or key < best[0]:
                best = (key, (u, v))
    return best[1]


def top_bars(birth: np.ndarray, death: np.ndarray, bsimp: np.ndarray, top: int = 5):
    """Indices of the `top` finite bars of largest float32 persistence, ties
    broken by the refined order of the birth simplex (birth asc, then birth
    simplex CNS index desc)."""
    fin = np.isfinite(death)
    idx = np.nonzero(fin)[0]
    pers = (death[idx].astype(np.float32) - birth[idx].astype(np.float32)).astype(np.float32)
    order = sorted(range(len(idx)),
                   key=lambda i: (-float(pers[i]), float(birth[idx[i]]), -int(bsimp[idx[i]])))
    return idx[order[:top]]


def loss_and_grad(points32: np.ndarray, bars_dim, dim: int = 1, top: int = 5):
    """L = sum over the top bars of dimension `dim` of (death - birth)^2, and
    dL/dx in float64 through the critical edges of the birth and death
    simplices. bars_dim: object with birth, death, birth_simplex,
    death_simplex arrays (canonical order)."""
    x64 = points32.astype(np.float64)
    g = np.zeros_like(x64)
    sel = top_bars(bars_dim.birth, bars_dim.death, bars_dim.birth_simplex, top)
    L = 0.0
    for i in sel:
        b, d = float(bars_dim.birth[i]), float(bars_dim.death[i])
        L += (d - b) ** 2
        for simp, k, coef in ((bars_dim.birth_simplex[i], dim, -2.0 * (d - b)),
                              (bars_dim.death_simplex[i], dim + 1, 2.0 * (d - b))):
            if k == 0 or simp < 0:
                continue
            u, v = critical_edge(points32, int(simp), k)
            diff = x64[u] - x64[v]
            nrm = np.linalg.norm(diff)
            if nrm == 0.0:
                continue
            g[u] += coef * diff / nrm
            g[v] -= coef * diff / nrm
    return L, g, sel
