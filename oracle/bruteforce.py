"""Brute-force persistence from ranks -- TEST INFRASTRUCTURE ONLY (part of the oracle).

Independent of ``rips_oracle.c``: no matrix reduction algorithm, no clearing,
no cohomology. For a simplexwise filtration the persistence pairs are fixed by
ranks of lower-left submatrices of the filtration boundary matrix (the
pairing-uniqueness statement behind the paper's Proposition on persistence
pairs): with r(i, j) the rank over Z/p of the submatrix of the d-boundary
matrix with rows >= i and columns <= j (rows and columns in filtration order),
(sigma_i, tau_j) is a persistence pair iff

    r(i, j) - r(i+1, j) - r(i, j-1) + r(i+1, j-1) = 1.

Essential simplices are those in no pair. Everything here is plain Python
(math.comb, itertools.combinations, Gaussian elimination with the topmost
pivot), sized for at most ~10 points.
"""

from __future__ import annotations

import itertools
import math

import numpy as np


def cns(vertices) -> int:
    """Combinatorial number system index of a simplex (any vertex order)."""
    vs = sorted(vertices)
    return sum(math.comb(v, l + 1) for l, v in enumerate(vs))


def full_matrix(dist_lower: np.ndarray, n: int) -> np.ndarray:
    d = np.zeros((n, n), dtype=np.float32)
    k = 0
    for i in range(1, n):
        for j in range(i):
            d[i, j] = d[j, i] = dist_lower[k]
            k += 1
    return d


def filtration(d: np.ndarray, max_dim: int, t: float):
    """All simplices of dims 0..max_dim+1 with diam <= t, as tuples
    (diam, dim, -cns, vertices) sorted in the refined order."""
    n = d.shape[0]
    out = []
    for k in range(max_dim + 2):
        for vs in itertools.combinations(range(n), k + 1):
            diam = np.float32(0.0)
            for a, b in itertools.combinations(vs, 2):
                diam = max(diam, d[a, b])
            if diam <= np.float32(t):
                out.append((float(diam), k, -cns(vs), vs))
    out.sort(key=lambda s: (s[0], s[1], s[2]))
    return out


def _rank_table(B: list, nrows: int, ncols: int, p: int) -> np.ndarray:
    """r[i][j+1] = rank of B[i:, :j+1] over Z/p, for 0 <= i <= nrows, -1 <= j < ncols."""
    r = np.zeros((nrows + 1, ncols + 1), dtype=np.int64)
    for i in range(nrows):
        basis = {}  # topmost nonzero row -> row vector (list) over rows i..nrows-1
        rank = 0
        for j in range(ncols):
            v = [B[row][j] % p for row in range(i, nrows)]
            # eliminate with the basis, topmost pivot first
            while True:
                top = next((q for q, x in enumerate(v) if x), None)
                if top is None or top not in basis:
                    break
                w = basis[top]
                f = v[top] * pow(w[top], p - 2, p) % p
                v = [(a - f * b) % p for a, b in zip(v, w)]
            if top is not None:
                basis[top] = v
                rank += 1
            r[i, j + 1] = rank
    return r


def pairs(points=None, *, dist_lower=None, max_dim: int = 1, threshold: float = math.inf,
          p: int = 2):
    """Persistence pairs and essential simplices of the refined Rips filtration
    (threshold used as given, no clamp). Returns per dimension k:
    (set of (birth cns, death cns), set of essential cns, list of (birth diam,
    death diam))."""
    if dist_lower is None:
        from . import distances
        dist_lower = distances(points)
        n = points.shape[0]
    else:
        n = int(round((1 + math.sqrt(1 + 8 * len(dist_lower))) / 2))
    d = full_matrix(dist_lower, n)
    filt = filtration(d, max_dim, threshold)
    by_dim = [[s for s in filt if s[1] == k] for k in range(max_dim + 2)]
    paired = [set() for _ in range(max_dim + 2)]
    result = []
    for k in range(max_dim + 1):
        rows, cols = by_dim[k], by_dim[k + 1]
        pos = {s[3]: i for i, s in enumerate(rows)}
        B = [[0] * len(cols) for _ in rows]
        for j, s in enumerate(cols):
            vs = s[3]  # increasing
            for m in range(len(vs)):
                face = vs[:m] + vs[m + 1:]
                B[pos[face]][j] = (-1) ** m % p
        r = _rank_table(B, len(rows), len(cols), p)
        prs, bars = set(), []
        for i in range(len(rows)):
            for j in range(len(cols)):
                mu = r[i, j + 1] - r[i + 1, j + 1] - r[i, j] + r[i + 1, j]
                if mu == 1:
                    prs.add((-rows[i][2], -cols[j][2]))
                    paired[k].add(i)
                    paired[k + 1].add(j)
                    bars.append((rows[i][0], cols[j][0]))
        result.append([prs, None, bars])
    for k in range(max_dim + 1):
        ess = {-s[2] for i, s in enumerate(by_dim[k]) if i not in paired[k]}
        result[k][1] = ess
    return [tuple(x) for x in result]


def betti_curve_check(points=None, *, dist_lower=None, max_dim: int = 1,
                      threshold: float = math.inf, p: int = 2):
    """For each distinct diameter r <= threshold, the Betti numbers
    beta_k(r) = dim C_k(r) - rank d_k(r) - rank d_{k+1}(r) of Rips_r over Z/p,
    k = 0..max_dim. Returns (radii, array [len(radii), max_dim+1])."""
    if dist_lower is None:
        from . import distances
        dist_lower = distances(points)
        n = points.shape[0]
    else:
        n = int(round((1 + math.sqrt(1 + 8 * len(dist_lower))) / 2))
    d = full_matrix(dist_lower, n)
    filt = filtration(d, max_dim, threshold)
    radii = sorted({s[0] for s in filt})

    def rank_mod(M):
        M = [row[:] for row in M]
        rk, ncol = 0, len(M[0]) if M else 0
        for c in range(ncol):
            piv = next((r for r in range(rk, len(M)) if M[r][c] % p), None)
            if piv is None:
                continue
            M[rk], M[piv] = M[piv], M[rk]
            inv = pow(M[rk][c], p - 2, p)
            M[rk] = [x * inv % p for x in M[rk]]
            for r in range(len(M)):
                if r != rk and M[r][c] % p:
                    f = M[r][c]
                    M[r] = [(a - f * b) % p for a, b in zip(M[r], M[rk])]
            rk += 1
        return rk

    out = np.zeros((len(radii), max_dim + 1), dtype=np.int64)
    for ri, rad in enumerate(radii):
        cx = [[s[3] for s in filt if s[1] == k and s[0] <= rad] for k in range(max_dim + 2)]
        ranks = [0] * (max_dim + 3)
        for k in range(1, max_dim + 2):
            rows, cols = cx[k - 1], cx[k]
            if not rows or not cols:
                continue
            pos = {v: i for i, v in enumerate(rows)}
            M = [[0] * len(cols) for _ in rows]
            for j, vs in enumerate(cols):
                for m in range(len(vs)):
                    M[pos[vs[:m] + vs[m + 1:]]][j] = (-1) ** m % p
            ranks[k] = rank_mod(M)
        for k in range(max_dim + 1):
            out[ri, k] = len(cx[k]) - ranks[k] - ranks[k + 1]
    return radii, out
