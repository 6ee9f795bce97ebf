"""Representative cocycles (rips_barcode_cocycles) checked by the properties
that define them, at any size: for the bar born at the d-simplex sigma_j and
dying at tau, the cochain V_j holds sigma_j with coefficient 1, nothing older
than sigma_j, and the oldest simplex of its coboundary is tau (so V_j is a
cocycle on every simplex older than tau); for an essential bar, V_j is a
cocycle. The coboundary is computed here from the combinatorial number system
and the oracle's float32 distances, with the orientation sign (-1)^(vertices
below the added one). The bars must equal rips_barcode's."""

from math import comb

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu
INF = float("inf")


def rips():
    import paper_1908_02518_amd as r
    return r


def full_distances(x):
    n = x.shape[0]
    dl = oracle.distances(x)
    D = np.zeros((n, n), np.float32)
    i, j = np.tril_indices(n, -1)
    D[i, j] = dl
    D[j, i] = dl
    return D


def decode(idx, k):
    """Vertices (decreasing) of the k-simplex with CNS index idx."""
    v = []
    for l in range(k, -1, -1):
        x = l
        while comb(x + 1, l + 1) <= idx:
            x += 1
        v.append(x)
        idx -= comb(x, l + 1)
    return v


def diam(D, v):
    return max((D[a, b] for a in v for b in v if a > b), default=np.float32(0.0))


class Coboundary:
    """delta of a d-cochain on the Rips complex at threshold t, over Z/p."""

    def __init__(self, D, d, t, p):
        self.D, self.d, self.t, self.p = D, d, np.float32(t), p
        n = D.shape[0]
        self.B = np.array([[comb(v, r) for r in range(d + 3)] for v in range(n)], dtype=np.int64)

    def __call__(self, simplices, coefs):
        D, d, p, B = self.D, self.d, self.p, self.B
        n = D.shape[0]
        js = np.arange(n)
        keys, vals, dias = [], [], []
        for s, a in zip(simplices, coefs):
            v = decode(int(s), d)
            ds = np.float32(diam(D, v))
            nd = np.maximum(ds, D[v, :].max(axis=0))
            ok = nd <= self.t
            ok[v] = False
            j = js[ok]
            above = (np.array(v)[None, :] > j[:, None]).sum(axis=1)
            s_above = np.zeros(d + 2, np.int64)
            s_below = np.zeros(d + 2, np.int64)
            for q in range(d + 2):
                s_above[q] = sum(comb(v[m], d + 2 - m) for m in range(q))
                s_below[q] = sum(comb(v[m], d + 1 - m) for m in range(q, d + 1))
            tau = s_above[above] + B[j, d + 2 - above] + s_below[above]
            sign = np.where((d + 1 - above) % 2 == 1, p - 1, 1).astype(np.int64)
            keys.append(tau)
            vals.append(sign * int(a) % p)
            dias.append(nd[ok])
        if not keys:
            return np.empty(0, np.int64), np.empty(0, np.int64), np.empty(0, np.float32)
        k = np.concatenate(keys)
        val = np.concatenate(vals)
        dia = np.concatenate(dias)
        uk, inv = np.unique(k, return_inverse=True)
        tot = np.zeros(len(uk), np.int64)
        np.add.at(tot, inv, val)
        tot %= p
        ud = np.zeros(len(uk), np.float32)
        ud[inv] = dia
        live = tot != 0
        return uk[live], tot[live], ud[live]


CASES = [
    ("rectangle-p3", lambda: workloads.rectangle(), 1, INF, 3, None),
    ("hexagon", lambda: workloads.regular_polygon(6), 1, INF, 2, None),
    ("cube-40-p5-d1", lambda: workloads.uniform_cube(40, 3, 31), 1, INF, 5, None),
    ("cube-40-p5-d2", lambda: workloads.uniform_cube(40, 3, 31), 2, INF, 5, None),
    ("lattice-ties-d2", lambda: workloads.integer_lattice(27, 3, 5, side=3), 2, INF, 2, None),
    ("sphere-100", lambda: workloads.config(1)["clouds"][0], 1, INF, 2, None),
    ("so3-1000-d1", lambda: workloads.config(2)["clouds"][0], 1, 1.4, 2, 60),
    ("so3-1000-d2", lambda: workloads.config(2)["clouds"][0], 2, 1.4, 2, 60),
    ("torus4-2000-d1-p3", lambda: workloads.config(3)["clouds"][0], 1, 0.5, 3, 60),
    ("torus4-2000-d2-p3", lambda: workloads.config(3)["clouds"][0], 2, 0.5, 3, 60),
]


@pytest.mark.parametrize("name,make,d,t,p,sample", CASES, ids=[c[0] for c in CASES])
def test_cocycle_properties(name, make, d, t, p, sample):
    r = rips()
    x = make()
    print(f"[case] cocycles {name}", flush=True)
    full = r.barcode(x, max_dim=d, threshold=t, p=p)
    got = r.cocycles(x, dim=d, threshold=t, p=p)
    for f in ("birth", "death", "birth_simplex", "death_simplex"):
        assert np.array_equal(getattr(got.bars, f), getattr(full.bars[d], f)), (name, f)
    nb = len(got.bars.birth)
    assert len(got.cocycles) == nb
    D = full_distances(x)
    delta = Coboundary(D, d, full.threshold, p)
    bars = range(nb)
    if sample is not None and nb > sample:
        # the longest bars and every essential one, then an even spread
        pers = got.bars.death - got.bars.birth
        order = list(np.argsort(-pers, kind="stable")[:sample // 2])
        order += list(range(0, nb, max(1, nb // (sample // 2))))
        bars = sorted(set(int(b) for b in order))
    for b in bars:
        simp, coef = got.cocycles[b]
        bs, ds = int(got.bars.birth_simplex[b]), int(got.bars.death_simplex[b])
        birth, death = got.bars.birth[b], got.bars.death[b]
        assert len(simp) == len(np.unique(simp)), (name, b, "repeated simplex")
        assert np.all((coef > 0) & (coef < p)), (name, b)
        at = np.nonzero(simp == bs)[0]
        assert len(at) == 1 and coef[at[0]] == 1, (name, b, "birth simplex")
        # nothing older than sigma_j in the refined order (diameter, then
        # larger index older): V_j adds only columns reduced before j, which
        # are younger
        for s in simp:
            ds_ = diam(D, decode(int(s), d))
            assert ds_ > birth or (ds_ == birth and int(s) <= bs), (name, b, "older simplex")
        tk, tv, td = delta(simp, coef)
        if ds < 0:
            assert len(tk) == 0, (name, b, "essential cocycle has a coboundary")
        else:
            assert len(tk) > 0, (name, b)
            oldest = np.lexsort((-tk, td))[0]  # smallest diameter, then largest index
            assert tk[oldest] == ds, (name, b, "death simplex")
            assert td[oldest] == death, (name, b, "death value")
