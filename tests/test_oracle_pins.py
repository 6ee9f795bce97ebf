"""Pins of the oracle against what the paper and the mathematics fix.

None of these tests compares the oracle with itself: each checks a printed
value of the paper (fixtures under tests/golden/), a closed form, an
invariant, a special case that reduces to a library routine, or the
independent rank-based brute force (oracle/bruteforce.py).
"""

import math

import numpy as np
import pytest
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import connected_components, minimum_spanning_tree

import oracle
import workloads
from oracle import bruteforce
from tests import golden_io

INF = float("inf")


def full_dist(points):
    dl = oracle.distances(points)
    return bruteforce.full_matrix(dl, points.shape[0])


# --------------------------------------------------------------------------
# distances
# --------------------------------------------------------------------------

def test_distances_exact_special_values():
    # integer Pythagorean distances are exact in float32
    d = full_dist(workloads.rectangle())
    assert d[1, 0] == 3.0 and d[2, 0] == 4.0 and d[3, 0] == 5.0
    assert d[3, 2] == 3.0 and d[3, 1] == 4.0 and d[2, 1] == 5.0
    # sqrt(2) correctly rounded to float32 is 0x3FB504F3
    x = np.array([[0, 0], [1, 1]], np.float32)
    assert oracle.distances(x)[0].view(np.uint32) == 0x3FB504F3


def test_distances_correctly_rounded_sqrt():
    # each distance is the float32 nearest to sqrt of the float32 sum of squares
    g = workloads.rng(7)
    x = g.standard_normal((40, 5)).astype(np.float32)
    dl = oracle.distances(x)
    k = 0
    for i in range(1, 40):
        for j in range(i):
            s = np.float32(0)
            for c in range(5):
                t = np.float32(x[i, c] - x[j, c])
                s = np.float32(s + np.float32(t * t))
            exact = math.sqrt(float(s))
            cand = np.float32(exact)
            lo, hi = np.nextafter(cand, np.float32(-1)), np.nextafter(cand, np.float32(INF))
            best = min((abs(float(c) - exact), c) for c in (lo, cand, hi))[1]
            assert dl[k] == best
            k += 1


# --------------------------------------------------------------------------
# combinatorial number system
# --------------------------------------------------------------------------

def test_cns_values_from_paper():
    vals, cof, _ = golden_io.cns()
    for s, v in vals.items():
        assert oracle.cns_index(s) == v
    s, n, expect = cof
    got = [oracle.cns_index((j,) + s) if j > s[0] else oracle.cns_index(
        tuple(sorted(s + (j,), reverse=True))) for j in range(n - 1, -1, -1) if j not in s]
    assert got == expect


def test_cns_bijection_small():
    n = 9
    for k in range(0, 4):
        import itertools
        idx = sorted(oracle.cns_index(c) for c in itertools.combinations(range(n), k + 1))
        assert idx == list(range(math.comb(n, k + 1)))


# --------------------------------------------------------------------------
# the paper's worked example
# --------------------------------------------------------------------------

def test_rectangle_refined_order_and_diameters():
    g = golden_io.rectangle()
    dims, idx, diam = oracle.filtration(workloads.rectangle(), 3)
    want = [(len(s) - 1, oracle_free_cns(s)) for s in g["order"]]
    assert list(zip(dims.tolist(), idx.tolist())) == want
    assert diam.tolist() == g["diam"]


def oracle_free_cns(s):
    # CNS written out here from its definition, independent of the oracle
    return sum(math.comb(v, l + 1) for l, v in enumerate(sorted(s)))


@pytest.mark.parametrize("p", [2, 3, 5])
def test_rectangle_apparent_pairs(p):
    g = golden_io.rectangle()
    r = oracle.barcode(workloads.rectangle(), max_dim=2, p=p)
    got = set()
    for k, (lo, hi) in enumerate(r.apparent):
        got |= {(k, int(a), int(b)) for a, b in zip(lo, hi)}
    want = {(len(s) - 1, oracle_free_cns(s), oracle_free_cns(t)) for s, t in g["apparent"]}
    assert got == want


def test_rectangle_morse_function():
    g = golden_io.rectangle()
    r = oracle.barcode(workloads.rectangle(), max_dim=2, p=2)
    dims, idx, _ = oracle.filtration(workloads.rectangle(), 3)
    pos = {(int(d), int(i)): q for q, (d, i) in enumerate(zip(dims, idx))}
    f = list(range(len(dims)))
    for k, (lo, hi) in enumerate(r.apparent):
        for a, b in zip(lo, hi):
            f[pos[(k + 1, int(b))]] = pos[(k, int(a))]
    assert f == g["morse"]
    # the only entry that differs from the printed table is the edge 1.0
    diff = [i for i, (a, b) in enumerate(zip(f, g["morse_printed"])) if a != b]
    assert [g["order"][i] for i in diff] == [(1, 0)]
    # f is monotone (a discrete Morse function): facets never exceed cofaces
    order = g["order"]
    for j, s in enumerate(order):
        for i, r in enumerate(order):
            if len(r) == len(s) - 1 and set(r) <= set(s):
                assert f[i] <= f[j]


@pytest.mark.parametrize("p", [2, 3])
def test_rectangle_barcode(p):
    g = golden_io.rectangle()
    r = oracle.barcode(workloads.rectangle(), max_dim=2, p=p)
    got = []
    for k, b in enumerate(r.bars):
        for i in range(len(b)):
            got.append((k, float(b.birth[i]), float(b.death[i]), int(b.birth_simplex[i]),
                        int(b.death_simplex[i])))
    want = [(d, bb, de, oracle_free_cns(bs), -1 if ds is None else oracle_free_cns(ds))
            for d, bb, de, bs, ds in g["bars"]]
    assert sorted(got) == sorted(want)
    # canonical order inside a dimension: birth asc, birth simplex desc
    assert [x[3] for x in got if x[0] == 0] == [3, 2, 1, 0]


# --------------------------------------------------------------------------
# independent brute force (ranks of lower-left submatrices)
# --------------------------------------------------------------------------

def _oracle_pairs(r, k):
    lo, hi, es = r.pairs[k]
    return {(int(a), int(b)) for a, b in zip(lo, hi)}, {int(e) for e in es}


CLOUDS_SMALL = [
    ("cube-7x3", lambda: workloads.uniform_cube(7, 3, 11), 2),
    ("cube-8x2", lambda: workloads.uniform_cube(8, 2, 12), 2),
    ("lattice-8x2", lambda: workloads.integer_lattice(8, 2, 13, side=3), 2),
    ("lattice-7x3-dups", lambda: workloads.integer_lattice(7, 3, 14, side=2), 2),
    ("sphere-9", lambda: workloads.sphere(9, 15), 1),
    ("hexagon", lambda: workloads.regular_polygon(6), 2),
]


@pytest.mark.parametrize("name,make,max_dim", CLOUDS_SMALL)
@pytest.mark.parametrize("p", [2, 3])
@pytest.mark.parametrize("clamp", [True, False])
def test_oracle_pairs_match_rank_bruteforce(name, make, max_dim, p, clamp):
    x = make()
    r = oracle.barcode(x, max_dim=max_dim, p=p, clamp=clamp)
    t = r.threshold
    bf = bruteforce.pairs(dist_lower=oracle.distances(x), max_dim=max_dim, threshold=t, p=p)
    for k in range(max_dim + 1):
        prs, ess = _oracle_pairs(r, k)
        assert prs == bf[k][0], (name, k)
        assert ess == bf[k][1], (name, k)


@pytest.mark.parametrize("name,make,max_dim", CLOUDS_SMALL[:4])
def test_bars_match_betti_curves(name, make, max_dim):
    x = make()
    r = oracle.barcode(x, max_dim=max_dim, p=2)
    radii, betti = bruteforce.betti_curve_check(dist_lower=oracle.distances(x),
                                                max_dim=max_dim, threshold=r.threshold, p=2)
    for ri, rad in enumerate(radii):
        for k in range(max_dim + 1):
            b = r.bars[k]
            alive = int(np.sum((b.birth <= rad) & (rad < b.death)))
            assert alive == betti[ri, k], (name, rad, k)


@pytest.mark.parametrize("seed", range(6))
def test_homology_equals_cohomology_pairs(seed):
    # duality (section "Persistent cohomology"): Algorithm 1 on the boundary
    # matrices gives the same pairs as cohomology with clearing
    g = workloads.rng(100 + seed)
    n = int(g.integers(10, 19))
    x = (g.standard_normal((n, 3)) if seed % 2 else g.integers(0, 3, (n, 3))).astype(np.float32)
    for p in (2, 3):
        r = oracle.barcode(x, max_dim=2, p=p, homology=True)
        for k in range(3):
            prs, ess = _oracle_pairs(r, k)
            hlo, hhi, hes = r.hom_pairs[k]
            assert prs == {(int(a), int(b)) for a, b in zip(hlo, hhi)}
            assert ess == {int(e) for e in hes}


# --------------------------------------------------------------------------
# special cases with a textbook answer
# --------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(5))
def test_h0_deaths_are_mst_edge_lengths(seed):
    g = workloads.rng(200 + seed)
    x = g.standard_normal((60, 3)).astype(np.float32)
    for t in (INF, 0.8):
        r = oracle.barcode(x, max_dim=0, threshold=t)
        d = full_dist(x).astype(np.float64)
        adj = np.where(d <= r.threshold, d, 0.0)
        np.fill_diagonal(adj, 0.0)
        mst = minimum_spanning_tree(csr_matrix(adj))
        fin = r.bars[0].death[np.isfinite(r.bars[0].death)]
        assert np.array_equal(np.sort(fin.astype(np.float64)), np.sort(mst.data))
        ncomp = connected_components(csr_matrix(adj > 0), directed=False)[0]
        assert int(np.sum(~np.isfinite(r.bars[0].death))) == ncomp


@pytest.mark.parametrize("n", [5, 7, 8, 10, 11, 6, 9, 12])
def test_regular_polygon_single_h1_bar(n):
    # Rips complexes of the circle (Adamaszek-Adams): the n-gon has one H1
    # class, born at the side length 2 sin(pi/n), dying at the chord of step
    # ceil(n/3); for n = 3k the complex at that scale is a wedge of k - 1
    # two-spheres, so k - 1 H2 classes appear
    x = workloads.regular_polygon(n)
    r = oracle.barcode(x, max_dim=2, p=2)
    b = r.bars[1]
    big = np.nonzero((b.death - b.birth) > 1e-4)[0]
    assert len(big) == 1
    i = big[0]
    assert abs(b.birth[i] - 2 * math.sin(math.pi / n)) < 1e-5
    k = -(-n // 3)
    assert abs(b.death[i] - 2 * math.sin(math.pi * k / n)) < 1e-5
    h2 = r.bars[2]
    n_h2 = int(np.sum((h2.death - h2.birth) > 1e-4))
    assert n_h2 == (n // 3 - 1 if n % 3 == 0 else 0)


def test_closed_form_column_counts_n192():
    c = golden_io.column_counts()
    n, p = c["n"], c["p"]
    C = math.comb
    assert sum(C(n, d + 1) for d in range(1, p + 2)) == c["homology_total"]
    assert sum(C(n - 1, d) for d in range(1, p + 2)) == c["homology_death"]
    assert sum(C(n - 1, d + 1) for d in range(1, p + 2)) == c["homology_birth"]
    assert sum(C(n - 1, d) for d in range(1, p + 3)) == c["homology_clearing_total"]
    assert sum(C(n - 1, d) for d in range(1, p + 3)) - c["homology_death"] == \
        c["homology_clearing_birth"]
    assert sum(C(n, d + 1) for d in range(0, p + 1)) == c["cohomology_total"]
    assert sum(C(n - 1, d) for d in range(0, p + 1)) == c["cohomology_birth"]
    assert sum(C(n - 1, d) for d in range(0, p + 2)) == c["cohomology_clearing_total"]


@pytest.mark.parametrize("n,max_dim", [(9, 2), (12, 1), (8, 3)])
def test_full_complex_counts(n, max_dim):
    # full (max_dim+1)-skeleton: the cohomology columns left by clearing are
    # sum_{d=0}^{max_dim+1} C(n-1, d) (section "Persistent cohomology"), and
    # each dimension k has C(n-1, k+1) pairs
    x = workloads.uniform_cube(n, 4, 300 + n)
    r = oracle.barcode(x, max_dim=max_dim, clamp=False)
    assert r.counts == [math.comb(n, k + 1) for k in range(max_dim + 2)]
    total = sum(c["reduced_columns"] for c in r.counters)
    assert total == sum(math.comb(n - 1, d) for d in range(max_dim + 2))
    for k in range(max_dim + 1):
        assert r.counters[k]["pairs"] == math.comb(n - 1, k + 1)
    assert [c["essential"] for c in r.counters] == [1] + [0] * max_dim


@pytest.mark.parametrize("seed", range(4))
def test_cone_pair_counts_and_euler(seed):
    # at the enclosing radius the complex is a cone: one essential class
    # (H0), so P_{k,k+1} = sum_{i<=k} (-1)^{k-i} |K_i| - (-1)^k
    g = workloads.rng(400 + seed)
    x = g.standard_normal((25, 3)).astype(np.float32)
    r = oracle.barcode(x, max_dim=2)
    K = r.counts
    assert [c["essential"] for c in r.counters] == [1, 0, 0]
    for k in range(3):
        want = sum((-1) ** (k - i) * K[i] for i in range(k + 1)) - (-1) ** k
        assert r.counters[k]["pairs"] == want


def test_enclosing_radius_closed_form():
    # "Input" paragraph: the enclosing radius is min over x of max over y of
    # d(x, y). Four points on a line at -3, 0, 2, 5 (exact float32 distances):
    # the row maxima are 8, 5, 5, 8, so the enclosing radius is 5; the
    # diameter (max max) is 8, max min is 3 and min min is 2, so swapping
    # either min or max gives another value.
    x = np.array([[-3.0], [0.0], [2.0], [5.0]], np.float32)
    r = oracle.barcode(x, max_dim=1)
    assert r.enclosing_radius == 5.0 and r.threshold == 5.0
    # a finite threshold is clamped to it, never raised
    assert oracle.barcode(x, max_dim=1, threshold=6.0).threshold == 5.0
    assert oracle.barcode(x, max_dim=1, threshold=4.0).threshold == 4.0
    # without the clamp the full complex is used
    assert oracle.barcode(x, max_dim=1, clamp=False).threshold == INF
    # unit square with its centre: the centre's farthest point is a corner at
    # sqrt(2) (correctly rounded: 0x3FB504F3), every corner's is 2 sqrt(2)
    sq = np.array([[0, 0], [2, 0], [0, 2], [2, 2], [1, 1]], np.float32)
    rs = oracle.barcode(sq, max_dim=1)
    assert np.float32(rs.enclosing_radius).view(np.uint32) == 0x3FB504F3
    # a star: centre 0, leaves at distances 1, 2, 3 and 4 on the coordinate
    # axes; the centre's row maximum is 4, the leaves' are sqrt(17), 6, 5, 6
    st = np.array([[0, 0], [1, 0], [0, 2], [-3, 0], [0, -4]], np.float32)
    assert oracle.barcode(st, max_dim=1).enclosing_radius == 4.0


def test_facets_from_paper():
    # facets of {v5, v3, v0} in forward colexicographic order (section
    # "Enumerating cofacets and facets"): dropping v5, then v3, then v0
    _, _, (s, want) = golden_io.cns()
    got = [oracle.cns_index(tuple(v for q, v in enumerate(s) if q != m)) for m in range(len(s))]
    assert got == want


@pytest.mark.parametrize("seed", range(4))
def test_enclosing_radius_cut_keeps_bars(seed):
    g = workloads.rng(500 + seed)
    x = g.standard_normal((14, 3)).astype(np.float32)
    a = oracle.barcode(x, max_dim=2, clamp=True)
    b = oracle.barcode(x, max_dim=2, clamp=False)
    assert a.threshold <= b.threshold
    for k in range(3):
        for f in ("birth", "death", "birth_simplex", "death_simplex"):
            assert np.array_equal(getattr(a.bars[k], f), getattr(b.bars[k], f))


@pytest.mark.parametrize("seed", range(4))
def test_apparent_pairs_field_independent(seed):
    g = workloads.rng(600 + seed)
    x = g.integers(0, 4, (16, 3)).astype(np.float32)
    sets = []
    for p in (2, 3, 7):
        r = oracle.barcode(x, max_dim=2, p=p)
        sets.append([{(int(a), int(b)) for a, b in zip(lo, hi)} for lo, hi in r.apparent])
    assert sets[0] == sets[1] == sets[2]
    # each simplex lies in at most one apparent pair
    for k in range(3):
        los = [a for a, _ in sets[0][k]]
        his = [b for _, b in sets[0][k]]
        assert len(set(los)) == len(los) and len(set(his)) == len(his)
        if k >= 1:
            prev_his = {b for _, b in sets[0][k - 1]}
            assert not (prev_his & set(los))


@pytest.mark.parametrize("seed", range(4))
def test_dim1_zero_pairs_are_apparent(seed):
    # Theorem (distinct distances): non-apparent, non-cleared dim-1 columns
    # are exactly the nonzero H1 bars plus the essential H1 classes
    x = workloads.sphere(70, 700 + seed)
    for t in (INF, 0.9):
        r = oracle.barcode(x, max_dim=1, threshold=t)
        assert len(r.columns[1][0]) == len(r.bars[1])


def test_apparent_pairs_are_persistence_pairs():
    x = workloads.uniform_cube(30, 3, 800)
    r = oracle.barcode(x, max_dim=2, p=3)
    for k in range(3):
        prs, _ = _oracle_pairs(r, k)
        lo, hi = r.apparent[k]
        assert {(int(a), int(b)) for a, b in zip(lo, hi)} <= prs


def test_invalid_arguments():
    x = workloads.sphere(10, 1)
    with pytest.raises(ValueError):
        oracle.barcode(x, p=4)
    with pytest.raises(ValueError):
        oracle.barcode(x, p=65537)
    bad = oracle.distances(x)
    bad[3] = np.nan
    with pytest.raises(ValueError):
        oracle.barcode(dist_lower=bad)
