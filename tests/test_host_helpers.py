"""The host helpers of the paper-scale checks, pinned on small clouds
against the oracle: CNS decoding and encoding round trips against the
oracle's own index, pair distances against the oracle's distance matrix bit
for bit, and the prefix restriction against the oracle run at the cut
itself (the pairs of a filtration prefix are the pairs inside it)."""

import numpy as np
import pytest

import oracle
import workloads
from tests import cns_np


def test_decode_round_trip_and_oracle_index():
    g = np.random.default_rng(7)
    n = 40
    for k in range(0, 5):
        verts = np.array([sorted(g.choice(n, k + 1, replace=False), reverse=True) for _ in range(50)])
        idx = np.array([oracle.cns_index(v) for v in verts])
        assert np.array_equal(cns_np.index_of(verts, n), idx)
        assert np.array_equal(cns_np.decode(idx, k, n), verts)
    # the paper's worked example: {5, 3, 0} has index 13
    assert cns_np.index_of(np.array([[5, 3, 0]]), 8)[0] == 13


def test_pair_dist_matches_oracle_bits():
    x = workloads.so3(60, 3)
    D = oracle.distances(x)
    i, j = np.tril_indices(60, -1)
    assert np.array_equal(cns_np.pair_dist(x, i, j).view(np.uint32), D.view(np.uint32))


@pytest.mark.parametrize("name,x,max_dim,t,r", [
    ("sphere-60", workloads.sphere(60, 5), 2, float("inf"), 0.6),
    ("o3-200", workloads.orthogonal(200, 6), 3, 1.4, 0.9),
    ("lattice", workloads.integer_lattice(40, 3, 8, side=3), 2, float("inf"), 1.5),
])
def test_prefix_restriction_is_the_cut_filtration(name, x, max_dim, t, r):
    full = oracle.barcode(x, max_dim=max_dim, threshold=t, p=2)
    cut = oracle.barcode(x, max_dim=max_dim, threshold=r, p=2)
    assert cut.threshold == np.float32(r)
    for d in range(max_dim + 1):
        b = full.bars[d]
        got = cns_np.restrict_to_prefix(b.birth, b.death, b.birth_simplex, b.death_simplex, r)
        want = (cut.bars[d].birth, cut.bars[d].death, cut.bars[d].birth_simplex,
                cut.bars[d].death_simplex)
        for g_, w_ in zip(got, want):
            assert np.array_equal(g_, w_), (name, d)
    # the cut is not trivial: some bar dies after r, or is born after it
    assert any(np.any(full.bars[d].death > np.float32(r)) for d in range(max_dim + 1))


def test_counter_summary_hash_ignores_comments_only():
    """The hash that ties a counter summary to the kernels it measured: a
    comment or whitespace edit leaves it, a code edit (even inside what
    looks like a comment marker in a string) changes it."""
    import bench
    base = 'int f(int x) {\n    return x + 1; // one more\n}\nconst char *s = "a // b";\n'
    same = '/* header */\nint f(int x) {   return x + 1; }\nconst char *s = "a // b"; // note\n'
    other = 'int f(int x) {\n    return x + 2; // one more\n}\nconst char *s = "a // b";\n'
    lit = 'int f(int x) {\n    return x + 1; // one more\n}\nconst char *s = "a // c";\n'
    code = bench._code_only
    assert code(base) == code(same)
    assert code(base) != code(other)
    assert code(base) != code(lit)
