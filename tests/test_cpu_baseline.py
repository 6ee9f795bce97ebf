"""The single-threaded CPU implementation of the paper's algorithm
(cpu_baseline/, a performance baseline for bench.py) against the oracle:
bars, birth and death simplices bit for bit, and its column and addition
counts against the oracle's reduction."""

import numpy as np
import pytest

import cpu_baseline
import oracle
import workloads

INF = float("inf")

CASES = [
    ("rectangle-p3", lambda: workloads.rectangle(), 2, INF, 3),
    ("9-gon-p3", lambda: workloads.regular_polygon(9), 2, INF, 3),
    ("cube-30x3-p5", lambda: workloads.uniform_cube(30, 3, 3), 2, INF, 5),
    ("cube-24x4-dim3", lambda: workloads.uniform_cube(24, 4, 4), 3, INF, 2),
    ("lattice-30x3-dups-p3", lambda: workloads.integer_lattice(30, 3, 6, side=3), 2, INF, 3),
    ("cube-300x3-sparse", lambda: workloads.uniform_cube(300, 3, 9), 2, 0.2, 2),
    ("torus-500-sparse", lambda: workloads.clifford_torus(500, 0.02, 11), 2, 0.6, 3),
    ("one-point", lambda: np.zeros((1, 3), np.float32), 1, INF, 2),
    ("all-duplicates", lambda: np.ones((6, 2), np.float32), 2, INF, 2),
    ("negative-threshold", lambda: workloads.uniform_cube(10, 2, 13), 1, -1.0, 2),
    ("sphere-100", lambda: workloads.config(1)["clouds"][0], 1, INF, 2),
]


@pytest.mark.parametrize("name,make,max_dim,t,p", CASES, ids=[c[0] for c in CASES])
def test_paper_cpu_matches_oracle(name, make, max_dim, t, p):
    x = make()
    ref = oracle.barcode(x, max_dim=max_dim, threshold=t, p=p)
    got = cpu_baseline.barcode(oracle.distances(x), x.shape[0], max_dim=max_dim, threshold=t, p=p)
    assert np.float32(got.threshold).tobytes() == np.float32(ref.threshold).tobytes()
    for d in range(max_dim + 1):
        a, b = got.bars[d], ref.bars[d]
        for f in ("birth", "death", "birth_simplex", "death_simplex"):
            assert np.array_equal(getattr(a, f), getattr(b, f)), (name, d, f)
    for k in range(1, max_dim + 1):
        # the same columns survive clearing and the apparent pairs
        assert got.columns[k] == len(ref.columns[k][0]), (name, k)
