"""GPU parity: the HIP path, called through the C ABI, against the oracle.

Bars (birth, death, birth simplex, death simplex), the threshold used and
the set of columns left for the reduction must be bit-identical to the
oracle's on the same seeded float32 inputs."""

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu
INF = float("inf")


def rips():
    import paper_1908_02518_amd as r
    return r


def assert_same(got, ref, max_dim, columns=True, tag=""):
    assert np.float32(got.threshold).tobytes() == np.float32(ref.threshold).tobytes(), tag
    for d in range(max_dim + 1):
        g, w = got.bars[d], ref.bars[d]
        for f in ("birth", "death", "birth_simplex", "death_simplex"):
            a, b = getattr(g, f), getattr(w, f)
            assert a.shape == b.shape, (tag, d, f, a.shape, b.shape)
            assert np.array_equal(a, b), (tag, d, f)
        assert got.simplex_count[d] == ref.counts[d], (tag, d)
        if columns and d >= 1:
            gi, gd = got.columns[d]
            wi, wd = ref.columns[d]
            assert np.array_equal(gi, wi), (tag, d, "columns")
            assert np.array_equal(gd, wd), (tag, d, "column diameters")


SMALL = [
    ("rectangle-p2", lambda: workloads.rectangle(), 2, INF, 2),
    ("rectangle-p3", lambda: workloads.rectangle(), 2, INF, 3),
    ("hexagon", lambda: workloads.regular_polygon(6), 2, INF, 2),
    ("9-gon-p3", lambda: workloads.regular_polygon(9), 2, INF, 3),
    ("12-gon", lambda: workloads.regular_polygon(12), 2, INF, 2),
    ("cube-30x3-p2", lambda: workloads.uniform_cube(30, 3, 1), 2, INF, 2),
    ("cube-30x3-p3", lambda: workloads.uniform_cube(30, 3, 2), 2, INF, 3),
    ("cube-30x3-p5", lambda: workloads.uniform_cube(30, 3, 3), 2, INF, 5),
    ("cube-24x4-dim3", lambda: workloads.uniform_cube(24, 4, 4), 3, INF, 2),
    ("lattice-40x2-ties", lambda: workloads.integer_lattice(40, 2, 5, side=5), 2, INF, 2),
    ("lattice-30x3-dups-p3", lambda: workloads.integer_lattice(30, 3, 6, side=3), 2, INF, 3),
    ("sphere-70", lambda: workloads.sphere(70, 7), 1, INF, 2),
    ("sphere-70-t0.6", lambda: workloads.sphere(70, 8), 2, 0.6, 2),
    ("cube-300x3-sparse", lambda: workloads.uniform_cube(300, 3, 9), 2, 0.2, 2),
    ("cube-300x3-sparse-p3", lambda: workloads.uniform_cube(300, 3, 10), 2, 0.22, 3),
    ("torus-500-sparse", lambda: workloads.clifford_torus(500, 0.02, 11), 2, 0.6, 3),
    ("so3-300", lambda: workloads.so3(300, 12), 2, 1.2, 2),
    ("one-point", lambda: np.zeros((1, 3), np.float32), 1, INF, 2),
    ("two-points", lambda: np.array([[0, 0], [1, 0]], np.float32), 1, INF, 2),
    ("all-duplicates", lambda: np.ones((6, 2), np.float32), 2, INF, 2),
    ("negative-threshold", lambda: workloads.uniform_cube(10, 2, 13), 1, -1.0, 2),
    ("zero-threshold-dups", lambda: workloads.integer_lattice(20, 2, 14, side=2), 2, 0.0, 2),
]


@pytest.mark.parametrize("name,make,max_dim,t,p", SMALL, ids=[c[0] for c in SMALL])
def test_small_parity(name, make, max_dim, t, p):
    x = make()
    print(f"[case] {name} n={x.shape[0]} max_dim={max_dim} t={t} p={p}", flush=True)
    got = rips().barcode(x, max_dim=max_dim, threshold=t, p=p)
    ref = oracle.barcode(x, max_dim=max_dim, threshold=t, p=p)
    assert_same(got, ref, max_dim, tag=name)


def test_distance_matrix_input():
    x = workloads.uniform_cube(40, 3, 21)
    d = oracle.distances(x)
    full = np.zeros((40, 40), np.float32)
    full[np.tril_indices(40, -1)] = d
    full = full + full.T
    got = rips().barcode(dist=full, max_dim=2, p=2)
    ref = oracle.barcode(dist_lower=d, max_dim=2, p=2)
    assert_same(got, ref, 2, tag="dist-input")


def test_nonfinite_input_rejected():
    x = workloads.uniform_cube(10, 2, 22)
    x[3, 1] = np.nan
    with pytest.raises(rips().RipsError) as e:
        rips().barcode(x, max_dim=1)
    assert e.value.status == -4


@pytest.mark.parametrize("cfg", [1, 2, 3])
def test_config_parity_full_size(cfg):
    c = workloads.config(cfg)
    x = c["clouds"][0]
    print(f"[case] config {cfg} {c['name']}", flush=True)
    got = rips().barcode(x, max_dim=c["max_dim"], threshold=c["threshold"], p=c["p"])
    ref = oracle.barcode(x, max_dim=c["max_dim"], threshold=c["threshold"], p=c["p"])
    assert_same(got, ref, c["max_dim"], tag=c["name"])
    # the counters add up with the oracle's
    for k in range(1, c["max_dim"] + 1):
        s, o = got.stats[k], ref.counters[k]
        assert s["candidates"] == ref.counts[k]
        assert s["cleared"] + s["apparent_pivot"] == o["cleared"]
        assert s["apparent_col"] == o["zero_apparent_col"]
        assert s["columns"] == len(ref.columns[k][0])
        assert s["bars_nonzero"] + s["essential"] == len(ref.bars[k])


def test_deterministic_repeat():
    c = workloads.config(2)
    x = c["clouds"][0]
    a = rips().barcode(x, max_dim=2, threshold=1.4, p=2)
    b = rips().barcode(x, max_dim=2, threshold=1.4, p=2)
    for d in range(3):
        for f in ("birth", "death", "birth_simplex", "death_simplex"):
            assert np.array_equal(getattr(a.bars[d], f), getattr(b.bars[d], f))


def test_device_entry_matches_host_entry():
    import torch
    c = workloads.config(3)
    x = c["clouds"][0]
    host = rips().barcode(x, max_dim=2, threshold=0.5, p=3)
    xt = torch.from_numpy(x).cuda()
    bars, info = rips().barcode_device(xt, max_dim=2, threshold=0.5, p=3, cap=16)
    torch.cuda.synchronize()
    for d in range(3):
        got = [t.cpu().numpy() for t in bars[d]]
        want = host.bars[d]
        assert np.array_equal(got[0], want.birth)
        assert np.array_equal(got[1], want.death)
        assert np.array_equal(got[2], want.birth_simplex)
        assert np.array_equal(got[3], want.death_simplex)
    assert info["threshold"] == host.threshold


@pytest.mark.parametrize("cfg,top", [(1, 2), (2, 3), (3, 3)])
def test_simplex_counts(cfg, top):
    import torch
    c = workloads.config(cfg)
    x = c["clouds"][0]
    ref = oracle.barcode(x, max_dim=top - 1, threshold=c["threshold"], p=2)
    got = rips().simplex_counts(torch.from_numpy(x).cuda(), top, threshold=c["threshold"])
    assert got == ref.counts


@pytest.mark.parametrize("cfg", [2, 3])
def test_reduce_workgroups_agree(cfg):
    """The reduction spread over workgroups (several counts, so that columns
    wait on each other in different interleavings) gives the oracle's bars
    and the same counters as the one-workgroup reduction."""
    c = workloads.config(cfg)
    x = c["clouds"][0]
    ref = oracle.barcode(x, max_dim=c["max_dim"], threshold=c["threshold"], p=c["p"])
    r = rips()
    base = None
    try:
        for g in (1, 2, 7, 64, 0):
            print(f"[case] config {cfg} {c['name']} reduce workgroups {g}", flush=True)
            r.set_reduce_workgroups(g)
            assert r.get_reduce_workgroups() == g
            got = r.barcode(x, max_dim=c["max_dim"], threshold=c["threshold"], p=c["p"])
            assert_same(got, ref, c["max_dim"], tag=f"{c['name']} workgroups={g}")
            if base is None:
                base = got
            for k in range(1, c["max_dim"] + 1):
                assert got.stats[k] == base.stats[k], (g, k, got.stats[k], base.stats[k])
    finally:
        r.set_reduce_workgroups(0)


SPREAD = [c for c in SMALL if c[0] in ("cube-30x3-p5", "cube-24x4-dim3", "lattice-30x3-dups-p3",
                                       "cube-300x3-sparse-p3", "torus-500-sparse", "so3-300")]


@pytest.mark.parametrize("name,make,max_dim,t,p", SPREAD, ids=[c[0] for c in SPREAD])
def test_reduce_workgroups_small(name, make, max_dim, t, p):
    """Few workgroups (2 and 3) make columns wait on each other most often;
    ties, duplicate points, Z/3 and Z/5 and dimension 3 included."""
    x = make()
    ref = oracle.barcode(x, max_dim=max_dim, threshold=t, p=p)
    r = rips()
    try:
        for g in (2, 3):
            print(f"[case] {name} reduce workgroups {g}", flush=True)
            r.set_reduce_workgroups(g)
            got = r.barcode(x, max_dim=max_dim, threshold=t, p=p)
            assert_same(got, ref, max_dim, tag=f"{name} workgroups={g}")
    finally:
        r.set_reduce_workgroups(0)
