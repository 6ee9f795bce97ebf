"""GPU parity of the batched persistent launch: every cloud's bars equal the
oracle's, bit for bit (the oracle runs on the host CPU in worker processes
while the GPU works), and the single-cloud path's. The pairs of a
simplexwise filtration are unique (section "Persistence pairs"), so every
cloud has exactly one correct barcode."""

import numpy as np
import pytest

import oracle
import workloads
from tests.oracle_pool import OraclePool

pytestmark = pytest.mark.gpu


def rips():
    import paper_1908_02518_amd as r
    return r


def seg(bb, b, d):
    return [t.cpu().numpy() for t in bb.segment(b, d)]


def assert_cloud(bb, b, ref_bars, max_dim, tag):
    for d in range(max_dim + 1):
        got = seg(bb, b, d)
        want = (ref_bars[d].birth, ref_bars[d].death, ref_bars[d].birth_simplex,
                ref_bars[d].death_simplex)
        for f, g, w in zip(("birth", "death", "bs", "ds"), got, want):
            assert g.shape == w.shape, (tag, b, d, f, g.shape, w.shape)
            assert np.array_equal(g, w), (tag, b, d, f)


def small_batch():
    clouds = [workloads.mixture_cloud(workloads.SEED_BASE + 4 + 1000 * b, 8, 60) for b in range(16)]
    clouds += [np.zeros((1, 3), np.float32), np.array([[0, 0, 0], [1, 0, 0]], np.float32),
               np.ones((5, 3), np.float32), workloads.integer_lattice(12, 3, 3, side=2)]
    return clouds


@pytest.mark.parametrize("p", [2, 3])
def test_small_batch_vs_oracle(p):
    import torch
    clouds = small_batch()
    x, off, nmax = rips().pack_clouds(clouds)
    print(f"[case] small batch B={len(clouds)} nmax={nmax} p={p}", flush=True)
    bb = rips().barcode_batched(x, off, nmax, max_dim=1, p=p)
    torch.cuda.synchronize()
    for b, c in enumerate(clouds):
        ref = oracle.barcode(c, max_dim=1, p=p)
        assert_cloud(bb, b, ref.bars, 1, "small")
        assert float(bb.thresholds[b]) == ref.threshold


def test_batch_threshold_and_h0_only():
    import torch
    clouds = small_batch()
    x, off, nmax = rips().pack_clouds(clouds)
    bb = rips().barcode_batched(x, off, nmax, max_dim=0, threshold=0.5, p=2)
    torch.cuda.synchronize()
    for b, c in enumerate(clouds):
        ref = oracle.barcode(c, max_dim=0, threshold=0.5, p=2)
        assert_cloud(bb, b, ref.bars, 0, "h0-only")


def _batch_vs_oracle_and_single(clouds, tag, max_dim=1, threshold=float("inf"), p=2,
                                single=True):
    import torch
    with OraclePool(clouds, max_dim, threshold, p) as pool:
        x, off, nmax = rips().pack_clouds(clouds)
        print(f"[case] {tag} B={len(clouds)} nmax={nmax} p={p}", flush=True)
        bb = rips().barcode_batched(x, off, nmax, max_dim=max_dim, threshold=threshold, p=p)
        torch.cuda.synchronize()
        thr = bb.thresholds.cpu().numpy()
        if single:
            for b in range(len(clouds)):
                one = rips().barcode(clouds[b], max_dim=max_dim, threshold=threshold, p=p)
                assert_cloud(bb, b, one.bars, max_dim, tag + "-vs-single")
        for b in range(len(clouds)):
            bars, t_ref = pool.get(b)
            ref = [oracle.Bars(*q) for q in bars]
            assert_cloud(bb, b, ref, max_dim, tag + "-vs-oracle")
            assert thr[b] == np.float32(t_ref), (tag, b, "threshold")


def test_mixture_512_every_cloud_vs_oracle():
    _batch_vs_oracle_and_single(workloads.config(4)["clouds"], "mixture-512")


def test_circles_64x400_every_cloud_vs_oracle():
    _batch_vs_oracle_and_single(workloads.config(5)["clouds"], "circles-64x400")


def lattice_batch(num=48):
    # integer lattices: many tied distances and duplicate points, sizes up to
    # the dense-LDS limit and above it
    g = workloads.rng(4242)
    return [workloads.integer_lattice(int(g.integers(2, 300)), 3, 9000 + b,
                                      side=int(g.integers(2, 6))) for b in range(num)]


@pytest.mark.parametrize("p", [2, 3])
def test_lattice_ties_batch_vs_oracle(p):
    _batch_vs_oracle_and_single(lattice_batch(), f"lattice-ties-p{p}", p=p, single=False)


def test_graph_replay_is_deterministic():
    import torch
    clouds = workloads.mixture_batch(64, 4)
    x, off, nmax = rips().pack_clouds(clouds)
    a = rips().barcode_batched(x, off, nmax, max_dim=1, p=2)
    torch.cuda.synchronize()
    got_a = [t.clone() for t in (a.birth, a.death, a.birth_simplex, a.death_simplex, a.offsets)]
    for _ in range(3):
        b = rips().barcode_batched(x, off, nmax, max_dim=1, p=2, cap=a.birth.shape[0])
        torch.cuda.synchronize()
        n = int(b.offsets[-1])
        for ta, tb in zip(got_a[:4], (b.birth, b.death, b.birth_simplex, b.death_simplex)):
            assert torch.equal(ta[:n], tb[:n])
        assert torch.equal(got_a[4], b.offsets)


def test_cloud_above_n_max_is_rejected():
    import torch
    clouds = [workloads.sphere(10, 1), workloads.sphere(40, 2)]
    x, off, _ = rips().pack_clouds(clouds)
    with pytest.raises(rips().RipsError) as e:
        rips().barcode_batched(x, off, 20, max_dim=1)
    assert e.value.status == -1
    torch.cuda.synchronize()


@pytest.mark.parametrize("p", [2, 3])
def test_spread_out_clouds_match_one_workgroup_per_cloud(p):
    """A batch smaller than the chip spreads each cloud over several
    workgroups (one leads, all reduce); the bars must equal those of one
    workgroup per cloud, bit for bit."""
    import torch
    r = rips()
    clouds = small_batch() + lattice_batch(12)
    x, off, nmax = r.pack_clouds(clouds)
    print(f"[case] spread vs one workgroup per cloud B={len(clouds)} p={p}", flush=True)
    r.batched_set_spread(1)
    try:
        one = r.barcode_batched(x, off, nmax, max_dim=1, p=p)
        torch.cuda.synchronize()
        one = [t.clone() for t in (one.birth, one.death, one.birth_simplex, one.death_simplex,
                                   one.offsets, one.stats)]
    finally:
        r.batched_set_spread(0)
    spread = r.barcode_batched(x, off, nmax, max_dim=1, p=p)
    torch.cuda.synchronize()
    n = int(spread.offsets[-1])
    assert torch.equal(one[4], spread.offsets)
    for a, b in zip(one[:4], (spread.birth, spread.death, spread.birth_simplex, spread.death_simplex)):
        assert torch.equal(a[:n], b[:n])
    # the counters that do not depend on the order of the reduction agree
    fields = r.STAT_FIELDS
    for f in ("candidates", "cleared", "apparent_col", "columns", "bars_nonzero", "essential"):
        q = fields.index(f)
        assert torch.equal(one[5][:, :, q], spread.stats[:, :, q]), f
