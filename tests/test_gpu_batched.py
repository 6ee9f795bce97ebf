"""GPU parity of the batched persistent launch: every cloud's bars equal the
single-cloud path's and, on a sample, the oracle's, bit for bit."""

import numpy as np
import pytest

import oracle
import workloads

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


def test_mixture_512_vs_single_and_oracle_sample():
    import torch
    c = workloads.config(4)
    clouds = c["clouds"]
    x, off, nmax = rips().pack_clouds(clouds)
    print(f"[case] mixture batch B={len(clouds)} nmax={nmax}", flush=True)
    bb = rips().barcode_batched(x, off, nmax, max_dim=1, p=2)
    torch.cuda.synchronize()
    for b in range(len(clouds)):
        single = rips().barcode(clouds[b], max_dim=1, p=2)
        assert_cloud(bb, b, single.bars, 1, "mixture-vs-single")
    for b in (0, 1, 97, 300, 511):
        ref = oracle.barcode(clouds[b], max_dim=1, p=2)
        assert_cloud(bb, b, ref.bars, 1, "mixture-vs-oracle")


def test_circles_64x400_vs_single_and_oracle_sample():
    import torch
    c = workloads.config(5)
    clouds = c["clouds"]
    x, off, nmax = rips().pack_clouds(clouds)
    print(f"[case] circles batch B={len(clouds)} nmax={nmax}", flush=True)
    bb = rips().barcode_batched(x, off, nmax, max_dim=1, p=2)
    torch.cuda.synchronize()
    for b in range(len(clouds)):
        single = rips().barcode(clouds[b], max_dim=1, p=2)
        assert_cloud(bb, b, single.bars, 1, "circles-vs-single")
    ref = oracle.barcode(clouds[0], max_dim=1, p=2)
    assert_cloud(bb, 0, ref.bars, 1, "circles-vs-oracle")


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
