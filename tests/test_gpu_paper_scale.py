"""GPU parity at paper scale: the o3-shaped workload on 1024 points with
threshold 1.8 and homology up to dimension 3 (142 M simplices up to
dimension 4), and a 10,000-point Clifford torus with threshold 0.25 up to
dimension 2 (15.8 M simplices up to dimension 3), over Z/2 and Z/3.

The oracle would take far too long here. The reference is the
single-threaded implementation of the paper's algorithm under
cpu_baseline/, which the CPU tests hold bit for bit to the oracle on every
benchmark workload; at these sizes it takes about 11 s and 3 s. Bars (birth,
death, birth simplex, death simplex) must be identical in every dimension."""

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def test_o3_1024_dims_0_to_3_against_cpu_paper_algorithm():
    import cpu_baseline
    import oracle
    import paper_1908_02518_amd as rips

    c = workloads.config(6)
    x = c["clouds"][0]
    md, t, p = c["max_dim"], c["threshold"], c["p"]
    print(f"[case] config 6 {c['name']} n={x.shape[0]} t={t} dims 0-{md}", flush=True)
    got = rips.barcode(x, max_dim=md, threshold=t, p=p)
    cpu_baseline.build(force=False)
    ref = cpu_baseline.barcode(oracle.distances(x), x.shape[0], max_dim=md, threshold=t, p=p)
    for d in range(md + 1):
        for f in ("birth", "death", "birth_simplex", "death_simplex"):
            a, b = getattr(got.bars[d], f), getattr(ref.bars[d], f)
            assert a.shape == b.shape, (d, f, a.shape, b.shape)
            assert np.array_equal(a, b), (d, f)
    # the homology of this cloud is not trivial in any dimension tested
    assert all(len(got.bars[d].birth) > 0 for d in range(md + 1))


@pytest.mark.parametrize("p", [2, 3])
def test_torus_10000_dims_0_to_2_against_cpu_paper_algorithm(p):
    import cpu_baseline
    import oracle
    import paper_1908_02518_amd as rips

    c = workloads.config(7)
    x = c["clouds"][0]
    md, t = c["max_dim"], c["threshold"]
    print(f"[case] config 7 {c['name']} n={x.shape[0]} t={t} dims 0-{md} p={p}", flush=True)
    got = rips.barcode(x, max_dim=md, threshold=t, p=p)
    cpu_baseline.build(force=False)
    ref = cpu_baseline.barcode(oracle.distances(x), x.shape[0], max_dim=md, threshold=t, p=p)
    for d in range(md + 1):
        for f in ("birth", "death", "birth_simplex", "death_simplex"):
            a, b = getattr(got.bars[d], f), getattr(ref.bars[d], f)
            assert a.shape == b.shape, (d, f, a.shape, b.shape)
            assert np.array_equal(a, b), (d, f)
