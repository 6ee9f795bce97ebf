"""The no-allocation entry point (rips_barcode_device_noalloc) against
rips_barcode_device, bit for bit, on two calls in a row (the second with a
smaller input, so that it runs on scratch left by the first), and its limits."""

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def rips():
    import paper_1908_02518_amd as r
    return r


def _same(a, b, max_dim, tag):
    (ba, ia), (bb, ib) = a, b
    for d in range(max_dim + 1):
        for f, ga, gb in zip(("birth", "death", "bs", "ds"), ba[d], bb[d]):
            x, y = ga.cpu().numpy(), gb.cpu().numpy()
            assert x.shape == y.shape and np.array_equal(x, y), (tag, d, f)
    assert ia["threshold"] == ib["threshold"], tag
    assert ia["simplex_count"] == ib["simplex_count"], tag
    for d in range(max_dim + 1):
        for key in ("candidates", "cleared", "apparent_col", "columns", "bars_nonzero", "essential"):
            assert ia["stats"][d][key] == ib["stats"][d][key], (tag, d, key)


CASES = [
    # (name, first input, second input (smaller), max_dim, threshold, p)
    ("sphere-256-then-80", lambda: workloads.sphere(256, 71), lambda: workloads.sphere(80, 72), 1,
     float("inf"), 2),
    ("mixture-then-lattice-p3", lambda: workloads.mixture_cloud(workloads.SEED_BASE + 4, 200, 256),
     lambda: workloads.integer_lattice(40, 3, 5, side=3), 1, float("inf"), 3),
    ("circle-250-t-then-30", lambda: workloads.noisy_circle_with_outliers(5, 220, 30),
     lambda: workloads.regular_polygon(30), 1, 1.0, 2),
]


@pytest.mark.parametrize("name,first,second,max_dim,t,p", CASES, ids=[c[0] for c in CASES])
def test_noalloc_matches_device_entry(name, first, second, max_dim, t, p):
    import torch
    for q, make in enumerate((first, second)):
        x = torch.from_numpy(make()).to("cuda:0")
        print(f"[case] noalloc {name} call {q} n={x.shape[0]}", flush=True)
        want = rips().barcode_device(x, max_dim=max_dim, threshold=t, p=p)
        got = rips().barcode_device(x, max_dim=max_dim, threshold=t, p=p, noalloc=True)
        torch.cuda.synchronize()
        _same(got, want, max_dim, (name, q))


def test_noalloc_limits():
    import torch
    x = torch.from_numpy(workloads.sphere(300, 3)).to("cuda:0")
    with pytest.raises(rips().RipsError) as e:
        rips().barcode_device(x, max_dim=1, noalloc=True)
    assert e.value.status == -1
    y = torch.from_numpy(workloads.sphere(40, 3)).to("cuda:0")
    with pytest.raises(rips().RipsError) as e:
        rips().barcode_device(y, max_dim=2, noalloc=True)
    assert e.value.status == -1
    # still usable after the rejections
    a = rips().barcode_device(y, max_dim=1, noalloc=True)
    b = rips().barcode_device(y, max_dim=1)
    torch.cuda.synchronize()
    _same(a, b, 1, "after-rejection")
