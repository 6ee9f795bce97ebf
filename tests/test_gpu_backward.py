"""GPU backward (rips_backward_device behind torch.autograd) on the
differentiation workload: 400-point noisy circles with 10% outliers, loss =
sum of (death - birth)^2 over the top-5 H1 bars.

Checked against (1) the float64 reference gradient of oracle/gradient.py on
the oracle's own pairing, (2) central finite differences of the GPU forward
(h = 1e-3, relative error <= 1e-3, coordinates where the pairing or a
critical edge changes within +-h excluded as kinks), (3) the batched
backward against the single-cloud one."""

import numpy as np
import pytest

import oracle
import workloads
from oracle import gradient

pytestmark = pytest.mark.gpu


def rips():
    import paper_1908_02518_amd as r
    return r


def gpu_loss_and_grad(x_np):
    import torch
    x = torch.from_numpy(x_np).cuda().requires_grad_(True)
    bars = rips().diagram(x, max_dim=1, p=2)
    L = rips().top_persistence_loss(bars[1].birth, bars[1].death, bars[1].birth_simplex, top=5)
    L.backward()
    torch.cuda.synchronize()
    return float(L), x.grad.detach().cpu().numpy().astype(np.float64), bars


def selection(x_np):
    """Loss (float64 from the float32 endpoints) and the identity of the
    active pairing: the selected bars' simplices and their critical edges."""
    import torch
    x = torch.from_numpy(x_np).cuda()
    bars, _ = rips().barcode_device(x, max_dim=1, p=2)
    b, d, bs, ds = [t.cpu().numpy() for t in bars[1]]
    sel = gradient.top_bars(b, d, bs, 5)
    L = sum((float(d[i]) - float(b[i])) ** 2 for i in sel)
    key = tuple((int(bs[i]), int(ds[i]), gradient.critical_edge(x_np, int(bs[i]), 1),
                 gradient.critical_edge(x_np, int(ds[i]), 2)) for i in sel)
    return L, key


@pytest.mark.parametrize("cloud", [0, 1, 2, 3])
def test_gradient_matches_reference(cloud):
    x = workloads.config(5)["clouds"][cloud]
    print(f"[case] reference gradient, circles cloud {cloud}", flush=True)
    L, g, _ = gpu_loss_and_grad(x)
    ref = oracle.barcode(x, max_dim=1, p=2)
    Lr, gr, _ = gradient.loss_and_grad(x, ref.bars[1], dim=1, top=5)
    assert abs(L - Lr) <= 1e-12 * max(1.0, abs(Lr))
    scale = np.abs(gr).max()
    assert scale > 0
    err = np.abs(g - gr).max() / scale
    assert err <= 1e-5, err
    # the gradient lives on the critical-edge points only
    assert set(np.nonzero(np.abs(g).sum(1))[0]) == set(np.nonzero(np.abs(gr).sum(1))[0])


@pytest.mark.parametrize("cloud", [0, 5])
def test_gradient_matches_central_differences(cloud):
    x = workloads.config(5)["clouds"][cloud]
    print(f"[case] finite differences, circles cloud {cloud}", flush=True)
    L0, g, _ = gpu_loss_and_grad(x)
    _, key0 = selection(x)
    # every coordinate of the critical-edge points, plus 16 random ones
    # (expected gradient 0)
    rows = sorted({v for k in key0 for e in k[2:] for v in e})
    coords = [(i, c) for i in rows for c in range(2)]
    rng = workloads.rng(4242 + cloud)
    others = [i for i in range(x.shape[0]) if i not in rows]
    coords += [(int(i), int(rng.integers(0, 2))) for i in rng.choice(others, 16, replace=False)]
    h = 1e-3
    got, fds, kinks = [], [], 0
    for i, c in coords:
        xp, xm = x.copy(), x.copy()
        xp[i, c] = np.float32(x[i, c] + h)
        xm[i, c] = np.float32(x[i, c] - h)
        Lp, kp = selection(xp)
        Lm, km = selection(xm)
        if kp != key0 or km != key0:
            kinks += 1  # the active pairing changes within +-h: not differentiable there
            continue
        step = float(xp[i, c]) - float(xm[i, c])
        got.append(g[i, c])
        fds.append((Lp - Lm) / step)
    got, fds = np.array(got), np.array(fds)
    print(f"[fd] cloud {cloud}: {len(fds)} coordinates, {kinks} kinks excluded", flush=True)
    assert len(fds) >= 0.75 * len(coords), (len(fds), kinks, len(coords))
    rel = np.linalg.norm(got - fds) / np.linalg.norm(fds)
    assert rel <= 1e-3, rel
    assert np.abs(got - fds).max() <= 1e-3 * np.abs(fds).max()


def test_batched_backward_matches_single():
    import torch
    c = workloads.config(5)
    clouds = c["clouds"][:16]
    x, off, nmax = rips().pack_clouds(clouds)
    print(f"[case] batched backward B={len(clouds)}", flush=True)
    xg = x.clone().requires_grad_(True)
    birth, death, bs, ds, seg = rips().batched_diagram(xg, off, nmax, max_dim=1, p=2)
    segh = seg.cpu().numpy()
    L = 0.0
    for b in range(len(clouds)):
        lo, hi = int(segh[2 * b + 1]), int(segh[2 * b + 2])
        L = L + rips().top_persistence_loss(birth[lo:hi], death[lo:hi], bs[lo:hi], top=5)
    L.backward()
    torch.cuda.synchronize()
    gb = xg.grad.cpu().numpy()
    offh = off.cpu().numpy()
    for b, cl in enumerate(clouds):
        _, g1, _ = gpu_loss_and_grad(cl)
        part = gb[offh[b]:offh[b + 1]].astype(np.float64)
        scale = max(np.abs(g1).max(), 1e-30)
        assert np.abs(part - g1).max() <= 1e-5 * scale, b


def test_distance_matrix_gradient():
    import torch
    x = workloads.config(5)["clouds"][2]
    print("[case] distance-matrix input gradient", flush=True)
    D = oracle.distances(x)  # lower triangle, row-major pairs (i > j)
    n = x.shape[0]
    full = np.zeros((n, n), np.float32)
    il = np.tril_indices(n, -1)
    full[il] = D
    full = full + full.T
    M = torch.from_numpy(full).cuda().requires_grad_(True)
    bars = rips().diagram(M, max_dim=1, p=2, is_distance=True)
    L = rips().top_persistence_loss(bars[1].birth, bars[1].death, bars[1].birth_simplex, top=5)
    L.backward()
    torch.cuda.synchronize()
    G = M.grad.cpu().numpy().astype(np.float64)
    # expected: +2(d-b) at the death simplex's critical entry, -2(d-b) at the
    # birth edge's entry, entry (u, v) with u > v
    ref = oracle.barcode(x, max_dim=1, p=2).bars[1]
    sel = gradient.top_bars(ref.birth, ref.death, ref.birth_simplex, 5)
    want = np.zeros((n, n))
    for i in sel:
        w = 2.0 * (float(ref.death[i]) - float(ref.birth[i]))
        u, v = gradient.critical_edge(x, int(ref.death_simplex[i]), 2)
        want[u, v] += w
        u, v = gradient.critical_edge(x, int(ref.birth_simplex[i]), 1)
        want[u, v] -= w
    assert np.abs(G - want).max() <= 1e-5 * np.abs(want).max()


def test_backward_rejects_bad_arguments():
    import torch
    x = torch.zeros((4, 2), device="cuda")
    z = torch.zeros(1, dtype=torch.int64, device="cuda")
    f = torch.zeros(1, device="cuda")
    with pytest.raises(rips().RipsError):
        rips().backward_scatter(x, 0, 2, 1, z, z, f, f, torch.zeros_like(x))
    with pytest.raises(rips().RipsError):
        rips().backward_scatter(x, 4, 2, 9, z, z, f, f, torch.zeros_like(x))
