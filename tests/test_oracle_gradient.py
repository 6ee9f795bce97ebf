"""Pin of the float64 reference gradient (oracle/gradient.py) against central
finite differences of the oracle's own loss. The gradient reading (critical
edge of each bar endpoint) is not in the paper; finite differences of the
barcode loss fix it wherever the pairing is locally constant."""

import numpy as np
import pytest

import oracle
import workloads
from oracle import gradient


def loss_of(x, top=5):
    r = oracle.barcode(x, max_dim=1, p=2)
    b = r.bars[1]
    sel = gradient.top_bars(b.birth, b.death, b.birth_simplex, top)
    L = sum((float(b.death[i]) - float(b.birth[i])) ** 2 for i in sel)
    edges = set()
    for i in sel:
        edges.add(gradient.critical_edge(x, int(b.birth_simplex[i]), 1))
        edges.add(gradient.critical_edge(x, int(b.death_simplex[i]), 2))
    return L, edges


@pytest.mark.parametrize("seed", [0, 1])
def test_reference_gradient_matches_finite_differences(seed):
    x = workloads.noisy_circle_with_outliers(workloads.SEED_BASE + 77 + seed, n_circle=45,
                                             n_out=5)
    r = oracle.barcode(x, max_dim=1, p=2)
    L0, g, sel = gradient.loss_and_grad(x, r.bars[1], dim=1, top=5)
    L0b, edges0 = loss_of(x)
    assert abs(L0 - L0b) < 1e-12
    assert np.count_nonzero(np.abs(g).sum(1)) > 0
    h = 1e-3
    rows = sorted({v for e in edges0 for v in e})
    coords = [(i, c) for i in rows for c in range(2)]
    g_rng = workloads.rng(seed + 5)
    others = [i for i in range(x.shape[0]) if i not in rows]
    coords += [(int(i), int(g_rng.integers(0, 2))) for i in g_rng.choice(others, 6, replace=False)]
    fd, ref, kinks = [], [], 0
    for i, c in coords:
        xp, xm = x.copy(), x.copy()
        xp[i, c] = np.float32(x[i, c] + h)
        xm[i, c] = np.float32(x[i, c] - h)
        Lp, ep = loss_of(xp)
        Lm, em = loss_of(xm)
        if ep != edges0 or em != edges0:
            kinks += 1
            continue
        step = float(xp[i, c]) - float(xm[i, c])
        fd.append((Lp - Lm) / step)
        ref.append(g[i, c])
    fd, ref = np.array(fd), np.array(ref)
    assert len(fd) >= len(coords) // 2
    rel = np.linalg.norm(ref - fd) / np.linalg.norm(fd)
    assert rel <= 1e-3, (rel, kinks)
