"""The shortcuts as ablation switches (the paper's Table 3): with any of the
apparent pair shortcut, the emergent pair shortcut and clearing turned off,
the HIP path must still give the oracle's bars bit for bit, and its counters
must show the shortcut off: no apparent columns or pivots (every candidate
that is not cleared becomes a column), no emergent pairs, or nothing cleared
(the columns of pivots of the dimension below reduce to zero and give no
bar)."""

from functools import lru_cache

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu
INF = float("inf")


def rips():
    import paper_1908_02518_amd as r
    return r


CASES = [
    ("rectangle-p3", lambda: workloads.rectangle(), 2, INF, 3),
    ("hexagon", lambda: workloads.regular_polygon(6), 2, INF, 2),
    ("lattice-ties", lambda: workloads.integer_lattice(27, 3, 5, side=3), 2, INF, 2),
    ("cube-40-p5", lambda: workloads.uniform_cube(40, 3, 31), 3, INF, 5),
    ("sphere-100", lambda: workloads.config(1)["clouds"][0], 1, INF, 2),
    ("so3-1000", lambda: workloads.config(2)["clouds"][0], 2, 1.4, 2),
    ("torus4-2000", lambda: workloads.config(3)["clouds"][0], 2, 0.5, 3),
]


@lru_cache(maxsize=None)
def case(name):
    _, make, max_dim, t, p = next(c for c in CASES if c[0] == name)
    x = make()
    return x, oracle.barcode(x, max_dim=max_dim, threshold=t, p=p)


@pytest.mark.parametrize("flags", [0, 1, 2, 3, 5, 6])
@pytest.mark.parametrize("name,make,max_dim,t,p", CASES, ids=[c[0] for c in CASES])
def test_bars_unchanged_without_shortcuts(flags, name, make, max_dim, t, p):
    r = rips()
    print(f"[case] shortcuts {flags} {name}", flush=True)
    x, ref = case(name)
    r.set_shortcuts(flags)
    try:
        assert r.get_shortcuts() == flags
        got = r.barcode(x, max_dim=max_dim, threshold=t, p=p)
        if not flags & r.SHORTCUT_CLEARING:
            r.set_shortcuts(flags | r.SHORTCUT_CLEARING)
            on = r.barcode(x, max_dim=max_dim, threshold=t, p=p)
    finally:
        r.set_shortcuts()
    for d in range(max_dim + 1):
        for f in ("birth", "death", "birth_simplex", "death_simplex"):
            assert np.array_equal(getattr(got.bars[d], f), getattr(ref.bars[d], f)), (name, d, f)
    for k in range(1, max_dim + 1):
        s = got.stats[k]
        assert s["candidates"] == ref.counts[k]
        if not flags & r.SHORTCUT_APPARENT:
            assert s["apparent_col"] == 0 and s["apparent_pivot"] == 0, (name, k)
            assert s["columns"] == s["candidates"] - s["cleared"], (name, k)
        if not flags & r.SHORTCUT_EMERGENT:
            assert s["emergent"] == 0, (name, k)
        if not flags & r.SHORTCUT_CLEARING:
            assert s["cleared"] == 0, (name, k)
            # a pivot of dimension k-1 is no zero apparent pair's birth, so
            # what clearing removed comes back as columns, and nothing else
            c = on.stats[k]
            assert s["columns"] == c["columns"] + c["cleared"], (name, k)


def test_defaults_restored_and_all_shortcuts_used():
    r = rips()
    assert r.get_shortcuts() == r.SHORTCUT_APPARENT | r.SHORTCUT_EMERGENT | r.SHORTCUT_CLEARING
    c = workloads.config(2)
    got = r.barcode(c["clouds"][0], max_dim=2, threshold=1.4, p=2)
    assert got.stats[1]["apparent_col"] > 0
    assert got.stats[2]["emergent"] > 0
    assert got.stats[1]["cleared"] > 0 and got.stats[2]["cleared"] > 0


@pytest.mark.parametrize("mode", [1, 2])
@pytest.mark.parametrize("name", ["cube-40-p5", "so3-1000", "torus4-2000"])
def test_bars_unchanged_with_r_stored_or_discarded(mode, name):
    """Table 3's storing / discarding of the reduced matrix R: the bars are
    the oracle's in every mode, and the stored entries order as the modes do
    (discarding keeps V only; storing keeps R whenever it fits)."""
    r = rips()
    print(f"[case] reduced storage {mode} {name}", flush=True)
    x, ref = case(name)
    _, _, max_dim, t, p = next(c for c in CASES if c[0] == name)
    r.set_reduced_storage(mode)
    try:
        assert r.get_reduced_storage() == mode
        got = r.barcode(x, max_dim=max_dim, threshold=t, p=p)
    finally:
        r.set_reduced_storage()
    # the modes order their stored entries within one working column; the
    # direct-mapped one (used with the default storage) keeps R whenever the
    # rule allows, far part or not, so the default is taken with the general one
    r.set_working_column(r.WORKING_COLUMN_GENERAL)
    try:
        auto = r.barcode(x, max_dim=max_dim, threshold=t, p=p)
    finally:
        r.set_working_column()
    for d in range(max_dim + 1):
        for f in ("birth", "death", "birth_simplex", "death_simplex"):
            assert np.array_equal(getattr(got.bars[d], f), getattr(ref.bars[d], f)), (name, d, f)
    for k in range(1, max_dim + 1):
        a, g = auto.stats[k]["entries_stored"], got.stats[k]["entries_stored"]
        assert (g <= a) if mode == r.R_DISCARD else (g >= a), (name, k, a, g)
    assert r.get_reduced_storage() == r.R_AUTO
