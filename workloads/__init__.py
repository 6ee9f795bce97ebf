"""Seeded synthetic point clouds shaped like the paper's benchmark workloads.

This module only draws random inputs. It holds none of the persistence
method's arithmetic (no distances, no thresholds, no simplices), so both the
CPU oracle and the GPU library can be fed from it without sharing any code of
the method.

Every generator draws in float64 with numpy's PCG64 bit generator and returns
float32 arrays (row-major, shape (n, m)); the float32 bytes are what every path
reads. Seeds are ``SEED_BASE + cfg_id`` for single clouds and
``SEED_BASE + cfg_id + 1000 * cloud_id`` for batches.

The shapes stand in for the data sets of the paper's experiments section
(sphere3: points on the unit 2-sphere; o3: random orthogonal 3x3 matrices;
torus4: points on the Clifford torus), whose files are not available here.
"""

from __future__ import annotations

import numpy as np

SEED_BASE = 190802518

__all__ = [
    "SEED_BASE",
    "rng",
    "sphere",
    "so3",
    "orthogonal",
    "clifford_torus",
    "mixture_cloud",
    "mixture_batch",
    "noisy_circle_with_outliers",
    "circle_batch",
    "rectangle",
    "regular_polygon",
    "uniform_cube",
    "integer_lattice",
    "config",
    "CONFIGS",
    "PAPER_SCALE",
]


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _f32(x: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))


def sphere(n: int, seed: int) -> np.ndarray:
    """n points uniform on the unit sphere S^2 in R^3 (normalised Gaussians)."""
    g = rng(seed)
    x = g.standard_normal((n, 3))
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    return _f32(x)


def _quat_to_rot(q: np.ndarray) -> np.ndarray:
    """Unit quaternions (k, 4) -> rotation matrices (k, 3, 3)."""
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    r = np.empty((q.shape[0], 3, 3))
    r[:, 0, 0] = 1 - 2 * (y * y + z * z)
    r[:, 0, 1] = 2 * (x * y - z * w)
    r[:, 0, 2] = 2 * (x * z + y * w)
    r[:, 1, 0] = 2 * (x * y + z * w)
    r[:, 1, 1] = 1 - 2 * (x * x + z * z)
    r[:, 1, 2] = 2 * (y * z - x * w)
    r[:, 2, 0] = 2 * (x * z - y * w)
    r[:, 2, 1] = 2 * (y * z + x * w)
    r[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return r


def so3(n: int, seed: int) -> np.ndarray:
    """n Haar-random rotations of R^3, each flattened row-major to R^9."""
    g = rng(seed)
    q = g.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return _f32(_quat_to_rot(q).reshape(n, 9))


def orthogonal(n: int, seed: int) -> np.ndarray:
    """n Haar-random orthogonal 3x3 matrices (the group O(3): a Haar rotation
    times an independent sign, so half have determinant -1), each flattened
    row-major to R^9. The two components lie at Frobenius distance >= 2."""
    g = rng(seed)
    q = g.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    sign = np.where(g.random(n) < 0.5, -1.0, 1.0)
    return _f32((_quat_to_rot(q) * sign[:, None, None]).reshape(n, 9))


def clifford_torus(n: int, sigma: float, seed: int) -> np.ndarray:
    """(cos a, sin a, cos b, sin b) + N(0, sigma^2 I_4), a, b ~ U[0, 2pi)."""
    g = rng(seed)
    a = g.uniform(0.0, 2.0 * np.pi, n)
    b = g.uniform(0.0, 2.0 * np.pi, n)
    x = np.stack([np.cos(a), np.sin(a), np.cos(b), np.sin(b)], axis=1)
    x += sigma * g.standard_normal((n, 4))
    return _f32(x)


def _haar_rotation(g: np.random.Generator) -> np.ndarray:
    q = g.standard_normal(4)
    q /= np.linalg.norm(q)
    return _quat_to_rot(q[None, :])[0]


def mixture_cloud(seed: int, n_min: int = 32, n_max: int = 256) -> np.ndarray:
    """One cloud in R^3: 1-3 noisy circles and 0-2 Gaussian blobs.

    n ~ U{n_min..n_max}; circles: radius U[0.5, 2], random plane (Haar
    rotation), centre U[-4, 4]^3, noise N(0, 0.05^2 I_3); blobs:
    N(centre, 0.3^2 I_3). Points are split multinomially over the
    components with at least one point per component.
    """
    g = rng(seed)
    n = int(g.integers(n_min, n_max + 1))
    n_circ = int(g.integers(1, 4))
    n_blob = int(g.integers(0, 3))
    k = n_circ + n_blob
    counts = np.ones(k, dtype=np.int64) + g.multinomial(n - k, np.full(k, 1.0 / k))
    parts = []
    for c in range(k):
        centre = g.uniform(-4.0, 4.0, 3)
        m = int(counts[c])
        if c < n_circ:
            radius = g.uniform(0.5, 2.0)
            rot = _haar_rotation(g)
            th = g.uniform(0.0, 2.0 * np.pi, m)
            local = np.stack([radius * np.cos(th), radius * np.sin(th), np.zeros(m)], axis=1)
            pts = local @ rot.T + centre + 0.05 * g.standard_normal((m, 3))
        else:
            pts = centre + 0.3 * g.standard_normal((m, 3))
        parts.append(pts)
    x = np.concatenate(parts, axis=0)
    x = x[g.permutation(n)]
    return _f32(x)


def mixture_batch(num: int = 512, cfg_id: int = 4, n_min: int = 32, n_max: int = 256):
    """Batch of mixture clouds; returns a list of float32 (n_b, 3) arrays."""
    return [mixture_cloud(SEED_BASE + cfg_id + 1000 * b, n_min, n_max) for b in range(num)]


def noisy_circle_with_outliers(seed: int, n_circle: int = 360, n_out: int = 40,
                               sigma: float = 0.1) -> np.ndarray:
    """Unit circle in R^2 with N(0, sigma^2 I_2) noise plus uniform outliers in [-2, 2]^2."""
    g = rng(seed)
    th = g.uniform(0.0, 2.0 * np.pi, n_circle)
    circ = np.stack([np.cos(th), np.sin(th)], axis=1) + sigma * g.standard_normal((n_circle, 2))
    out = g.uniform(-2.0, 2.0, (n_out, 2))
    x = np.concatenate([circ, out], axis=0)
    x = x[g.permutation(n_circle + n_out)]
    return _f32(x)


def circle_batch(num: int = 64, cfg_id: int = 5, n_circle: int = 360, n_out: int = 40):
    return [noisy_circle_with_outliers(SEED_BASE + cfg_id + 1000 * b, n_circle, n_out)
            for b in range(num)]


def rectangle() -> np.ndarray:
    """The 3x4 rectangle used as the running example of the paper's filtration section."""
    return np.array([[0.0, 0.0], [3.0, 0.0], [0.0, 4.0], [3.0, 4.0]], dtype=np.float32)


def regular_polygon(n: int) -> np.ndarray:
    """Vertices of a regular n-gon on the unit circle (float32)."""
    th = 2.0 * np.pi * np.arange(n) / n
    return _f32(np.stack([np.cos(th), np.sin(th)], axis=1))


def uniform_cube(n: int, m: int, seed: int) -> np.ndarray:
    g = rng(seed)
    return _f32(g.uniform(0.0, 1.0, (n, m)))


def integer_lattice(n: int, m: int, seed: int, side: int = 4) -> np.ndarray:
    """Points with small integer coordinates: many tied distances and duplicates."""
    g = rng(seed)
    return _f32(g.integers(0, side, (n, m)))


# name -> (generator thunk, max_dim, threshold (inf = none), p)
def config(cfg_id: int):
    """The five benchmark workloads (1-5), and four at paper scale: 6, the shape
    of the paper's o3 run on 1024 orthogonal matrices (threshold 1.8, homology
    up to dimension 3); 7, a 10,000-point Clifford torus (threshold 0.25, up
    to dimension 2); 8, the o3 run at the paper's full size, 4096 matrices
    (threshold 1.4, up to dimension 3); 9, the paper's torus4 run, 50,000
    points on the Clifford torus (threshold 0.15, up to dimension 2).
    Returns a dict describing one of them."""
    inf = float("inf")
    if cfg_id == 1:
        return dict(name="sphere-100", clouds=[sphere(100, SEED_BASE + 1)], max_dim=1,
                    threshold=inf, p=2)
    if cfg_id == 2:
        return dict(name="so3-1000", clouds=[so3(1000, SEED_BASE + 2)], max_dim=2,
                    threshold=1.4, p=2)
    if cfg_id == 3:
        return dict(name="torus4-2000", clouds=[clifford_torus(2000, 0.02, SEED_BASE + 3)],
                    max_dim=2, threshold=0.5, p=3)
    if cfg_id == 4:
        return dict(name="mixture-512x[32,256]", clouds=mixture_batch(512, 4), max_dim=1,
                    threshold=inf, p=2)
    if cfg_id == 5:
        return dict(name="circles-64x400", clouds=circle_batch(64, 5), max_dim=1,
                    threshold=inf, p=2)
    if cfg_id == 6:
        return dict(name="o3-1024-t1.8", clouds=[orthogonal(1024, SEED_BASE + 6)], max_dim=3,
                    threshold=1.8, p=2)
    if cfg_id == 7:
        return dict(name="torus4-10000-t0.25", clouds=[clifford_torus(10000, 0.02, SEED_BASE + 7)],
                    max_dim=2, threshold=0.25, p=2)
    if cfg_id == 8:
        return dict(name="o3-4096-t1.4", clouds=[orthogonal(4096, SEED_BASE + 8)], max_dim=3,
                    threshold=1.4, p=2)
    if cfg_id == 9:
        return dict(name="torus4-50000-t0.15", clouds=[clifford_torus(50000, 0.0, SEED_BASE + 9)],
                    max_dim=2, threshold=0.15, p=2)
    raise ValueError(cfg_id)


CONFIGS = (1, 2, 3, 4, 5)
PAPER_SCALE = (6, 7, 8, 9)
