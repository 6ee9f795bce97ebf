"""The oracle over many clouds at once, in worker processes on the host CPU.

Test infrastructure only: the workers import the oracle (a ctypes library)
and numpy, never torch or the GPU library, and they are started with the
"spawn" method so that no worker inherits a process that has initialised
the GPU. Each worker returns only the bars and the threshold of its cloud.
"""

from __future__ import annotations

import multiprocessing as mp
import os

import numpy as np


def _oracle_bars(args):
    points, max_dim, threshold, p = args
    import oracle
    r = oracle.barcode(points, max_dim=max_dim, threshold=threshold, p=p)
    return ([(b.birth, b.death, b.birth_simplex, b.death_simplex) for b in r.bars],
            r.threshold)


def workers() -> int:
    """Host threads this process may use, at most 16 (the CPU share of one
    GPU machine)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


class OraclePool:
    """Starts the oracle on every cloud at construction (largest first, so
    that the long ones do not come last) and hands the results out by
    cloud number; use as a context manager."""

    def __init__(self, clouds, max_dim: int = 1, threshold: float = float("inf"), p: int = 2,
                 jobs=None):
        """clouds with one (max_dim, threshold, p) for all, or jobs: a list of
        (points, max_dim, threshold, p), one per result."""
        if jobs is None:
            jobs = [(c, max_dim, threshold, p) for c in clouds]
        self._pool = mp.get_context("spawn").Pool(min(workers(), max(1, len(jobs))))
        order = sorted(range(len(jobs)), key=lambda b: -int(np.asarray(jobs[b][0]).shape[0]))
        self._async = {b: self._pool.apply_async(_oracle_bars, (jobs[b],)) for b in order}

    def get(self, b: int, timeout: float = 900.0):
        return self._async[b].get(timeout)

    def close(self):
        self._pool.terminate()
        self._pool.join()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False
