"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle
runs.  Holds no arithmetic of the method: only the random numbers."""
from __future__ import annotations

import numpy as np


def level_batch(seed: int = 0, count: int = 4096, lo_log2: float = 6.0, hi_log2: float = 16.0,
                balanced: bool = False):
    """A level-batch of `count` products with operand lengths log-uniform in
    [2^lo_log2, 2^hi_log2] limbs, drawn independently for a and b (so the
    batch is uneven), and limbs uniform in [0, 2^32): lengths of a, lengths of
    b, then the limbs of all a, then of all b, from one generator.  With
    `balanced`, b takes a's lengths (no draw for them)."""
    rng = np.random.default_rng(seed)
    la = np.rint(2 ** rng.uniform(lo_log2, hi_log2, count)).astype(np.int64)
    lb = la.copy() if balanced else np.rint(2 ** rng.uniform(lo_log2, hi_log2, count)).astype(np.int64)
    a = rng.integers(0, 2**32, size=int(la.sum()), dtype=np.uint64).astype(np.uint32)
    b = rng.integers(0, 2**32, size=int(lb.sum()), dtype=np.uint64).astype(np.uint32)
    a_off = np.concatenate([[0], np.cumsum(la)]).astype(np.uint64)
    b_off = np.concatenate([[0], np.cumsum(lb)]).astype(np.uint64)
    return a, a_off, b, b_off


def serving_requests(seed: int = 11621, count: int = 1100, lo_exp: float = 3.0, hi_exp: float = 7.0):
    """Request stream: n = floor(10^(lo + (hi-lo) u)), u uniform, and
    exponential inter-arrival draws (unit mean; scale by 1/rate)."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(0.0, 1.0, count)
    ns = np.floor(10 ** (lo_exp + (hi_exp - lo_exp) * u)).astype(np.int64)
    gaps = rng.exponential(1.0, count)
    return ns, gaps
