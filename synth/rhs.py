"""Seeded random right-hand sides (input data only): Re and Im i.i.d. N(0, 1),
drawn with numpy's default_rng(seed) as an (L, n, 2) array, returned as a
complex128 (L, n) array, i.e. one contiguous length-n vector per frequency."""
from __future__ import annotations

import numpy as np


def random_complex(L: int, n: int, seed: int) -> np.ndarray:
    g = np.random.default_rng(seed).standard_normal((L, n, 2))
    return (g[..., 0] + 1j * g[..., 1]).astype(np.complex128)


def sample_rows(n: int, count: int, seed: int = 0) -> np.ndarray:
    """``count`` distinct row indices drawn uniformly without replacement."""
    count = min(count, n)
    return np.sort(np.random.default_rng(seed).choice(n, size=count, replace=False)).astype(np.int32)
