"""Seeded query generators: uniform (s, t) pairs and mixed (eps, L) draws."""

from __future__ import annotations

import numpy as np


def uniform_pairs(n: int, count: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """``count`` pairs drawn uniformly from ordered pairs of distinct nodes."""
    rng = np.random.default_rng(seed)
    s = rng.integers(0, n, size=count, dtype=np.int64)
    t = rng.integers(0, n - 1, size=count, dtype=np.int64)
    t = t + (t >= s)  # uniform over [n] \ {s}
    return s.astype(np.int32), t.astype(np.int32)


def mixed_eps_L(count: int, eps_choices, L_choices, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """i.i.d. uniform draws of eps and L from the given finite sets."""
    rng = np.random.default_rng(seed)
    eps = np.asarray(eps_choices, dtype=np.float64)[rng.integers(0, len(eps_choices), size=count)]
    L = np.asarray(L_choices, dtype=np.int32)[rng.integers(0, len(L_choices), size=count)]
    return eps, L
