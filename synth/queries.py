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


# Query sets of the workloads: (pairs, eps choices, L choices); eps and L are
# drawn per query when more than one value is listed.
WORKLOAD_QUERIES = {
    "ba1k": (256, (0.1,), (200,)),
    "cl100k": (4096, (0.05,), (1000,)),
    "grid1414": (65536, (0.02, 0.05, 0.1), (500, 2000, 5000)),
    "cl10m": (4096, (0.02, 0.05, 0.1), (1000,)),
    "cl40m": (262144, (0.05,), (1000, 10000)),
}


def workload_batch(key: str, n: int, count: int | None = None):
    """(s, t, eps, L) of a workload's query set (first ``count`` queries)."""
    from synth.graphs import GRAPH_SEED, QUERY_SEED_OFFSET, WORKLOAD_INDEX

    total, eps_choices, L_choices = WORKLOAD_QUERIES[key]
    seed = GRAPH_SEED + WORKLOAD_INDEX[key] + QUERY_SEED_OFFSET
    s, t = uniform_pairs(n, total, seed)
    eps, L = mixed_eps_L(total, eps_choices, L_choices, seed + 1)
    m = total if count is None else count
    return s[:m], t[:m], eps[:m], L[:m]


def served_requests(n: int, count: int, seed: int, max_log2: int = 12,
                    eps_choices=(0.02, 0.05, 0.1)):
    """``count`` request batches: sizes 2^U with U uniform on {0..max_log2}
    (1 to 4,096 pairs), uniform pairs, eps drawn per query. Returns a list of
    (s, t, eps) arrays."""
    rng = np.random.default_rng(seed)
    sizes = 2 ** rng.integers(0, max_log2 + 1, size=count)
    out = []
    for i, m in enumerate(sizes):
        s, t = uniform_pairs(n, int(m), seed + 1 + i)
        eps = np.asarray(eps_choices, dtype=np.float64)[rng.integers(0, len(eps_choices), size=int(m))]
        out.append((s, t, eps))
    return out


def poisson_arrivals(count: int, rate: float, seed: int) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson process of the given rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=count))
