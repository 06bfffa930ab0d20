"""Pins of the oracle's random walks (Algorithm 1 walk loop, eq. for phi-hat).

  * every trajectory starts at its endpoint and moves along edges;
  * the neighbour choices are reproduced from Philox words by the stated
    counter layout (the generator itself is pinned by known answers);
  * the binary32 sum of z/d along a trajectory equals an independent numpy
    float32 recomputation from the trajectory and the probe values;
  * one step is uniform over N(x) (chi-square) and L steps follow P^L
    (total-variation distance).
"""

import numpy as np
import pytest
from scipy import stats

from oracle import estimator as E
from synth import graphs

SEED = 0x0B1A5ED5EED


def test_trajectory_follows_edges_and_counters():
    g = graphs.barabasi_albert(300, 3, 7)
    rp, col = g.row_ptr, g.col
    key = [SEED & 0xFFFFFFFF, SEED >> 32]
    for (start, k, p, side, uid) in [(0, 0, 0, 0, 0), (17, 5, 123, 1, 9), (299, 2 ** 20, 7, 0, 2 ** 30)]:
        L = 37
        tr, _ = E.walk_trace(g, start, L, SEED, uid, k, p, side)
        assert tr[0] == start
        words = None
        for i in range(1, L + 1):
            x = tr[i - 1]
            nb = col[rp[x]:rp[x + 1]]
            assert tr[i] in nb
            if (i - 1) % 4 == 0:
                words = E.philox([(i - 1) >> 2, p, k, (uid << 1) | side], key)
            u = int(words[(i - 1) % 4])
            j = (u * len(nb)) >> 32
            assert tr[i] == nb[j]


def test_walk_sum_matches_float32_recomputation():
    g = graphs.random_connected(50, 0.1, 3)
    deg = g.deg
    inv = (np.float32(1.0) / deg.astype(np.float32)).astype(np.float32)
    for (start, k, p, side) in [(0, 0, 0, 0), (11, 3, 40, 1), (49, 77, 5, 0)]:
        L = 200
        tr, acc = E.walk_trace(g, start, L, SEED, 4, k, p, side)
        _, z, _ = E.probe(g.n, SEED, 4, k)
        a = np.float32(0.0)
        for x in tr:
            if z[x] > 0:
                a = np.float32(a + inv[x])
            elif z[x] < 0:
                a = np.float32(a - inv[x])
        assert a == np.float32(acc)


def test_one_step_is_uniform_over_neighbours():
    g = graphs.barabasi_albert(400, 3, 1)
    hub = int(np.argmax(g.deg))
    nb = g.col[g.row_ptr[hub]:g.row_ptr[hub + 1]]
    counts = dict.fromkeys(nb.tolist(), 0)
    N = 30 * len(nb)
    for p in range(N):
        tr, _ = E.walk_trace(g, hub, 1, SEED, 0, 0, p, 0)
        counts[int(tr[1])] += 1
    obs = np.array(list(counts.values()))
    chi2 = ((obs - N / len(nb)) ** 2 / (N / len(nb))).sum()
    assert stats.chi2.sf(chi2, len(nb) - 1) > 1e-4


def test_L_steps_follow_transition_matrix():
    g = graphs.random_connected(12, 0.3, 8)
    A = g.scipy().toarray()
    P = A / A.sum(1, keepdims=True)
    L = 4
    start = 3
    target = np.linalg.matrix_power(P, L)[start]
    N = 40000
    hits = np.zeros(g.n)
    for p in range(N):
        tr, _ = E.walk_trace(g, start, L, SEED, 1, 2, p, 1)
        hits[tr[L]] += 1
    tv = 0.5 * np.abs(hits / N - target).sum()
    assert tv < 0.02
