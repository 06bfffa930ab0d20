"""Pins of the oracle's walk sharing (probes of a block scored in groups of M
on common walks; an extension of Algorithm 1, which is the case M = 1).

  * Groups never hold more than a block: with B = 1 every group is one probe
    and the result is Algorithm 1's bit for bit.
  * The first probe of a group uses exactly the walks Algorithm 1 gives it
    (the group's streams are keyed by that probe), so its Q_k equals the
    unshared Q_k; this also fixes where groups start (every M-th probe inside
    each block, restarting at block boundaries).
  * Every other probe of a group: Q_k recomputed from the group's walk traces,
    the probe's own z values and a numpy binary32 sum in step order, with the
    U-statistic in exact rational arithmetic.
  * Unbiasedness survives sharing: the mean of Q_k over many groups tends to
    beta^(L) (Lemmas 3.3 and 3.4 hold per probe).
  * The sampled-probe routine scores a probe on its group's walks.
"""

from fractions import Fraction

import numpy as np
import pytest

from oracle import estimator as E
from oracle import exact, planner
from synth import graphs

SEED = 0x0B1A5ED5EED


def _group_first(k, B, M):
    blk = k // B
    return blk * B + ((k - blk * B) // M) * M


def test_block_of_one_is_algorithm1():
    g = graphs.random_connected(41, 0.12, 5)
    plan = (1, 9, 9, 6)
    a = E.estimate(g, [3, 7], [30, 2], 25, [plan] * 2, SEED)
    b = E.estimate(g, [3, 7], [30, 2], 25, [plan] * 2, SEED, share=4)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("B,M", [(6, 4), (5, 2), (8, 8), (3, 7)])
def test_group_starts_match_algorithm1(B, M):
    g = graphs.random_connected(37, 0.15, 8)
    s, t, L, G, R = 5, 22, 12, 5, 7
    plan = (B, G, B * G, R)
    _, q1, y1 = E.estimate(g, [s], [t], L, [plan], SEED, uid=[9], want_q=True)
    _, qm, ym = E.estimate(g, [s], [t], L, [plan], SEED, uid=[9], want_q=True, share=M)
    firsts = [k for k in range(B * G) if _group_first(k, B, M) == k]
    assert firsts == sorted({_group_first(k, B, M) for k in range(B * G)})
    assert np.array_equal(q1[firsts], qm[firsts])
    others = [k for k in range(B * G) if k not in firsts]
    if others:
        # different walks: the other probes' Q differ from Algorithm 1's
        assert not np.array_equal(q1[others], qm[others])


def _q_from_traces(g, s, t, L, uid, k, kw, R):
    _, z, _ = E.probe(g.n, SEED, uid, k)
    inv = (np.float32(1.0) / g.deg.astype(np.float32)).astype(np.float32)
    U = []
    for p in range(R):
        sums = []
        for start, side in ((s, 0), (t, 1)):
            tr, _ = E.walk_trace(g, start, L, SEED, uid, kw, p, side)
            a = np.float32(0.0)
            for x in tr:
                if z[x] > 0:
                    a = np.float32(a + inv[x])
                elif z[x] < 0:
                    a = np.float32(a - inv[x])
            sums.append(a)
        U.append(np.float32(sums[0] - sums[1]))
    S1 = sum(Fraction(float(u)) for u in U)
    S2 = sum(Fraction(float(u)) ** 2 for u in U)
    return (S1 * S1 - S2) / (R * (R - 1)), U


def test_shared_probe_from_traces():
    g = graphs.barabasi_albert(60, 2, 4)
    s, t, L, R = 2, 51, 9, 5
    B, G, M = 6, 3, 4
    plan = (B, G, B * G, R)
    _, q, _ = E.estimate(g, [s], [t], L, [plan], SEED, uid=[4], want_q=True, share=M)
    for k in (1, 3, 5, 7, 13, 17):
        kw = _group_first(k, B, M)
        assert kw != k
        ref, U = _q_from_traces(g, s, t, L, 4, k, kw, R)
        scale = float(sum(Fraction(float(u)) ** 2 for u in U)) / (R * (R - 1)) + 1e-300
        assert abs(q[k] - float(ref)) <= 1e-13 * scale, k
    # the sampled-probe routine agrees
    ks = np.arange(B * G, dtype=np.uint32)
    assert np.array_equal(E.probe_q(g, s, t, L, 4, R, SEED, ks, B=B, share=M), q)


@pytest.mark.parametrize("M", [2, 4])
def test_sharing_keeps_the_mean(M):
    # mean of Q_k over 40 * 32 probes vs the exact truncated distance
    g = graphs.random_connected(23, 0.2, 3)
    s, t, L = 1, 17, 6
    B, G, R = 32, 40, 8
    plan = (B, G, B * G, R)
    _, q, _ = E.estimate(g, [s], [t], L, [plan], SEED, uid=[11], want_q=True, share=M)
    ref = exact.beta_truncated(g, s, t, L)
    # groups of M probes share walks: the standard error comes from the G*B/M groups' means
    grp = q.reshape(-1, M).mean(axis=1)
    se = grp.std(ddof=1) / np.sqrt(grp.size)
    assert abs(q.mean() - ref) <= 5 * se, (q.mean(), ref, se)


def test_walk_steps_with_sharing():
    assert planner.walk_steps(6, 37, 10, 100, 1) == 2 * 6 * 37 * 10 * 100
    assert planner.walk_steps(6, 37, 10, 100, 4) == 2 * 2 * 37 * 10 * 100
    assert planner.walk_steps(8, 37, 10, 100, 4) == 2 * 2 * 37 * 10 * 100
    assert planner.walk_steps(1, 37, 10, 100, 4) == 2 * 37 * 10 * 100
