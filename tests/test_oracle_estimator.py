"""Pins of the oracle estimator (section 3.2, Lemmas 3.3/3.4, Theorem 3.8).

  * U-statistic with exact sums: Q from the oracle vs an exact rational
    evaluation of ((sum U)^2 - sum U^2)/(R(R-1)).
  * L = 0: walks have no randomness, so Q_k = (z_s/d_s - z_t/d_t)^2 exactly
    for every probe (eq. for phi-hat at L = 0).
  * Unbiasedness (eq. for phi-hat, Lemma 3.4): at a fixed probe, the mean of
    U_p tends to phi(z) = z^T h^(L) and the mean of Q_R to phi(z)^2, with
    h^(L) from the exact series.
  * Lemma 3.3: the mean over probes of phi(z)^2 tends to beta^(L).
  * Two-endpoint identity by brute force: enumerating every length-L path on
    a tiny graph gives E[phi-hat | z] = phi(z).
  * Median-of-means structure: block means of consecutive probes, median.
  * Theorem 3.8 with the paper's constants on tiny graphs.
"""

import itertools
from fractions import Fraction

import numpy as np
import pytest

from oracle import estimator as E
from oracle import exact, planner
from synth import graphs

SEED = 0x0B1A5ED5EED


def _inv32(d):
    return np.float32(1.0) / np.float32(d)


def test_q_matches_exact_rational():
    rng = np.random.default_rng(3)
    degs = rng.integers(1, 5000, size=64)
    invs = [_inv32(d) for d in degs]
    for R in (2, 3, 17, 256):
        U = []
        for _ in range(R):
            a = np.float32(0.0)
            for _ in range(int(rng.integers(1, 40))):
                v = invs[int(rng.integers(len(invs)))]
                a = np.float32(a + v) if rng.random() < 0.5 else np.float32(a - v)
            U.append(a)
        U = np.array(U, dtype=np.float32)
        S1 = sum(Fraction(float(u)) for u in U)
        S2 = sum(Fraction(float(u)) ** 2 for u in U)
        q_exact = (S1 * S1 - S2) / (R * (R - 1))
        scale = float((S1 * S1 + S2) / (R * (R - 1))) + 1e-300
        assert abs(E.q_from_u(U) - float(q_exact)) <= 1e-13 * scale


def test_L0_probe_statistic_is_exact():
    g = graphs.random_connected(31, 0.15, 6)
    d = g.deg
    s, t = 4, 20
    pol = planner.Policy("fixed", B_fixed=3, R_fixed=5)
    B, G, K, R = planner.plan(0.1, 0, d[s], d[t], g.d_min, pol)
    beta, q, ybar = E.estimate(g, [s], [t], 0, [(B, G, K, R)], SEED, uid=[7], want_q=True)
    for k in range(K):
        _, z, _ = E.probe(g.n, SEED, 7, k, nodes=np.array([s, t], dtype=np.uint32))
        u = np.float32(np.float32(z[0]) * _inv32(d[s]) - np.float32(z[1]) * _inv32(d[t]))
        assert q[k] == pytest.approx(float(u) ** 2, rel=1e-14, abs=1e-300)
    assert np.allclose(ybar, [q[i * B:(i + 1) * B].mean() for i in range(G)], rtol=1e-14, atol=0)
    assert beta[0] == np.median(ybar)


def test_L0_estimate_tends_to_beta0():
    g = graphs.random_connected(31, 0.15, 6)
    s, t = 4, 20
    pol = planner.Policy("fixed", B_fixed=400, R_fixed=2)
    plan = planner.plan(0.1, 0, 1, 1, 1, pol)
    beta, q, _ = E.estimate(g, [s], [t], 0, [plan], SEED, want_q=True)
    ref = exact.beta_truncated(g, s, t, 0)
    assert abs(q.mean() - ref) < 5 * q.std() / np.sqrt(q.size)


@pytest.mark.parametrize("L", [1, 5, 40])
def test_fixed_probe_unbiased(L):
    g = graphs.random_connected(25, 0.15, 12)
    s, t, k, uid = 2, 19, 3, 1
    _, z, _ = E.probe(g.n, SEED, uid, k)
    phi = exact.phi(g, s, t, L, z)
    N = 40000
    U = E.replicas(g, s, t, L, uid, k, 0, N, SEED).astype(np.float64)
    assert abs(U.mean() - phi) < 5 * U.std() / np.sqrt(N)
    R = 8
    Q = np.array([E.q_from_u(U[i:i + R].astype(np.float32)) for i in range(0, N, R)])
    assert abs(Q.mean() - phi ** 2) < 5 * Q.std() / np.sqrt(Q.size)


def test_lemma33_probe_average():
    g = graphs.random_connected(20, 0.2, 5)
    s, t, L = 1, 13, 6
    h = exact.h_truncated(g, s, t, L)
    nk = 30000
    ph2 = np.array([(E.probe(g.n, SEED, 0, k)[1].astype(np.float64) @ h) ** 2 for k in range(nk)])
    ref = exact.beta_truncated(g, s, t, L)
    assert abs(ph2.mean() - ref) < 5 * ph2.std() / np.sqrt(nk)


def test_two_endpoint_identity_brute_force():
    g = graphs.random_connected(6, 0.4, 1)
    rp, col, d = g.row_ptr, g.col, g.deg
    s, t, L = 0, 4, 3
    for k in range(5):
        _, z, _ = E.probe(g.n, SEED, 0, k)

        def expect(a):
            tot = 0.0
            for steps in itertools.product(*[range(int(d.max()))] * L):
                x, pr, acc = a, 1.0, z[a] / d[a]
                ok = True
                for j in steps:
                    if j >= d[x]:
                        ok = False
                        break
                    pr /= d[x]
                    x = col[rp[x] + j]
                    acc += z[x] / d[x]
                if ok:
                    tot += pr * acc
            return tot

        assert expect(s) - expect(t) == pytest.approx(exact.phi(g, s, t, L, z), abs=1e-12)


def test_deterministic_across_threads_and_uid():
    g = graphs.barabasi_albert(200, 3, 2)
    s = np.array([1, 5, 9, 100], dtype=np.int32)
    t = np.array([2, 50, 150, 199], dtype=np.int32)
    plan = [(2, 37, 74, 16)] * 4
    a = E.estimate(g, s, t, 30, plan, SEED, threads=1)
    b = E.estimate(g, s, t, 30, plan, SEED, threads=4)
    assert np.array_equal(a, b)
    c = E.estimate(g, s[2:3], t[2:3], 30, plan[:1], SEED, uid=[2])
    assert c[0] == a[2]
    d = E.estimate(g, s[2:3], t[2:3], 30, plan[:1], SEED, uid=[3])
    assert d[0] != a[2]


@pytest.mark.slow
@pytest.mark.parametrize("maker,s,t", [(lambda: graphs.cycle_graph(5), 0, 2),
                                       (lambda: graphs.complete_graph(5), 1, 3)])
def test_theorem38_paper_constants(maker, s, t):
    # Proof of Theorem 3.8: with the paper's B, G, R the median of block means
    # is within (eps/4) beta^(L) of beta^(L) with probability >= 1 - delta.
    g = maker()
    eps, L = 0.5, 2
    plan = planner.plan(eps, L, g.deg[s], g.deg[t], g.d_min)
    nq = 8
    beta = E.estimate(g, [s] * nq, [t] * nq, L, [plan] * nq, SEED, uid=np.arange(nq), threads=8)
    ref = exact.beta_truncated(g, s, t, L)
    assert np.all(np.abs(beta - ref) <= eps / 4 * ref)
