"""Pins of the exact-distance oracle (Definition 2.1, Eq. (1), Lemmas 2.2/2.3).

Every expected value here comes from a closed form or an identity that the
mathematics fixes, never from the code under test:
  * complete graph K_n: L = nH, so L^+ = H/n and beta = 2/n^2;
  * cycle C_n with arc lengths D and c = n - D: beta = Dc(Dc+2)/(12n);
  * path P_n, s < t, D = t - s, p = s + 1 (0-based s): the unit-current
    potential is D on nodes <= s, falls by one per edge to 0 at t, and is 0
    beyond; centring it gives
    beta = p D^2 + D(D-1)(2D-1)/6 - (p D + D(D-1)/2)^2 / n;
  * truncated K_n: P^i D^{-1} b = (-1/(n-1))^i b/(n-1), so
    beta^(L) = (2/n^2) (1 - (-1/(n-1))^(L+1))^2;
  * L = 0 on any graph: beta^(0) = (1/d_s^2 + 1/d_t^2) - (1/d_s - 1/d_t)^2/n;
  * Lemma 3.5: beta >= (1/8)(1/d_s + 1/d_t)^2; and n^-2 <= beta <= n^3.
"""

import itertools

import numpy as np
import pytest

from oracle import exact
from synth import graphs


def _pairs(n):
    return [(s, t) for s, t in itertools.permutations(range(n), 2)]


@pytest.mark.parametrize("n", [2, 3, 5, 8, 13])
def test_complete_graph(n):
    g = graphs.complete_graph(n)
    Lp = exact.pinv_dense(g)
    for s, t in _pairs(n):
        b1, b2 = exact.beta_dense(g, s, t, Lp)
        assert b1 == pytest.approx(2.0 / n ** 2, rel=1e-12)
        assert b2 == pytest.approx(2.0 / n ** 2, rel=1e-10)


@pytest.mark.parametrize("n", [3, 4, 7, 10, 15])
def test_cycle_closed_form(n):
    g = graphs.cycle_graph(n)
    Lp = exact.pinv_dense(g)
    for s, t in _pairs(n):
        D = (t - s) % n
        c = n - D
        ref = D * c * (D * c + 2) / (12.0 * n)
        b1, b2 = exact.beta_dense(g, s, t, Lp)
        assert b1 == pytest.approx(ref, rel=1e-11)
        assert b2 == pytest.approx(ref, rel=1e-9)


@pytest.mark.parametrize("n", [2, 4, 7, 12])
def test_path_closed_form(n):
    g = graphs.path_graph(n)
    Lp = exact.pinv_dense(g)
    for s in range(n):
        for t in range(s + 1, n):
            p, D = s + 1, t - s
            ref = p * D * D + D * (D - 1) * (2 * D - 1) / 6.0 - (p * D + D * (D - 1) / 2.0) ** 2 / n
            b1, b2 = exact.beta_dense(g, s, t, Lp)
            assert b1 == pytest.approx(ref, rel=1e-10)
            assert exact.beta_dense(g, t, s, Lp)[0] == pytest.approx(ref, rel=1e-10)


def test_cg_two_solves_agree_with_dense():
    g = graphs.random_connected(60, 0.08, 5)
    Lp = exact.pinv_dense(g)
    rng = np.random.default_rng(0)
    for _ in range(10):
        s, t = rng.choice(g.n, 2, replace=False)
        b_dense = exact.beta_dense(g, s, t, Lp)[0]
        b1, b2, _ = exact.beta_cg(g, int(s), int(t))
        assert b1 == pytest.approx(b_dense, rel=1e-9)
        assert b2 == pytest.approx(b_dense, rel=1e-9)


def test_cg_on_cycle_closed_form():
    n = 301
    g = graphs.cycle_graph(n)
    for s, t in [(0, 1), (0, 150), (7, 100)]:
        D = (t - s) % n
        c = n - D
        ref = D * c * (D * c + 2) / (12.0 * n)
        b1, b2, _ = exact.beta_cg(g, s, t)
        assert b1 == pytest.approx(ref, rel=1e-9)
        assert b2 == pytest.approx(ref, rel=1e-9)


@pytest.mark.parametrize("n,L", [(5, 0), (5, 1), (5, 2), (6, 7), (9, 30)])
def test_truncated_complete_graph(n, L):
    g = graphs.complete_graph(n)
    q = -1.0 / (n - 1)
    ref = 2.0 / n ** 2 * (1.0 - q ** (L + 1)) ** 2
    assert exact.beta_truncated(g, 0, 3, L) == pytest.approx(ref, rel=1e-12)


def test_truncated_multi_complete_graph_and_L0():
    # all pairs of K_n share the closed form; several L from one pass
    n = 7
    g = graphs.complete_graph(n)
    q = -1.0 / (n - 1)
    Ls = [0, 1, 3, 12]
    out = exact.beta_truncated_multi(g, [0, 2, 6], [3, 5, 1], Ls)
    for i, L in enumerate(Ls):
        ref = 2.0 / n ** 2 * (1.0 - q ** (L + 1)) ** 2
        assert out[i] == pytest.approx([ref] * 3, rel=1e-12)
    # L = 0 and large L on a non-complete graph: the L = 0 formula and beta
    g = graphs.random_connected(30, 0.15, 9)
    d = g.deg
    s, t = np.array([0, 4, 29]), np.array([1, 17, 3])
    out = exact.beta_truncated_multi(g, s, t, [0, 2000])
    ref0 = (1 / d[s] ** 2 + 1 / d[t] ** 2) - (1 / d[s] - 1 / d[t]) ** 2 / g.n
    assert out[0] == pytest.approx(ref0, rel=1e-13)
    Lp = exact.pinv_dense(g)
    ref = [exact.beta_dense(g, int(a), int(b), Lp)[0] for a, b in zip(s, t)]
    assert out[1] == pytest.approx(ref, rel=1e-9)


def test_truncated_L0_formula():
    g = graphs.random_connected(30, 0.15, 9)
    d = g.deg
    n = g.n
    for s, t in [(0, 1), (4, 17), (29, 3)]:
        ref = (1 / d[s] ** 2 + 1 / d[t] ** 2) - (1 / d[s] - 1 / d[t]) ** 2 / n
        assert exact.beta_truncated(g, s, t, 0) == pytest.approx(ref, rel=1e-13)


def test_truncation_converges_to_exact():
    # Lemma 2.3: beta^(L) -> beta on a connected non-bipartite graph.
    g = graphs.random_connected(40, 0.1, 2)
    Lp = exact.pinv_dense(g)
    s, t = 3, 31
    b = exact.beta_dense(g, s, t, Lp)[0]
    gaps = [abs(exact.beta_truncated(g, s, t, L) - b) / b for L in (10, 50, 200, 800)]
    assert gaps[-1] < 1e-9
    assert gaps[0] > gaps[1] > gaps[2]


def test_lemma35_lower_bound_and_range():
    for g in [graphs.random_connected(25, 0.2, 1), graphs.complete_graph(7),
              graphs.cycle_graph(9), graphs.path_graph(6),
              graphs.barabasi_albert(40, 2, 3)]:
        Lp = exact.pinv_dense(g)
        d = g.deg
        n = g.n
        for s, t in _pairs(n):
            b = exact.beta_dense(g, s, t, Lp)[0]
            assert b >= (1 / 8) * (1 / d[s] + 1 / d[t]) ** 2 * (1 - 1e-12)
            assert n ** -2 * (1 - 1e-12) <= b <= n ** 3


def test_alternative_expression_lemma22():
    # beta = ||h||^2 - (1^T h)^2/n with the full series (Lemma 2.2), approximated
    # by a long truncation, equals the dense value.
    g = graphs.random_connected(20, 0.2, 4)
    Lp = exact.pinv_dense(g)
    h = exact.h_truncated(g, 2, 11, 3000)
    b_series = h @ h - h.sum() ** 2 / g.n
    assert b_series == pytest.approx(exact.beta_dense(g, 2, 11, Lp)[0], rel=1e-9)


@pytest.mark.parametrize("maker,closed", [
    (lambda: graphs.complete_graph(9), lambda n, s, t: 2.0 / n ** 2),
    (lambda: graphs.cycle_graph(11),
     lambda n, s, t: ((t - s) % n) * (n - (t - s) % n) * (((t - s) % n) * (n - (t - s) % n) + 2) / (12.0 * n)),
])
def test_beta_dense_all_closed_forms(maker, closed):
    # the many-pairs routine (the reference of the BA accuracy test) on every
    # ordered pair, against the closed forms and the one-pair routine
    g = maker()
    s, t = zip(*_pairs(g.n))
    got = exact.beta_dense_all(g, s, t)
    for j, (a, b) in enumerate(zip(s, t)):
        assert got[j] == pytest.approx(closed(g.n, a, b), rel=1e-11)
        assert got[j] == pytest.approx(exact.beta_dense(g, a, b)[0], rel=1e-13)


def test_beta_dense_all_path_closed_form():
    n = 9
    g = graphs.path_graph(n)
    s, t = zip(*_pairs(n))
    got = exact.beta_dense_all(g, s, t)
    for j, (a, b) in enumerate(zip(s, t)):
        lo, hi = min(a, b), max(a, b)  # beta is symmetric in (s, t)
        p, D = lo + 1, hi - lo
        ref = p * D * D + D * (D - 1) * (2 * D - 1) / 6.0 - (p * D + D * (D - 1) / 2.0) ** 2 / n
        assert got[j] == pytest.approx(ref, rel=1e-10)


def test_beta_dense_all_random_graph_vs_one_pair():
    g = graphs.random_connected(40, 0.15, 3)
    rng = np.random.default_rng(1)
    s = rng.integers(0, 40, 60)
    t = (s + 1 + rng.integers(0, 39, 60)) % 40
    got = exact.beta_dense_all(g, s, t)
    ref = np.array([exact.beta_dense(g, int(a), int(b))[0] for a, b in zip(s, t)])
    assert np.allclose(got, ref, rtol=1e-12, atol=0)
    # Lemma 3.5 lower bound on every pair
    assert np.all(got >= (1 / 8) * (1.0 / g.deg[s] + 1.0 / g.deg[t]) ** 2)
