"""Pins of the oracle's spectral helpers, Theorem 3.8's L and the
stabilization rule (section 4.3).

The rule: start at L = 1; estimate at L and 2L; accept L_stop = 2L and the
estimate at 2L once |beta-hat^(2L) - beta-hat^(L)| <= (eps/2)|beta-hat^(2L)|,
else double L; doubling stops at L_max (reading), returning the estimate there.
On K_5 the truncated distance is known in closed form,
beta^(L) = (2/25)(1 - (-1/4)^(L+1))^2, so with a budget that brings the
estimates within about 1% of it the accepted L and value are fixed:
L = 1 -> 2 differs by 14.8% (> eps/2 = 5% at eps = 0.1), 2 -> 4 by 2.9%
(accepted), so L_stop = 4 and the value is beta^(4), not beta^(2).
"""

import math

import numpy as np
import pytest

from oracle import estimator, exact, planner, stabilize
from synth import graphs


@pytest.mark.parametrize("n", [3, 5, 8, 20])
def test_mixing_factor_complete(n):
    # P = (J - I)/(n-1): eigenvalues 1 and -1/(n-1)
    assert exact.mixing_factor(graphs.complete_graph(n)) == pytest.approx(1.0 / (n - 1), rel=1e-12)


@pytest.mark.parametrize("n", [5, 9, 15])
def test_mixing_factor_odd_cycle(n):
    # eigenvalues cos(2 pi k / n); the most negative one is -cos(pi / n)
    assert exact.mixing_factor(graphs.cycle_graph(n)) == pytest.approx(math.cos(math.pi / n), rel=1e-12)


def test_mixing_factor_even_cycle_is_one():
    assert exact.mixing_factor(graphs.cycle_graph(8)) == pytest.approx(1.0, rel=1e-12)  # bipartite


def test_theorem_L_hand_worked():
    # n=1000, eps=0.1, lambda=0.5, d_s=d_t=2: log(96000/(0.1*0.25*1))/log 2 = log2(3840000) = 21.87 -> 22
    assert planner.theorem_L(1000, 0.1, 0.5, 2, 2) == 22
    # n=100, eps=0.5, lambda=0.9, d_s=4, d_t=4: log(9600/(0.5*0.01*0.25))/log(1/0.9) = 148.4 -> 149
    assert planner.theorem_L(100, 0.5, 0.9, 4, 4) == math.ceil(math.log(9600 / (0.5 * 0.01 * 0.25)) / math.log(1 / 0.9))


def _beta_k5(L):
    return (2.0 / 25.0) * (1.0 - (-0.25) ** (L + 1)) ** 2


K5_POL = planner.Policy("fixed", B_fixed=4000, R_fixed=16)


def test_stabilization_closed_form_k5():
    g = graphs.complete_graph(5)
    # the closed form against the oracle's own series first
    for L in (1, 2, 4):
        assert exact.beta_truncated(g, 1, 3, L) == pytest.approx(_beta_k5(L), rel=1e-13)
    beta, L_stop = stabilize.stabilized(g, 1, 3, 0.1, 256, 0x5EED, 0, K5_POL)
    assert L_stop == 4
    assert abs(beta - _beta_k5(4)) <= 0.015 * _beta_k5(4)
    assert abs(beta - _beta_k5(2)) > 0.015 * _beta_k5(2)  # not the estimate at L


def test_stabilization_cap_k5():
    # eps = 0.001: no doubling is accepted; the cap returns the estimate at L_max
    g = graphs.complete_graph(5)
    beta, L_stop = stabilize.stabilized(g, 1, 3, 0.001, 3, 0x5EED, 0, K5_POL)
    assert L_stop == 3
    assert abs(beta - _beta_k5(3)) <= 0.015 * _beta_k5(3)
    assert abs(beta - _beta_k5(2)) > 0.015 * _beta_k5(2)


def test_stabilization_acceptance_from_estimates():
    # The rule replayed on per-L estimates of the oracle's estimator: the
    # accepted pair must be (estimate at 2L, 2L) for the first L whose doubling
    # agrees within eps/2, or (estimate at L_max, L_max).
    g = graphs.barabasi_albert(60, 2, 5)
    pol = planner.Policy("scaled", c_B=0.02, c_R=4.0 / 65 ** 2)
    seen = set()
    for (s, t, eps, L_max) in [(0, 7, 0.1, 64), (3, 40, 0.2, 64), (11, 59, 0.05, 16), (5, 6, 0.3, 5),
                               (20, 21, 0.1, 1), (2, 33, 0.02, 32)]:
        def est(L):
            plan = planner.plan(eps, L, int(g.deg[s]), int(g.deg[t]), g.d_min, pol)
            return float(estimator.estimate(g, [s], [t], L, [plan], 0x77, uid=[9])[0])

        L, prev = 1, est(1)
        want = (prev, 1)
        while L_max > 1:
            L2 = min(2 * L, L_max)
            cur = est(L2)
            if abs(cur - prev) <= 0.5 * eps * abs(cur) or L2 >= L_max:
                want = (cur, L2)
                break
            L, prev = L2, cur
        got = stabilize.stabilized(g, s, t, eps, L_max, 0x77, 9, pol)
        assert got == want
        seen.add(want[1] == L_max)
    assert seen == {True, False}  # both an accepted doubling and the cap occur


def test_stabilization_complete_graph():
    # On K_5, beta^(L) = (2/25)(1 - (-1/4)^(L+1))^2 settles within a few doublings.
    g = graphs.complete_graph(5)
    pol = planner.Policy("fixed", B_fixed=60, R_fixed=64)
    beta, L_stop = stabilize.stabilized(g, 1, 3, 0.1, 256, 0x5EED, 0, pol)
    assert L_stop in (2, 4, 8, 16)
    assert beta == pytest.approx(2.0 / 25.0, rel=0.1)
