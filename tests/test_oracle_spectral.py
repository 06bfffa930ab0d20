"""Pins of the oracle's spectral helpers, Theorem 3.8's L and the
stabilization rule (section 4.3)."""

import math

import numpy as np
import pytest

from oracle import exact, planner, stabilize
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


def test_stabilization_complete_graph():
    # On K_5, beta^(L) = (2/25)(1 - (-1/4)^(L+1))^2 settles within a few doublings.
    g = graphs.complete_graph(5)
    pol = planner.Policy("fixed", B_fixed=60, R_fixed=64)
    beta, L_stop = stabilize.stabilized(g, 1, 3, 0.1, 256, 0x5EED, 0, pol)
    assert L_stop in (2, 4, 8, 16)
    assert beta == pytest.approx(2.0 / 25.0, rel=0.1)
