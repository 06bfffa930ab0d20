"""Pins of the oracle planner (Algorithm 1 parameters, Theorem 3.8).

Expected values are worked by hand from the formulas with exact rationals.
"""

import math
from fractions import Fraction

import pytest

from oracle import planner


@pytest.mark.parametrize("eps,B", [
    (0.01, 4_480_000), (0.02, 1_120_000), (0.04, 280_000), (0.05, 179_200),
    (0.06, 124_445), (0.1, 44_800), (0.2, 11_200), (0.5, 1_792),
])
def test_paper_B(eps, B):
    b, G, K, R = planner.plan(eps, 10, 3, 3, 3)
    assert b == B
    assert G == 37  # ceil(8 ln 100) = ceil(36.84)
    assert K == B * 37


def test_G_natural_log():
    assert planner.plan(0.1, 1, 1, 1, 1, planner.Policy(delta=0.05))[1] == 24  # 8 ln 20 = 23.97
    assert planner.plan(0.1, 1, 1, 1, 1, planner.Policy(delta=0.5))[1] == 6    # 8 ln 2 = 5.55


def _exact_R(eps, L, ds, dt, dmin, c=128):
    e = Fraction(eps).limit_denominator(10 ** 6)
    val = Fraction(c * (L + 1) ** 2) / (dmin ** 2 * (1 - e / 2) * (Fraction(1, ds) + Fraction(1, dt)) ** 2)
    return max(2, math.ceil(val))


@pytest.mark.parametrize("eps,L,ds,dt,dmin,R", [
    (0.1, 200, 3, 3, 3, 1_360_876),     # 128*201^2/(9*0.95*4/9) = 1360875.79
    (0.5, 2, 2, 2, 2, 384),             # 128*9/(4*0.75*1)
    (0.05, 1000, 4, 4, 1, None),
    (0.3, 3, 4, 4, 4, None),
    (0.02, 5000, 4, 3, 1, None),
])
def test_paper_R(eps, L, ds, dt, dmin, R):
    ref = _exact_R(eps, L, ds, dt, dmin)
    if R is not None:
        assert ref == R
    assert planner.plan(eps, L, ds, dt, dmin)[3] == ref


def test_L0_gives_R_at_least_2():
    # (L+1)^2 = 1, d_min = 1, d_s = d_t = 1: 128/(0.95*4) = 33.7
    assert planner.plan(0.1, 0, 1, 1, 1)[3] == 34
    assert planner.plan(0.9, 0, 1, 1, 1, planner.Policy("scaled", c_B=1, c_R=1e-6))[3] == 2


def test_scaled_and_fixed():
    p = planner.Policy("scaled", c_B=0.5, c_R=0.001)
    B, G, K, R = planner.plan(0.05, 1000, 10, 10, 1, p)
    assert B == 200  # 0.5/0.0025
    assert R == math.ceil(0.001 * 1001 ** 2 / (0.975 * 0.04) * (1 - 2 ** -40))
    B, G, K, R = planner.plan(0.05, 1000, 10, 10, 1, planner.Policy("fixed", B_fixed=3, R_fixed=64))
    assert (B, G, K, R) == (3, 37, 111, 64)
