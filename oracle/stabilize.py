"""Truncation length by the paper's stabilization rule (section 4.3) -- oracle.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Start at L = L0 = 1; estimate beta at L and at 2L; accept L_stop = 2L (and the
estimate at 2L) once |beta-hat^(2L) - beta-hat^(L)| <= (eps/2) |beta-hat^(2L)|,
otherwise double L. Reading: doubling stops at L_max, where the estimate at
L_max is returned with L_stop = L_max.
"""

from __future__ import annotations

from . import estimator, planner


def stabilized(g, s: int, t: int, eps: float, L_max: int, seed: int, uid: int, policy: planner.Policy):
    """(beta-hat at L_stop, L_stop) for one query."""
    d = g.deg

    def est(L):
        plan = planner.plan(eps, L, int(d[s]), int(d[t]), g.d_min, policy)
        return float(estimator.estimate(g, [s], [t], L, [plan], seed, uid=[uid])[0])

    L = 1
    b_prev = est(L)
    if L_max == 1:
        return b_prev, 1
    while True:
        L2 = min(2 * L, L_max)
        b2 = est(L2)
        if abs(b2 - b_prev) <= 0.5 * eps * abs(b2) or L2 >= L_max:
            return b2, L2
        b_prev, L = b2, L2
