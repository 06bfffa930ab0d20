"""Walk counts of Algorithm 1 (section 3, Theorem 3.8) -- oracle copy.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Algorithm 1 sets
    B = ceil(448 / eps^2),  G = ceil(8 ln(1/delta)),  K = B G,
    R = ceil(128 (L+1)^2 / (d_min^2 (1 - eps/2) (1/d_s + 1/d_t)^2)),
from the proof of Theorem 3.8 (R = 4 sigma_0^2 / theta_0 with the variance
bound of Lemma 3.6 and the distance lower bound of Lemma 3.5).

Readings:
  * ``log`` in G is the natural logarithm: the proof of Theorem 3.8 uses
    exp(-G/8) <= delta.
  * Every ceiling is taken as ceil(x (1 - 2^-40)) so that a quotient that
    lands a few ulps above an integer in binary64 is not bumped up by one.
  * R is at least 2 (the U-statistic needs two replicas, Lemma 3.4).
  * Policies: "paper" uses 448 and 128; "scaled" keeps the formulas with
    smaller constants (c_B, c_R); "fixed" takes B and R as given.
  * ``share`` (walk sharing, an extension): the probes of a block are scored
    in groups of ``share`` on common walks; B, G, K and R are unchanged and
    the walk count drops by about that factor.
"""

from __future__ import annotations

import dataclasses
import math

GUARD = 1.0 - 2.0 ** -40


def ceil_guarded(x: float) -> int:
    return int(math.ceil(x * GUARD))


@dataclasses.dataclass(frozen=True)
class Policy:
    kind: str = "paper"  # "paper" | "scaled" | "fixed"
    c_B: float = 448.0
    c_R: float = 128.0
    delta: float = 0.01
    B_fixed: int = 0
    R_fixed: int = 0
    share: int = 1  # walk-sharing group size M (1 = Algorithm 1)


PAPER = Policy()


def plan(eps: float, L: int, d_s: int, d_t: int, d_min: int, policy: Policy = PAPER):
    """Return (B, G, K, R) for one query."""
    G = ceil_guarded(8.0 * math.log(1.0 / policy.delta))
    if policy.kind == "fixed":
        B, R = int(policy.B_fixed), int(policy.R_fixed)
    else:
        c_B, c_R = (448.0, 128.0) if policy.kind == "paper" else (policy.c_B, policy.c_R)
        B = ceil_guarded(c_B / (eps * eps))
        theta_scale = (1.0 - eps / 2.0) * (1.0 / d_s + 1.0 / d_t) ** 2
        R = ceil_guarded(c_R * (L + 1) ** 2 / (d_min * d_min * theta_scale))
    B = max(B, 1)
    R = max(R, 2)
    return B, G, B * G, R


def walk_steps(B: int, G: int, R: int, L: int, share: int = 1) -> int:
    """Transitions a query runs: 2 R L per walk pair, R pairs per group of
    ``share`` probes, ceil(B / share) groups in each of the G blocks."""
    groups = G * -(-B // max(1, share))
    return 2 * groups * R * L


def theorem_L(n: int, eps: float, lam: float, d_s: int, d_t: int) -> int:
    """Truncation length of Theorem 3.8 (Algorithm 1, first line)."""
    arg = 96.0 * n / (eps * (1.0 - lam) ** 2 * (1.0 / d_s + 1.0 / d_t) ** 2)
    return ceil_guarded(math.log(arg) / math.log(1.0 / lam))
