"""Walk-count budgets (the "scaled" policy) per workload.

Algorithm 1 sets B = ceil(448/eps^2) and
R = ceil(128 (L+1)^2 / (d_min^2 (1 - eps/2) (1/d_s + 1/d_t)^2)) from worst-case
bounds (Lemma 3.6 on the walk variance, Lemma 3.5 on beta, Chebyshev in the
proof of Theorem 3.8). At the workloads below those constants ask for
10^14 - 10^22 walk steps per query. The scaled policy keeps both formulas and
replaces 448 and 128 by c_B and c_R, the smallest values on a x2 ladder that
put at least 95% of the reference queries within eps of the exact distance.
"""

from __future__ import annotations

from . import binding

# workload key -> (c_B, c_R, how the constants were obtained)
BUDGETS = {
    "ba1k": (448.0 / 1024, 128.0 / 2 ** 17, "provisional"),
    "cl100k": (448.0 / 1024, 128.0 / 2 ** 18, "provisional"),
    "grid1414": (448.0 / 1024, 128.0 / 2 ** 22, "provisional"),
    "cl10m": (448.0 / 1024, 128.0 / 2 ** 18, "provisional"),
    "cl40m": (448.0 / 1024, 128.0 / 2 ** 18, "provisional"),
}


def budget_policy(workload: str, delta: float = 0.01, max_steps: int = 0) -> binding.BdPolicy:
    c_B, c_R, _ = BUDGETS[workload]
    return binding.policy("scaled", c_B=c_B, c_R=c_R, delta=delta, max_steps=max_steps)
