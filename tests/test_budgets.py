"""The walk-count budgets of paper_2512_05460_amd/budgets.py: the policies it
hands to the library carry its constants, and the block and replica counts
its comments state follow from them under the planner of Algorithm 1 (the
oracle's copy)."""

import os

import numpy as np
import pytest

from oracle import planner as OP
from paper_2512_05460_amd import binding as B
from paper_2512_05460_amd.budgets import BUDGETS, SHARED_BUDGETS, budget_policy


@pytest.mark.parametrize("key", sorted(BUDGETS))
def test_policy_carries_the_constants(key):
    c_B, c_R, how = BUDGETS[key]
    p = budget_policy(key)
    assert p.kind == B.BD_POLICY_SCALED and p.c_B == c_B and p.c_R == c_R and p.delta == 0.01
    assert p.share <= 1
    assert how.startswith("calibrated") or how.startswith("throughput")


def test_shared_policy():
    M, c_B, c_R, _ = SHARED_BUDGETS["cl100k"]
    p = budget_policy("cl100k", shared=True)
    assert (p.share, p.c_B, p.c_R) == (M, c_B, c_R) and M == 4


def _B(key, eps):
    c_B, c_R, _ = BUDGETS[key]
    return OP.plan(eps, 1000, 1, 1, 1, OP.Policy("scaled", c_B=c_B, c_R=c_R))[0]


def test_stated_block_sizes():
    # G = 37 blocks at delta = 0.01; B per eps as the comments state
    assert OP.plan(0.05, 1000, 1, 1, 1, OP.Policy("scaled", c_B=0.64, c_R=1.0))[1] == 37
    assert _B("cl100k", 0.05) == 256
    assert [_B("cl10m", e) for e in (0.02, 0.05, 0.1)] == [100, 16, 4]
    assert [_B("grid1414", e) for e in (0.02, 0.05, 0.1)] == [16, 3, 1]
    assert _B("cl40m", 0.05) == 1
    assert _B("cl10m@1000", 0.05) == 384 and _B("cl40m@1000", 0.05) == 256
    assert _B("grid1414@2000", 0.05) == 256
    M, c_B, _, _ = SHARED_BUDGETS["cl100k"]
    assert OP.plan(0.05, 1000, 1, 1, 1, OP.Policy("scaled", c_B=c_B, c_R=1.0))[0] == 384


@pytest.mark.parametrize("L", [500, 2000, 5000])
def test_grid_replicas_per_L(L):
    # c_R = 16/(L+1)^2 on the grid (d_min 1): R from 37 to 68 for the endpoint
    # degrees of the 32 calibration pairs (tests/golden), whatever L
    ref = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "grid1414_truncated_reference.txt"),
                     comments="#")
    c_B, c_R, _ = BUDGETS[f"grid1414@{L}"]
    Rs = [OP.plan(e, L, int(ds), int(dt), 1, OP.Policy("scaled", c_B=c_B, c_R=c_R))[3]
          for e in (0.02, 0.05, 0.1) for ds, dt in ref[:, 3:5]]
    assert min(Rs) == 37 and max(Rs) == 68


@pytest.mark.parametrize("key,count,B_,R_median", [("ba1k", 256, 96, 176), ("cl100k", 128, 256, 934)])
def test_calibrated_budgets_on_their_pairs(key, count, B_, R_median):
    # the calibration sets: B and the median R over the reference pairs
    from synth import graphs, queries

    g = graphs.workload_graph(key)
    s, t, eps, L = queries.workload_batch(key, g.n, count)
    c_B, c_R, _ = BUDGETS[key]
    pol = OP.Policy("scaled", c_B=c_B, c_R=c_R)
    plans = [OP.plan(float(eps[i]), int(L[i]), int(g.deg[s[i]]), int(g.deg[t[i]]), g.d_min, pol)
             for i in range(count)]
    assert {p[0] for p in plans} == {B_}
    assert np.median([p[3] for p in plans]) == R_median


@pytest.mark.parametrize("key,B_,R_median,R_max", [("cl10m", 384, 716.5, 36201), ("cl40m", 256, 515.5, 6995)])
def test_large_graph_budgets_on_their_reference_pairs(key, B_, R_median, R_max):
    # the 64 CG reference pairs of the two large graphs (d_min = 1), L = 1000
    from paper_2512_05460_amd.calibrate import load_reference

    ref = load_reference(os.path.join(os.path.dirname(__file__), "golden", f"{key}_cg_reference.txt"))
    c_B, c_R, _ = BUDGETS[f"{key}@1000"]
    pol = OP.Policy("scaled", c_B=c_B, c_R=c_R)
    plans = [OP.plan(0.05, 1000, int(a), int(b), 1, pol) for a, b in zip(ref["d_s"], ref["d_t"])]
    assert {p[0] for p in plans} == {B_}
    R = [p[3] for p in plans]
    assert np.median(R) == R_median and max(R) == R_max
