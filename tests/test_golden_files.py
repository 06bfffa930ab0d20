"""The stored reference values of tests/golden match what the oracle and the
seeded generators produce now (CPU only).

  * cl100k_cg_reference.txt: the pairs are the workload's first 128, the two CG
    solves agree, and two sampled pairs are solved again.
  * grid1414_truncated_reference.txt: the pairs are the grid workload's first
    32 with their degrees; pair 0 at L = 500 is recomputed with the one-pair
    series (a different routine from the many-pair one that wrote the file);
    beta^(L) grows with L.
"""

import os

import numpy as np
import pytest

from oracle import exact
from synth import graphs, queries

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_cl100k_reference():
    ref = np.loadtxt(os.path.join(HERE, "cl100k_cg_reference.txt"), comments="#")
    g = graphs.workload_graph("cl100k")
    s, t, _, _ = queries.workload_batch("cl100k", g.n, 128)
    assert np.array_equal(ref[:, 1], s) and np.array_equal(ref[:, 2], t)
    assert np.array_equal(ref[:, 3], g.deg[s]) and np.array_equal(ref[:, 4], g.deg[t])
    assert np.all(np.abs(ref[:, 5] - ref[:, 6]) <= 1e-9 * ref[:, 5])
    for i in (0, 77):
        b1, _, _ = exact.beta_cg(g, int(s[i]), int(t[i]))
        assert b1 == pytest.approx(ref[i, 5], rel=1e-9)


def test_grid_reference():
    ref = np.loadtxt(os.path.join(HERE, "grid1414_truncated_reference.txt"), comments="#")
    g = graphs.workload_graph("grid1414")
    s, t, _, _ = queries.workload_batch("grid1414", g.n, 32)
    assert np.array_equal(ref[:, 1], s) and np.array_equal(ref[:, 2], t)
    assert np.array_equal(ref[:, 3], g.deg[s]) and np.array_equal(ref[:, 4], g.deg[t])
    assert np.all(np.diff(ref[:, 5:8], axis=1) > 0)
    b = exact.beta_truncated(g, int(s[0]), int(t[0]), 500)
    assert b == pytest.approx(ref[0, 5], rel=1e-12)
