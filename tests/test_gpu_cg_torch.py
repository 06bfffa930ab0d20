"""The oracle's binary64 CG in plain torch, on the GPU (the route that writes
the n=1e7 and n=4e7 references), against the stored CPU CG of the 128
Chung-Lu n=1e5 reference pairs (scipy route, tests/golden): relative
difference at most 1e-9 on both solves. It runs torch's own sparse product,
not the HIP library."""

import os

import numpy as np
import pytest

from oracle import cg_torch
from synth import graphs

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "cl100k_cg_reference.txt")


def test_torch_cg_on_gpu_matches_cpu_cg():
    g = graphs.workload_graph("cl100k")
    ref = np.loadtxt(GOLDEN, comments="#")
    b1, b2, its, res = cg_torch.beta_cg_many(g, ref[:, 1], ref[:, 2], device="cuda", chunk=64)
    assert np.all(res <= 1e-12)
    assert np.abs(b1 - ref[:, 5]).max() <= 1e-9 * ref[:, 5].min()
    assert np.abs(b2 - ref[:, 5]).max() <= 1e-9 * ref[:, 5].min()
    bl = cg_torch.beta_truncated_many(g, ref[:8, 1], ref[:8, 2], 1000, device="cuda")
    assert np.allclose(bl, ref[:8, 7], rtol=1e-10, atol=0)
