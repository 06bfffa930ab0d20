"""Pins of the oracle's many-pairs binary64 CG and truncated series in plain
torch (``oracle/cg_torch.py``), run here on the CPU device.

  * complete graph K_n: beta = 2/n^2; cycle C_n: beta = Dc(Dc+2)/(12n);
    path P_n: the centred unit-current potential (Definition 2.1 closed forms);
  * a random graph: the dense pseudoinverse on every pair;
  * Chung-Lu n=1e5: the stored CPU CG values of tests/golden (scipy route)
    to 1e-10 relative, and the two solves agree;
  * truncated series: the K_n closed form (2/n^2)(1 - (-1/(n-1))^(L+1))^2 and
    the numpy series of ``exact.beta_truncated``.
"""

import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import cg_torch, exact  # noqa: E402
from synth import graphs  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "cl100k_cg_reference.txt")


def test_complete_and_cycle_closed_forms():
    g = graphs.complete_graph(9)
    b1, b2, _, res = cg_torch.beta_cg_many(g, [0, 3, 8], [1, 7, 2], device="cpu")
    assert np.allclose(b1, 2.0 / 81, rtol=1e-12) and np.allclose(b2, 2.0 / 81, rtol=1e-12)
    n = 13
    g = graphs.cycle_graph(n)
    s = [0] * (n - 1)
    t = list(range(1, n))
    b1, b2, _, _ = cg_torch.beta_cg_many(g, s, t, device="cpu", chunk=5)
    D = np.arange(1, n)
    c = n - D
    ref = D * c * (D * c + 2) / (12.0 * n)
    assert np.allclose(b1, ref, rtol=1e-11) and np.allclose(b2, ref, rtol=1e-10)


def test_path_closed_form():
    n = 10
    g = graphs.path_graph(n)
    s, t = [1, 0, 4], [6, 9, 5]
    b1, b2, _, _ = cg_torch.beta_cg_many(g, s, t, device="cpu")
    for j, (a, b) in enumerate(zip(s, t)):
        p, D = a + 1, b - a
        ref = p * D * D + D * (D - 1) * (2 * D - 1) / 6.0 - (p * D + D * (D - 1) / 2.0) ** 2 / n
        assert b1[j] == pytest.approx(ref, rel=1e-10) and b2[j] == pytest.approx(ref, rel=1e-9)


def test_random_graph_vs_dense():
    g = graphs.random_connected(50, 0.1, 8)
    rng = np.random.default_rng(2)
    s = rng.integers(0, 50, 20)
    t = (s + 1 + rng.integers(0, 49, 20)) % 50
    b1, b2, _, _ = cg_torch.beta_cg_many(g, s, t, device="cpu", chunk=7)
    ref = exact.beta_dense_all(g, s, t)
    assert np.allclose(b1, ref, rtol=1e-10) and np.allclose(b2, ref, rtol=1e-9)


def test_cl100k_against_stored_cpu_cg():
    g = graphs.workload_graph("cl100k")
    ref = np.loadtxt(GOLDEN, comments="#")[:16]
    b1, b2, its, res = cg_torch.beta_cg_many(g, ref[:, 1], ref[:, 2], device="cpu", chunk=16)
    assert np.all(res <= 1e-12)
    assert np.allclose(b1, ref[:, 5], rtol=1e-10, atol=0)
    assert np.allclose(b2, ref[:, 5], rtol=1e-10, atol=0)


def test_truncated_series():
    n = 7
    g = graphs.complete_graph(n)
    for L in (0, 1, 4):
        got = cg_torch.beta_truncated_many(g, [0, 2], [5, 3], L, device="cpu")
        ref = (2.0 / n ** 2) * (1.0 - (-1.0 / (n - 1)) ** (L + 1)) ** 2
        assert np.allclose(got, ref, rtol=1e-13)
    g = graphs.barabasi_albert(300, 3, 4)
    s, t = [0, 17, 250], [299, 5, 251]
    got = cg_torch.beta_truncated_many(g, s, t, 30, device="cpu")
    ref = [exact.beta_truncated(g, a, b, 30) for a, b in zip(s, t)]
    assert np.allclose(got, ref, rtol=1e-12)
