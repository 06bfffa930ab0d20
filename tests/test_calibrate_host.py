"""Host logic of the walk-count calibration (paper_2512_05460_amd/calibrate.py):
the estimate for a smaller B formed from the per-probe values of a run at a
larger B equals the oracle's own estimate at that smaller B, bit for bit
(Q_k depends on k and R, not on B), for odd and even G."""

import numpy as np
import pytest

from oracle import estimator as E
from oracle import planner as OP
from paper_2512_05460_amd.calibrate import median_of_means
from synth import graphs


@pytest.mark.parametrize("delta", [0.01, 0.3])  # G = 37 (odd) and G = 10 (even)
def test_smaller_B_from_larger_run(delta):
    g = graphs.barabasi_albert(200, 3, 11)
    s, t, L, seed = 3, 150, 12, 0x77
    big = OP.Policy("fixed", B_fixed=12, R_fixed=20, delta=delta)
    plan = OP.plan(0.1, L, 1, 1, 1, big)
    beta, q, y = E.estimate(g, [s], [t], L, [plan], seed, uid=[5], want_q=True)
    G = plan[1]
    assert median_of_means(q, 12, G) == beta[0]
    for b in (1, 2, 5, 7):
        small = OP.plan(0.1, L, 1, 1, 1, OP.Policy("fixed", B_fixed=b, R_fixed=20, delta=delta))
        ref = E.estimate(g, [s], [t], L, [small], seed, uid=[5])[0]
        assert median_of_means(q, b, G) == ref


def test_reference_columns_by_name():
    import os

    from paper_2512_05460_amd.calibrate import load_reference
    here = os.path.join(os.path.dirname(__file__), "golden")
    for key in ("cl10m", "cl40m", "cl100k"):
        ref = load_reference(os.path.join(here, f"{key}_cg_reference.txt"))
        assert np.array_equal(ref["index"], np.arange(ref["index"].size))
        assert np.all(ref["s"] != ref["t"]) and np.all(ref["d_s"] >= 1)
        assert np.all((ref["beta_cg"] > 0) & (ref["beta_cg"] < 10))
        assert np.allclose(ref["beta_2nd"], ref["beta_cg"], rtol=1e-10)
        # Lemma 3.5: beta >= (1/8)(1/d_s + 1/d_t)^2
        assert np.all(ref["beta_cg"] >= (1.0 / ref["d_s"] + 1.0 / ref["d_t"]) ** 2 / 8)
    ref = load_reference(os.path.join(here, "cl40m_cg_reference.txt"))
    assert set(np.unique(ref["L"])) == {1000.0, 10000.0}


def test_select_pairs():
    from paper_2512_05460_amd.calibrate import load_reference, select_pairs
    import os
    ref = load_reference(os.path.join(os.path.dirname(__file__), "golden", "cl40m_cg_reference.txt"))
    all10 = np.flatnonzero(ref["L"] == 10000)
    assert all10.size == 31 and np.all(np.diff(all10) > 0)
    assert np.array_equal(select_pairs(ref, 10000), all10)
    assert np.array_equal(select_pairs(ref, 10000, 0, 16), all10[:16])
    assert np.array_equal(select_pairs(ref, 10000, 16), all10[16:])
    assert np.array_equal(select_pairs(ref, 0, 0, 8), np.arange(8))
    assert np.array_equal(np.sort(np.concatenate([select_pairs(ref, 1000), all10])), np.arange(ref["index"].size))
