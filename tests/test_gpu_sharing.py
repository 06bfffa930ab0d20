"""Walk sharing on the GPU against the oracle, bit for bit.

The probes of each median-of-means block are scored in groups of M on common
walks (an extension of Algorithm 1; M = 1 is the algorithm itself). Checked:
per-probe Q_k, block means and beta-hat in every layout and execution mode
(plain, batched, replica-split groups, served), block sizes that M does not
divide, the walk-step count, and the range check on M.
"""

import sys

import numpy as np
import pytest

from oracle import estimator as E
from oracle import planner as OP
from paper_2512_05460_amd import binding as B
from synth import graphs, queries

pytestmark = pytest.mark.gpu

SEED = graphs.PHILOX_SEED
LAYOUTS = [B.BD_LAYOUT_COMPACT, B.BD_LAYOUT_CSR | B.BD_RELABEL_DEGREE, B.BD_LAYOUT_FAT,
           B.BD_LAYOUT_COMPACT | B.BD_RELABEL_DEGREE, B.BD_LAYOUT_COMPACT | B.BD_RELABEL_DEGREE | B.BD_WIDE_IDS]

_cache = {}


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _graph(key, flags):
    if (key, flags) not in _cache:
        g = graphs.workload_graph(key)
        _cache[(key, flags)] = (g, B.graph_load_csr(g.n, g.row_ptr, g.col, flags))
    return _cache[(key, flags)]


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("M", [2, 3, 4])
def test_probe_q_and_blocks(layout, M):
    g, dg = _graph("ba1k", layout)
    s, t, L, uid = 17, 640, 40, 5
    Bb, R = 7, 60                      # B not a multiple of M; R >= 48: wave-uniform kernel
    pol = B.policy("fixed", B=Bb, R=R, share=M)
    plan = (Bb, 37, Bb * 37, R)
    ob, oq, oy = E.estimate(g, [s], [t], L, [plan], SEED, uid=[uid], want_q=True, share=M)
    for ex in (B.exec_cfg("plain"), B.exec_cfg("batched"), B.exec_cfg("batched", uniform_min_r=-1),
               B.exec_cfg("batched", uniform_min_r=48)):
        res, q, y = B.bd_query_probes(dg, s, t, 0.1, L, uid, SEED, pol, ex)
        assert np.array_equal(q, oq), ex.as_dict()
        assert np.array_equal(y, oy) and res["beta"] == ob[0]
        assert res["walk_steps"] == OP.walk_steps(Bb, 37, R, L, M)


@pytest.mark.parametrize("M", [2, 4])
def test_split_groups(M):
    # R = 5000 > 4096: batched and served launches cut each group's replicas
    g, dg = _graph("ba1k", B.BD_LAYOUT_COMPACT)
    s, t, L = 10, 900, 5
    pol = B.policy("fixed", B=3, R=5000, share=M)
    plan = (3, 37, 111, 5000)
    ob, oq, _ = E.estimate(g, [s], [t], L, [plan], SEED, uid=[3], want_q=True, share=M, threads=1)
    for ex in (B.exec_cfg("batched"), B.exec_cfg("batched", chunk_pairs=1500),
               B.exec_cfg("batched", uniform_min_r=-1, chunk_pairs=2000)):
        res, q, _ = B.bd_query_probes(dg, s, t, 0.1, L, 3, SEED, pol, ex)
        assert np.array_equal(q, oq), ex.as_dict()
        assert res["beta"] == ob[0]


@pytest.mark.parametrize("layout", [B.BD_LAYOUT_COMPACT, B.BD_LAYOUT_CSR])
def test_batch_and_server(layout):
    g, dg = _graph("ba1k", layout)
    n = 12
    s, t = queries.uniform_pairs(g.n, n, 91)
    eps, L = queries.mixed_eps_L(n, [0.3, 0.5], [0, 1, 9, 70], 92)
    M = 3
    pol = B.policy("scaled", c_B=0.05, c_R=0.002, share=M)
    opol = OP.Policy("scaled", c_B=0.05, c_R=0.002)
    d = g.deg
    plans = [OP.plan(eps[i], int(L[i]), d[s[i]], d[t[i]], g.d_min, opol) for i in range(n)]
    _say("R", [p[3] for p in plans])
    ref = E.estimate(g, s, t, L, plans, SEED, threads=8, share=M)
    for ex in (B.exec_cfg("plain"), B.exec_cfg("batched"), B.exec_cfg("batched", chunk_probes=5, grid_wgs=3),
               B.exec_cfg("batched", use_graph=True)):
        res = B.bd_query_batch(dg, s, t, eps, L, SEED, pol, ex)
        assert np.all(res["status"] == 0)
        assert np.array_equal(res["beta"], ref), ex.as_dict()
    srv = B.Server(dg, pol)
    try:
        rids = [srv.submit(s[i::2], t[i::2], eps[i::2], L[i::2], SEED, uid=np.arange(n)[i::2]) for i in range(2)]
        for i, rid in enumerate(rids):
            out, _ = srv.wait(rid)
            assert np.array_equal(out["beta"], ref[i::2])
    finally:
        srv.destroy()


def test_share_range():
    g, dg = _graph("ba1k", B.BD_LAYOUT_COMPACT)
    for M, ok in ((0, True), (1, True), (4, True), (5, False), (-1, False)):
        res = B.bd_query_batch(dg, [1], [2], 0.3, 5, SEED, B.policy("fixed", B=2, R=4, share=M))
        assert (res["status"][0] == 0) == ok, M
    # M = 0 and M = 1 are Algorithm 1
    a = B.bd_query_batch(dg, [1, 5], [2, 9], 0.3, 5, SEED, B.policy("fixed", B=5, R=4, share=0))
    b = B.bd_query_batch(dg, [1, 5], [2, 9], 0.3, 5, SEED, B.policy("fixed", B=5, R=4))
    assert np.array_equal(a["beta"], b["beta"])
