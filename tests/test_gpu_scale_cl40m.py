"""The scale workload at full size: Chung-Lu n=4*10^7 (mean degree 25,
exponent 2.2, largest component: 39,944,860 nodes, 996,486,866 adjacency
entries) in the compact layout with hubs first, which above 2^24 nodes keeps
4-byte neighbour ids, and in the layout the library picks (fat: 16-byte
adjacency entries, 16 GB at this size).

Queries of the workload's set (eps = 0.05, L in {1000, 10000}) in one
persistent launch and through the server; sampled queries are checked bit for
bit against the oracle, and the served results against the batched ones.
Walk counts: the throughput setting of paper_2512_05460_amd/budgets.py.
"""

import sys

import numpy as np
import pytest

from oracle import estimator as E
from oracle import planner as OP
from paper_2512_05460_amd import binding as B
from paper_2512_05460_amd.budgets import BUDGETS, budget_policy
from synth import graphs, queries

pytestmark = pytest.mark.gpu

SEED = graphs.PHILOX_SEED


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def cl40m():
    _say("[cl40m] building the graph (native generator)")
    g = graphs.workload_graph("cl40m")
    _say(f"[cl40m] n={g.n} nnz={g.nnz}; loading (hubs first)")
    dg = B.graph_load_csr(g.n, g.row_ptr, g.col, B.BD_LAYOUT_COMPACT | B.BD_RELABEL_DEGREE)
    _say("[cl40m] loaded")
    yield g, dg
    dg.free()


@pytest.mark.timeout(900)
def test_cl40m_resident(cl40m):
    g, dg = cl40m
    info = dg.info()
    assert info["n"] == g.n and info["nnz"] == g.nnz and info["d_min"] == 1 and info["layout"] == 4
    assert g.nnz > 9.9e8
    # 8-byte node entries, 4-byte neighbour ids, 4-byte row offsets
    assert 12 * g.n + 4 * g.nnz <= info["device_bytes"] <= 12 * g.n + 4 * g.nnz + (64 << 20)
    _say(f"[cl40m] device bytes {info['device_bytes']:,}")


@pytest.mark.timeout(900)
def test_cl40m_batched_and_served_sampled_parity(cl40m):
    g, dg = cl40m
    n = 4096
    s, t, eps, L = queries.workload_batch("cl40m", g.n, n)
    pol = budget_policy("cl40m")
    res, st = B.bd_query_batch(dg, s, t, eps, L, SEED, pol, B.exec_cfg("batched"), with_stats=True)
    assert np.all(res["status"] == 0)
    _say(f"[cl40m] {n} queries: {st['walk_steps']:.3e} steps in {st['walk_kernel_ms']:.0f} ms")
    c_B, c_R, _ = BUDGETS["cl40m"]
    op = OP.Policy("scaled", c_B=c_B, c_R=c_R)
    d, dmin = g.deg, g.d_min
    plans = [OP.plan(float(eps[i]), int(L[i]), int(d[s[i]]), int(d[t[i]]), dmin, op) for i in range(n)]
    assert [(int(r["K"]), int(r["R"])) for r in res] == [(p[2], p[3]) for p in plans]
    W = np.array([2 * p[2] * p[3] * int(L[i]) for i, p in enumerate(plans)])
    pick = [i for i in range(n) if W[i] <= 2e8 and L[i] == 10000][:6] + \
           [i for i in range(n) if W[i] <= 2e8 and L[i] == 1000][:6]
    ref = E.estimate(g, s[pick], t[pick], L[pick], [plans[i] for i in pick], SEED,
                     uid=np.array(pick, dtype=np.uint32), threads=12)
    assert np.array_equal(res["beta"][pick], ref)
    # served: the first 256 queries as four requests submitted together
    srv = B.Server(dg, pol)
    try:
        rids = [srv.submit(s[j:j + 64], t[j:j + 64], eps[j:j + 64], L[j:j + 64], SEED,
                           uid=np.arange(j, j + 64)) for j in range(0, 256, 64)]
        for k, rid in enumerate(rids):
            out, _ = srv.wait(rid)
            assert np.array_equal(out["beta"], res["beta"][64 * k:64 * k + 64])
    finally:
        srv.destroy()


@pytest.mark.timeout(900)
def test_cl40m_fat_equals_hubs_first(cl40m):
    g, dg = cl40m
    n = 4096
    s, t, eps, L = queries.workload_batch("cl40m", g.n, n)
    pol = budget_policy("cl40m")
    ref = B.bd_query_batch(dg, s, t, eps, L, SEED, pol, B.exec_cfg("batched"))
    _say("[cl40m] loading the automatic layout")
    fat = B.graph_load_csr(g.n, g.row_ptr, g.col, B.BD_LAYOUT_AUTO | B.BD_SKIP_VALIDATION)
    try:
        info = fat.info()
        assert info["layout"] == 1
        assert info["nontemporal"] == 1  # 20.7 GB of fat tables: above the 4 GiB threshold
        assert 16 * g.n + 20 * g.nnz <= info["device_bytes"] <= 20 * g.n + 20 * g.nnz + (64 << 20)
        res = B.bd_query_batch(fat, s, t, eps, L, SEED, pol, B.exec_cfg("batched"))
        assert np.array_equal(res["beta"], ref["beta"])
        srv = B.Server(fat, pol)
        try:
            rid = srv.submit(s[:512], t[:512], eps[:512], L[:512], SEED)
            out, _ = srv.wait(rid)
            assert np.array_equal(out["beta"], ref["beta"][:512])
        finally:
            srv.destroy()
    finally:
        fat.free()
