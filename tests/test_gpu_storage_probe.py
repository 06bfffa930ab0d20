"""The hubs-first layout with the probe on storage ids (BD_PROBE_STORAGE_IDS,
layout code 5) against the oracle run on the relabelled graph.

The relabelled graph is built with numpy (synth.graphs.storage_order): node i
of it is the caller's node of rank i in descending degree (ties by ascending
id), each row keeps the caller's neighbour order with the ids renamed. On that graph the library's
results must equal the oracle's bit for bit (Algorithm 1: probe values,
walks, per-probe Q, block means, estimates, in every mode, with split probes
and with walk sharing), and its walks, reported in caller ids, are the same
walks as every other layout's. The same holds for its kernels: every node's
row offset and degree in LDS (the degree-run table) in two work groups per CU
with one replica pair per thread (the default where the table fits 64 KB,
and BD_NARROW_HUBS) or in one group per CU with two pairs per thread
(BD_WIDE_HUBS), and the row offsets of the highest-degree nodes instead
(BD_DIRECT_HUBS: 36,864 in one group per CU, 16,384 in two).
"""

import numpy as np
import pytest

from oracle import estimator as E
from oracle import planner as OP
from paper_2512_05460_amd import binding as B
from synth import graphs, queries

pytestmark = pytest.mark.gpu

SEED = graphs.PHILOX_SEED
FLAGS = B.BD_LAYOUT_COMPACT | B.BD_RELABEL_DEGREE | B.BD_PROBE_STORAGE_IDS


def relabelled(g):
    return graphs.storage_order(g)


KERNELS = (0, B.BD_WIDE_HUBS, B.BD_DIRECT_HUBS, B.BD_NARROW_HUBS, B.BD_NARROW_HUBS | B.BD_DIRECT_HUBS)


@pytest.fixture(scope="module", params=[(key, kernel) for kernel in KERNELS for key in ("ba1k", "cl100k")])
def pair(request):
    key, kernel = request.param
    g = graphs.workload_graph(key)
    g5, order, internal = relabelled(g)
    dg = B.graph_load_csr(g.n, g.row_ptr, g.col, FLAGS | kernel)
    info = dg.info()
    assert info["layout"] == 5
    # nodes resolved in LDS: all with the run table, else the staged offsets
    assert info["lds_hubs"] == {0: g.n, B.BD_WIDE_HUBS: g.n, B.BD_DIRECT_HUBS: min(g.n, 36864), B.BD_NARROW_HUBS: g.n,
                                B.BD_NARROW_HUBS | B.BD_DIRECT_HUBS: min(g.n, 16384)}[kernel]
    yield g, g5, order, internal, dg
    dg.free()


def _plans(L, b, r, n):
    return [OP.plan(0.1, int(x), 1, 1, 1, OP.Policy("fixed", B_fixed=b, R_fixed=r)) for x in L] if n else []


@pytest.mark.parametrize("mode", ["plain", "batched"])
def test_estimates_equal_oracle_on_relabelled_graph(pair, mode):
    g, g5, order, internal, dg = pair
    s, t = queries.uniform_pairs(g.n, 12, 5)
    L = np.array([0, 1, 5, 50, 200, 1000] * 2, dtype=np.int32)
    res = B.bd_query_batch(dg, s, t, 0.1, L, SEED, B.policy("fixed", B=2, R=70), B.exec_cfg(mode))
    assert np.all(res["status"] == 0)
    ref = E.estimate(g5, internal[s], internal[t], L, _plans(L, 2, 70, 1), SEED, threads=8)
    assert np.array_equal(res["beta"], ref)


def test_split_probes_and_served(pair):
    g, g5, order, internal, dg = pair
    s, t = queries.uniform_pairs(g.n, 5, 17)
    pol = B.policy("fixed", B=1, R=5000)  # R above the split size
    res = B.bd_query_batch(dg, s, t, 0.1, 20, SEED, pol, B.exec_cfg("batched"))
    ref = E.estimate(g5, internal[s], internal[t], 20, _plans([20] * 5, 1, 5000, 1), SEED, threads=8)
    assert np.array_equal(res["beta"], ref)
    srv = B.Server(dg, pol)
    o, _ = srv.wait(srv.submit(s, t, 0.1, 20, SEED))
    srv.destroy()
    assert np.array_equal(o["beta"], ref)


def test_probe_q_and_block_means(pair):
    g, g5, order, internal, dg = pair
    s, t = queries.uniform_pairs(g.n, 1, 23)
    pol = B.policy("fixed", B=3, R=97)
    r, q, y = B.bd_query_probes(dg, int(s[0]), int(t[0]), 0.1, 77, 4, SEED, pol, B.exec_cfg("batched"))
    plan = OP.plan(0.1, 77, 1, 1, 1, OP.Policy("fixed", B_fixed=3, R_fixed=97))
    rb, rq, ry = E.estimate(g5, [internal[s[0]]], [internal[t[0]]], 77, [plan], SEED, uid=[4], want_q=True)
    assert np.array_equal(q, rq) and np.array_equal(y, ry) and r["beta"] == rb[0]


def test_walks_same_as_other_layouts_and_sums_match_oracle(pair):
    g, g5, order, internal, dg = pair
    starts = queries.uniform_pairs(g.n, 16, 3)[0]
    n = starts.size
    uid, k, p = np.arange(n) % 7, np.arange(n) % 5, np.arange(n) % 3
    side = np.arange(n) % 2
    tr, acc = B.bd_walk_trace(dg, starts, uid, k, p, side, 300, SEED)
    other = B.graph_load_csr(g.n, g.row_ptr, g.col, B.BD_LAYOUT_COMPACT | B.BD_RELABEL_DEGREE)
    tr3, _ = B.bd_walk_trace(other, starts, uid, k, p, side, 300, SEED)
    other.free()
    assert np.array_equal(tr, tr3)  # the same walks in caller ids
    for i in range(n):
        otr, oacc = E.walk_trace(g5, int(internal[starts[i]]), 300, SEED, int(uid[i]), int(k[i]), int(p[i]),
                                 int(side[i]))
        assert np.array_equal(order[otr], tr[i])
        assert np.float32(acc[i]) == np.float32(oacc)


def test_every_node_entry(pair):
    # one short walk from every node: X_1 is read at row offset + floor(u d)
    # of the start and X_2 likewise from X_1, so every node's row offset and
    # degree as the kernel resolves it (the LDS run table by default) is
    # checked against the plain row offsets of layout 3
    g, g5, order, internal, dg = pair
    starts = np.arange(g.n, dtype=np.int32)
    z = np.zeros(g.n, dtype=np.int64)
    tr, acc = B.bd_walk_trace(dg, starts, z + 5, z + 1, np.arange(g.n) % 11, np.arange(g.n) % 2, 2, SEED)
    other = B.graph_load_csr(g.n, g.row_ptr, g.col, B.BD_LAYOUT_COMPACT | B.BD_RELABEL_DEGREE)
    tr3, _ = B.bd_walk_trace(other, starts, z + 5, z + 1, np.arange(g.n) % 11, np.arange(g.n) % 2, 2, SEED)
    other.free()
    assert np.array_equal(tr, tr3)


@pytest.mark.parametrize("M", [2, 4])
def test_walk_sharing(pair, M):
    g, g5, order, internal, dg = pair
    s, t = queries.uniform_pairs(g.n, 6, 29)
    L = np.array([3, 40, 200] * 2, dtype=np.int32)
    pol = B.policy("fixed", B=5, R=90, share=M)
    res = B.bd_query_batch(dg, s, t, 0.1, L, SEED, pol, B.exec_cfg("batched"))
    ref = E.estimate(g5, internal[s], internal[t], L, _plans(L, 5, 90, 1), SEED, threads=8, share=M)
    assert np.array_equal(res["beta"], ref)


@pytest.mark.parametrize("mode", ["plain", "batched"])
def test_bench_shape_sampled_probes(pair, mode):
    # The headline's shape: Chung-Lu n=1e5, eps = 0.05, L = 1000 at its
    # calibrated walk counts; sampled per-probe Q against the oracle on the
    # relabelled graph, for query 0 of the set and the first one whose R
    # exceeds the batched split size (its probes run as replica parts).
    from paper_2512_05460_amd.budgets import budget_policy
    g, g5, order, internal, dg = pair
    if g.name != "cl100k":
        pytest.skip("bench shape is the Chung-Lu n=1e5 graph")
    s, t = queries.uniform_pairs(g.n, 4096, graphs.GRAPH_SEED + 1 + graphs.QUERY_SEED_OFFSET)
    pol = budget_policy("cl100k")
    Rs = B.bd_plan(dg, s[:200], t[:200], 0.05, 1000, pol)["R"]
    split = int(np.flatnonzero((Rs > 4096) & (Rs <= 20000))[0])
    for i in sorted({0, split}):
        plan = B.bd_plan(dg, s[i:i + 1], t[i:i + 1], [0.05], [1000], pol)[0]
        res, q, y = B.bd_query_probes(dg, int(s[i]), int(t[i]), 0.05, 1000, i, SEED, pol, B.exec_cfg(mode))
        ks = np.linspace(0, plan["K"] - 1, 8).astype(np.uint32)
        oq = E.probe_q(g5, int(internal[s[i]]), int(internal[t[i]]), 1000, i, int(plan["R"]), SEED, ks, threads=8)
        assert np.array_equal(q[ks], oq), (i, int(plan["R"]))


def test_run_table_with_large_blocks():
    # The grid (2e6 nodes, degrees 1-4) needs blocks of 256 storage ids for its
    # run table to fit two work groups per CU (128 for one): every node's entry
    # through one-step walks against layout 3, and estimates equal to the
    # per-node-offset kernel's, in both
    g = graphs.workload_graph("grid1414")
    dg = B.graph_load_csr(g.n, g.row_ptr, g.col, FLAGS)
    wide = B.graph_load_csr(g.n, g.row_ptr, g.col, FLAGS | B.BD_WIDE_HUBS)
    direct = B.graph_load_csr(g.n, g.row_ptr, g.col, FLAGS | B.BD_DIRECT_HUBS)
    other = B.graph_load_csr(g.n, g.row_ptr, g.col, B.BD_LAYOUT_COMPACT | B.BD_RELABEL_DEGREE)
    try:
        assert dg.info()["lds_hubs"] == g.n and wide.info()["lds_hubs"] == g.n
        assert direct.info()["lds_hubs"] == 36864
        starts = np.arange(0, g.n, 3, dtype=np.int32)
        z = np.zeros(starts.size, dtype=np.int64)
        side = np.arange(starts.size) % 2
        tr3, _ = B.bd_walk_trace(other, starts, z + 2, z, np.arange(starts.size) % 5, side, 2, SEED)
        for h in (dg, wide):
            tr, _ = B.bd_walk_trace(h, starts, z + 2, z, np.arange(starts.size) % 5, side, 2, SEED)
            assert np.array_equal(tr, tr3)
        s, t = queries.uniform_pairs(g.n, 16, 41)
        L = np.array([10, 300, 2000, 5000] * 4, dtype=np.int32)
        pol = B.policy("fixed", B=2, R=100)
        for mode in ("plain", "batched"):
            b = B.bd_query_batch(direct, s, t, 0.1, L, SEED, pol, B.exec_cfg(mode))
            for h in (dg, wide):
                a = B.bd_query_batch(h, s, t, 0.1, L, SEED, pol, B.exec_cfg(mode))
                assert np.array_equal(a["beta"], b["beta"]), mode
    finally:
        other.free()
        direct.free()
        wide.free()
        dg.free()


def test_run_table_with_short_last_run():
    # A full 2,200 x 2,200 grid (4.8e6 nodes): degree 4 inside, 3 on the
    # border and 2 at the four corners, whose run of 4 storage ids comes last.
    # Its table needs blocks of 512 storage ids and a block that ends in that
    # short run; every node entry against layout 3, corners included, and
    # estimates against the per-node-offset kernel
    side = 2200
    g = graphs.grid_minus_edges(side, 0.0, 5)
    dg = B.graph_load_csr(g.n, g.row_ptr, g.col, FLAGS)
    direct = B.graph_load_csr(g.n, g.row_ptr, g.col, FLAGS | B.BD_DIRECT_HUBS)
    other = B.graph_load_csr(g.n, g.row_ptr, g.col, B.BD_LAYOUT_COMPACT | B.BD_RELABEL_DEGREE)
    try:
        assert dg.info()["lds_hubs"] == g.n
        corners = np.array([0, side - 1, g.n - side, g.n - 1])
        near = np.array([1, side - 2, g.n - side + 1, g.n - 2])
        starts = np.concatenate([np.arange(0, g.n, 7), corners, near]).astype(np.int32)
        z = np.zeros(starts.size, dtype=np.int64)
        side_bit = np.arange(starts.size) % 2
        tr, _ = B.bd_walk_trace(dg, starts, z + 3, z, np.arange(starts.size) % 5, side_bit, 2, SEED)
        tr3, _ = B.bd_walk_trace(other, starts, z + 3, z, np.arange(starts.size) % 5, side_bit, 2, SEED)
        assert np.array_equal(tr, tr3)
        s = np.concatenate([corners, queries.uniform_pairs(g.n, 8, 43)[0]])
        t = np.concatenate([corners[::-1], queries.uniform_pairs(g.n, 8, 43)[1]])
        L = np.array([4, 50, 400, 3000] * 3, dtype=np.int32)
        pol = B.policy("fixed", B=2, R=80)
        for mode in ("plain", "batched"):
            a = B.bd_query_batch(dg, s, t, 0.1, L, SEED, pol, B.exec_cfg(mode))
            b = B.bd_query_batch(direct, s, t, 0.1, L, SEED, pol, B.exec_cfg(mode))
            assert np.all(a["status"] == 0) and np.array_equal(a["beta"], b["beta"]), mode
    finally:
        other.free()
        direct.free()
        dg.free()


@pytest.mark.parametrize("kernel", [0, B.BD_DIRECT_HUBS])
@pytest.mark.parametrize("make", [lambda: graphs.complete_graph(5), lambda: graphs.path_graph(2),
                                  lambda: graphs.cycle_graph(6), lambda: graphs.random_connected(37, 0.1, 4)],
                         ids=["K5", "P2", "C6", "G37"])
def test_tiny_graphs(make, kernel):
    # graphs of one or a few runs, fewer nodes than a block: estimates in both
    # modes against the oracle on the graph in storage order, walks against
    # layout 3
    g = make()
    gs, order, internal = relabelled(g)
    dg = B.graph_load_csr(g.n, g.row_ptr, g.col, FLAGS | kernel)
    try:
        assert dg.info()["lds_hubs"] == (g.n if kernel == 0 else min(g.n, 36864))
        s = np.array([0, 1, g.n - 1, 1], dtype=np.int32)
        t = np.array([1, g.n - 1, 0, 0], dtype=np.int32)
        keep = s != t
        s, t = s[keep], t[keep]
        L = np.array([0, 3, 40, 200][:s.size], dtype=np.int32)
        pol = B.policy("fixed", B=2, R=70)
        ref = E.estimate(gs, internal[s], internal[t], L, _plans(L, 2, 70, 1), SEED, threads=4)
        for mode in ("plain", "batched"):
            res = B.bd_query_batch(dg, s, t, 0.1, L, SEED, pol, B.exec_cfg(mode))
            assert np.all(res["status"] == 0) and np.array_equal(res["beta"], ref), mode
        starts = np.arange(g.n, dtype=np.int32)
        z = np.zeros(g.n, dtype=np.int64)
        tr, _ = B.bd_walk_trace(dg, starts, z + 1, z + 2, z, np.arange(g.n) % 2, 30, SEED)
        other = B.graph_load_csr(g.n, g.row_ptr, g.col, B.BD_LAYOUT_COMPACT | B.BD_RELABEL_DEGREE)
        tr3, _ = B.bd_walk_trace(other, starts, z + 1, z + 2, z, np.arange(g.n) % 2, 30, SEED)
        other.free()
        assert np.array_equal(tr, tr3)
    finally:
        dg.free()
