"""GPU parity: the HIP path against the CPU oracle, through the C ABI.

Bit-exact: probe values pi_k and z^(k), walk trajectories, per-walk binary32
sums, per-probe Q_k, block means and beta-hat (all sums are exact fixed point,
so no tolerance applies). Also: the planner, every execution mode and both
adjacency layouts, chunk sizes, uid handling, invalid queries, and the edge
cases L = 0, n = 2, odd/even n, degree-1 endpoints, the maximum L.
"""

import sys

import numpy as np
import pytest

from oracle import estimator as E
from oracle import planner as OP
from paper_2512_05460_amd import binding as B
from synth import graphs, queries

pytestmark = pytest.mark.gpu

SEED = 0x0B1A5ED5EED


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


_graph_cache = {}


def load(g, layout):
    key = (g.name, g.n, g.nnz, layout)
    if key not in _graph_cache:
        _say(f"[load] {g.name} n={g.n} nnz={g.nnz} layout={layout}")
        _graph_cache[key] = B.graph_load_csr(g.n, g.row_ptr, g.col, layout)
    return _graph_cache[key]


SMALL = {
    "K5": lambda: graphs.complete_graph(5),
    "C6": lambda: graphs.cycle_graph(6),
    "P2": lambda: graphs.path_graph(2),
    "G37": lambda: graphs.random_connected(37, 0.1, 4),
}


@pytest.fixture(scope="module")
def ba1k():
    return graphs.workload_graph("ba1k")


@pytest.fixture(scope="module")
def cl100k():
    return graphs.workload_graph("cl100k")


def test_device_info():
    info = B.bd_device_info()
    _say(info)
    assert "gfx950" in info


@pytest.mark.parametrize("layout,code", [(B.BD_LAYOUT_CSR, 0), (B.BD_LAYOUT_FAT, 1),
                                         (B.BD_LAYOUT_FAT | B.BD_RELABEL_DEGREE, 1), (B.BD_LAYOUT_COMPACT, 2),
                                         (B.BD_LAYOUT_COMPACT | B.BD_RELABEL_DEGREE, 3),
                                         (B.BD_LAYOUT_COMPACT | B.BD_RELABEL_DEGREE | B.BD_WIDE_IDS, 4),
                                         (B.BD_LAYOUT_FAT | B.BD_NONTEMPORAL, 1),
                                         (B.BD_LAYOUT_FAT | B.BD_RELABEL_DEGREE | B.BD_TEMPORAL, 1)])
def test_graph_info(ba1k, layout, code):
    gi = load(ba1k, layout).info()
    assert gi["n"] == ba1k.n and gi["nnz"] == ba1k.nnz
    assert gi["d_min"] == ba1k.d_min and gi["d_max"] == ba1k.d_max
    assert gi["layout"] == code and gi["bipartite"] == 0
    assert gi["nontemporal"] == (1 if layout & B.BD_NONTEMPORAL else 0)  # small fat tables: ordinary loads


def test_auto_layout(ba1k):
    # hubs-first compact tables within 12 MiB, else the fat layout
    assert load(ba1k, B.BD_LAYOUT_AUTO).info()["layout"] == 3
    assert load(graphs.workload_graph("cl100k"), B.BD_LAYOUT_AUTO).info()["layout"] == 3
    grid = graphs.workload_graph("grid1414")
    for flags in (B.BD_LAYOUT_AUTO, B.BD_LAYOUT_AUTO | B.BD_RELABEL_DEGREE):
        gi = load(grid, flags | B.BD_SKIP_VALIDATION).info()
        assert gi["layout"] == 1 and gi["device_bytes"] >= 16 * grid.nnz


def test_bipartite_flag():
    gi = load(graphs.cycle_graph(6), B.BD_LAYOUT_CSR).info()
    assert gi["bipartite"] == 1
    gi = load(graphs.complete_graph(5), B.BD_LAYOUT_CSR).info()
    assert gi["bipartite"] == 0


@pytest.mark.parametrize("name", list(SMALL) + ["ba1k", "cl100k"])
def test_probe_parity(name):
    g = SMALL[name]() if name in SMALL else graphs.workload_graph(name)
    dg = load(g, B.BD_LAYOUT_CSR | B.BD_RELABEL_DEGREE)
    nodes = np.arange(g.n, dtype=np.uint32)
    for uid, k in [(0, 0), (3, 1), (7, 12345), (2 ** 31 - 1, 2 ** 32 - 2)]:
        pi, z = B.bd_probe_eval(dg, SEED, uid, k, nodes)
        opi, oz, _ = E.probe(g.n, SEED, uid, k, nodes)
        assert np.array_equal(pi, opi), (name, uid, k)
        assert np.array_equal(z, oz), (name, uid, k)


LAYOUTS = [B.BD_LAYOUT_CSR, B.BD_LAYOUT_FAT, B.BD_LAYOUT_CSR | B.BD_RELABEL_DEGREE,
           B.BD_LAYOUT_FAT | B.BD_RELABEL_DEGREE, B.BD_LAYOUT_COMPACT, B.BD_LAYOUT_COMPACT | B.BD_RELABEL_DEGREE,
           B.BD_LAYOUT_COMPACT | B.BD_RELABEL_DEGREE | B.BD_WIDE_IDS,
           B.BD_LAYOUT_FAT | B.BD_RELABEL_DEGREE | B.BD_NONTEMPORAL]


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("name", ["ba1k", "cl100k", "K5", "P2", "G37"])
@pytest.mark.parametrize("L", [0, 1, 2, 3, 4, 5, 37, 1000])
def test_trace_parity(name, layout, L):
    g = SMALL[name]() if name in SMALL else graphs.workload_graph(name)
    dg = load(g, layout)
    rng = np.random.default_rng(L * 7 + layout)
    n = 24
    start = rng.integers(0, g.n, n).astype(np.int32)
    start[0] = int(np.argmax(g.deg))  # a hub
    start[1] = int(np.argmin(g.deg))  # a minimum-degree node
    uid = rng.integers(0, 2 ** 31, n).astype(np.uint32)
    k = rng.integers(0, 2 ** 32 - 1, n).astype(np.uint32)
    p = rng.integers(0, 2 ** 32 - 1, n).astype(np.uint32)
    side = rng.integers(0, 2, n).astype(np.uint32)
    tr, acc = B.bd_walk_trace(dg, start, uid, k, p, side, L, SEED)
    for i in range(n):
        otr, oacc = E.walk_trace(g, int(start[i]), L, SEED, int(uid[i]), int(k[i]), int(p[i]), int(side[i]))
        assert np.array_equal(tr[i], otr), (name, L, i)
        assert np.float32(acc[i]) == np.float32(oacc), (name, L, i, acc[i], oacc)


def test_trace_max_L():
    g = graphs.random_connected(37, 0.1, 4)
    dg = load(g, B.BD_LAYOUT_FAT)
    tr, acc = B.bd_walk_trace(dg, [5], [1], [2], [3], [1], 16383, SEED)
    otr, oacc = E.walk_trace(g, 5, 16383, SEED, 1, 2, 3, 1)
    assert np.array_equal(tr[0], otr) and np.float32(acc[0]) == np.float32(oacc)
    with pytest.raises(B.ProbeWalkError):
        B.bd_walk_trace(dg, [5], [1], [2], [3], [1], 16384, SEED)


def _oracle_probes(g, s, t, L, uid, plan):
    beta, q, y = E.estimate(g, [s], [t], L, [plan], SEED, uid=[uid], want_q=True)
    return beta[0], q, y


PROBE_CASES = [
    # graph, s, t, L, B, R, layout, chunk_probes
    ("K5", 1, 3, 3, 2, 2, B.BD_LAYOUT_CSR, 0),
    ("C6", 0, 3, 7, 1, 257, B.BD_LAYOUT_CSR, 0),
    ("P2", 0, 1, 5, 2, 3, B.BD_LAYOUT_FAT, 0),
    ("G37", 2, 30, 0, 2, 5, B.BD_LAYOUT_CSR, 3),
    ("G37", 2, 30, 40, 3, 100, B.BD_LAYOUT_FAT, 7),
    ("ba1k", 10, 900, 200, 3, 300, B.BD_LAYOUT_CSR, 0),
    ("ba1k", 10, 900, 200, 3, 300, B.BD_LAYOUT_FAT, 2),
    ("cl100k", 5, 77, 1000, 1, 70, B.BD_LAYOUT_CSR, 0),
    ("cl100k", 5, 77, 1000, 1, 70, B.BD_LAYOUT_FAT, 0),
    ("cl100k", 5, 77, 1000, 1, 70, B.BD_LAYOUT_CSR | B.BD_RELABEL_DEGREE, 0),
    ("G37", 2, 30, 40, 3, 100, B.BD_LAYOUT_FAT | B.BD_RELABEL_DEGREE, 7),
    ("G37", 2, 30, 40, 3, 100, B.BD_LAYOUT_COMPACT, 7),
    ("ba1k", 10, 900, 200, 3, 300, B.BD_LAYOUT_COMPACT, 0),
    ("cl100k", 5, 77, 1000, 1, 70, B.BD_LAYOUT_COMPACT, 0),
    ("P2", 0, 1, 5, 2, 3, B.BD_LAYOUT_COMPACT, 0),
    # hubs first: 1,024-thread work groups with 8,192 staged node entries; on
    # cl100k steps go to staged and unstaged nodes, on ba1k every node is staged;
    # R = 40 runs the general kernel, R = 70 and 300 the wave-uniform one
    ("cl100k", 5, 77, 1000, 1, 70, B.BD_LAYOUT_COMPACT | B.BD_RELABEL_DEGREE, 0),
    ("cl100k", 5, 77, 1000, 2, 40, B.BD_LAYOUT_COMPACT | B.BD_RELABEL_DEGREE, 0),
    ("cl100k", 5, 77, 1000, 1, 70, B.BD_LAYOUT_COMPACT | B.BD_RELABEL_DEGREE | B.BD_WIDE_IDS, 0),
    ("ba1k", 10, 900, 200, 3, 300, B.BD_LAYOUT_COMPACT | B.BD_RELABEL_DEGREE, 0),
    ("G37", 2, 30, 40, 3, 100, B.BD_LAYOUT_COMPACT | B.BD_RELABEL_DEGREE, 7),
]


@pytest.mark.parametrize("case", PROBE_CASES, ids=[f"{c[0]}-L{c[3]}-R{c[5]}-lay{c[6]}-kc{c[7]}" for c in PROBE_CASES])
@pytest.mark.parametrize("mode", ["plain", "batched"])
def test_query_probe_parity(case, mode):
    name, s, t, L, Bf, Rf, layout, kc = case
    g = SMALL[name]() if name in SMALL else graphs.workload_graph(name)
    dg = load(g, layout)
    pol = B.policy("fixed", B=Bf, R=Rf)
    uid = 17
    res, q, y = B.bd_query_probes(dg, s, t, 0.1, L, uid, SEED, pol, B.exec_cfg(mode, chunk_probes=kc))
    assert res["status"] == 0
    plan = OP.plan(0.1, L, 1, 1, 1, OP.Policy("fixed", B_fixed=Bf, R_fixed=Rf))
    assert (res["B"], res["G"], res["K"], res["R"]) == plan
    ob, oq, oy = _oracle_probes(g, s, t, L, uid, plan)
    assert np.array_equal(q, oq), np.abs(q - oq).max()
    assert np.array_equal(y, oy)
    assert res["beta"] == ob


def test_planner_parity(cl100k):
    dg = load(cl100k, B.BD_LAYOUT_CSR)
    s, t = queries.uniform_pairs(cl100k.n, 400, 99)
    eps, L = queries.mixed_eps_L(400, [0.01, 0.02, 0.05, 0.06, 0.1, 0.3], [0, 1, 200, 1000, 5000], 5)
    pols = [(B.policy("paper"), OP.PAPER),
            (B.policy("scaled", c_B=0.3, c_R=1e-4), OP.Policy("scaled", c_B=0.3, c_R=1e-4)),
            (B.policy("scaled", c_B=1.7, c_R=3e-3, delta=0.05), OP.Policy("scaled", c_B=1.7, c_R=3e-3, delta=0.05))]
    for bp, op in pols:
        res = B.bd_plan(dg, s, t, eps, L, bp)
        for i in range(400):
            d = cl100k.deg
            ref = OP.plan(eps[i], int(L[i]), d[s[i]], d[t[i]], cl100k.d_min, op)
            got = (res["B"][i], res["G"][i], res["K"][i], res["R"][i])
            if ref[2] < 2 ** 32 - 1 and ref[3] < 2 ** 32 - 1:
                assert got == ref, (i, got, ref)
                assert res["status"][i] == 0
                assert res["walk_steps"][i] == min(2 * ref[2] * ref[3] * int(L[i]), 2 ** 63 - 1)
            else:
                assert res["status"][i] == B.BD_E_BUDGET


def test_budget_cap_and_invalid_queries(ba1k):
    dg = load(ba1k, B.BD_LAYOUT_CSR)
    s = [1, 3, 3, -1, 5, 6, 7, 2000]
    t = [2, 3, 4, 5, 6, 7, 8, 9]
    eps = [0.1, 0.1, 0.0, 0.1, 1.0, 0.1, 0.1, 0.1]
    L = [10, 10, 10, 10, 10, -1, 20000, 10]
    pol = B.policy("fixed", B=1, R=4, max_steps=2 * 37 * 4 * 10)
    res = B.bd_query_batch(dg, s, t, eps, L, SEED, pol)
    assert res["status"].tolist() == [0] + [B.BD_E_INVALID] * 7
    res = B.bd_query_batch(dg, [1, 1], [2, 2], [0.1, 0.1], [10, 11], SEED, pol)
    assert res["status"].tolist() == [0, B.BD_E_BUDGET]


def test_empty_and_all_invalid_batches(ba1k):
    dg = load(ba1k, B.BD_LAYOUT_COMPACT)
    pol = B.policy("fixed", B=1, R=2)
    e = np.zeros(0, dtype=np.int32)
    for ex in (B.exec_cfg("plain"), B.exec_cfg("batched"), B.exec_cfg("batched", use_graph=True)):
        assert B.bd_query_batch(dg, e, e, 0.1, 5, SEED, pol, ex).size == 0
        bad = B.bd_query_batch(dg, [1, 4], [1, 4], 0.1, 5, SEED, pol, ex)   # s == t only
        assert bad["status"].tolist() == [B.BD_E_INVALID] * 2 and np.all(bad["beta"] == 0)
    assert B.bd_truncated_beta(dg, e, e, 10).size == 0
    srv = B.Server(dg, pol)
    try:
        out, _ = srv.wait(srv.submit(e, e, 0.1, 5, SEED))
        assert out.size == 0
        out, _ = srv.wait(srv.submit([3], [3], 0.1, 5, SEED))
        assert out["status"].tolist() == [B.BD_E_INVALID]
    finally:
        srv.destroy()
    # the smallest walk counts (K = 37, R = 2) at L = 0 and L = 1 against the oracle
    for L in (0, 1):
        r = B.bd_query_batch(dg, [5], [600], 0.1, L, SEED, pol, B.exec_cfg("batched"))
        ref = E.estimate(ba1k, [5], [600], L, [(1, 37, 37, 2)], SEED, uid=[0])
        assert r["beta"][0] == ref[0]


def _mixed_batch(g, n, seed):
    s, t = queries.uniform_pairs(g.n, n, seed)
    eps, L = queries.mixed_eps_L(n, [0.3, 0.5, 0.7], [0, 1, 7, 60, 200], seed + 1)
    return s, t, eps, L


@pytest.mark.parametrize("layout", LAYOUTS)
def test_batch_parity_all_modes(ba1k, layout):
    dg = load(ba1k, layout)
    s, t, eps, L = _mixed_batch(ba1k, 10, 3)
    pol = B.policy("scaled", c_B=0.05, c_R=2e-4)
    opol = OP.Policy("scaled", c_B=0.05, c_R=2e-4)
    d = ba1k.deg
    plans = [OP.plan(eps[i], int(L[i]), d[s[i]], d[t[i]], ba1k.d_min, opol) for i in range(10)]
    uid = np.arange(100, 110, dtype=np.uint32)
    ref = E.estimate(ba1k, s, t, L, plans, SEED, uid=uid, threads=8)
    runs = [B.exec_cfg("plain"), B.exec_cfg("batched"), B.exec_cfg("batched", chunk_probes=1),
            B.exec_cfg("batched", chunk_probes=5, grid_wgs=3), B.exec_cfg("plain", chunk_probes=256)]
    for ex in runs:
        res = B.bd_query_batch(dg, s, t, eps, L, SEED, pol, ex, uid=uid)
        assert np.all(res["status"] == 0)
        assert [(r["B"], r["G"], r["K"], r["R"]) for r in res] == plans
        assert np.array_equal(res["beta"], ref), (ex.mode, ex.chunk_probes, res["beta"] - ref)


def test_alone_equals_in_batch(ba1k):
    dg = load(ba1k, B.BD_LAYOUT_FAT | B.BD_RELABEL_DEGREE)
    s, t, eps, L = _mixed_batch(ba1k, 16, 11)
    pol = B.policy("scaled", c_B=0.05, c_R=2e-4)
    full = B.bd_query_batch(dg, s, t, eps, L, SEED, pol)
    for i in (0, 7, 15):
        one = B.bd_query_batch(dg, s[i:i + 1], t[i:i + 1], eps[i:i + 1], L[i:i + 1], SEED, pol,
                               B.exec_cfg("plain"), uid=[i])
        assert one["beta"][0] == full["beta"][i]
    other = B.bd_query_batch(dg, s, t, eps, L, SEED + 1, pol)
    assert not np.array_equal(other["beta"], full["beta"])


@pytest.mark.parametrize("layout", [B.BD_LAYOUT_COMPACT, B.BD_LAYOUT_FAT, B.BD_LAYOUT_COMPACT | B.BD_RELABEL_DEGREE])
@pytest.mark.parametrize("mode", ["plain", "batched"])
def test_full_size_sampled_parity(cl100k, layout, mode):
    # Bench shape: Chung-Lu n=1e5, L = 1000, eps = 0.05; per-probe Q checked on
    # sampled probes (the oracle runs R walk pairs of 1000 steps per probe).
    # Queries 0 and 1 of the set, and the first with R above the batched split
    # size (4096 replicas), whose probes the batched mode cuts into replica parts.
    from paper_2512_05460_amd.budgets import budget_policy
    dg = load(cl100k, layout)
    s, t = queries.uniform_pairs(cl100k.n, 4096, graphs.GRAPH_SEED + 1 + graphs.QUERY_SEED_OFFSET)
    pol = budget_policy("cl100k")
    Rs = B.bd_plan(dg, s[:200], t[:200], 0.05, 1000, pol)["R"]
    split = int(np.flatnonzero((Rs > 4096) & (Rs <= 20000))[0])
    for i in sorted({0, 1, split}):
        plan = B.bd_plan(dg, s[i:i + 1], t[i:i + 1], [0.05], [1000], pol)[0]
        if plan["R"] > 20000:
            continue
        res, q, y = B.bd_query_probes(dg, int(s[i]), int(t[i]), 0.05, 1000, i, SEED, pol, B.exec_cfg(mode))
        ks = np.linspace(0, plan["K"] - 1, 8).astype(np.uint32)
        _say(f"[sampled] query {i} K={plan['K']} R={plan['R']}")
        oq = E.probe_q(cl100k, int(s[i]), int(t[i]), 1000, i, int(plan["R"]), SEED, ks, threads=8)
        assert np.array_equal(q[ks], oq)
