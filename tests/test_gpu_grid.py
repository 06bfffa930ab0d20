"""The 1,414 x 1,414 grid workload (bipartite, large L) through the batched mode.

65,536 queries with eps over {0.02, 0.05, 0.1} and L over {500, 2000, 5000}
run in one persistent launch, with chunking from the autotuner, captured into a
hipGraph and replayed, on the layout the library picks (fat at this size). Walk counts are the throughput setting of
paper_2512_05460_amd/budgets.py (scaled policy of Algorithm 1).

  * planner parity over all 65,536 queries;
  * sampled parity at full size: beta-hat of two queries of every (eps, L)
    pair equals the oracle's bit for bit (all sums are exact fixed point);
  * graph replays equal the eager persistent launch, any number of chunk
    queues, the plain mode and the compact layout;
  * the same launch on the benchmark's tables (the probe on storage ids, the
    degree-run kernel) against the oracle on the grid in storage order.
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
def grid():
    g = graphs.workload_graph("grid1414")
    _say(f"[grid] n={g.n} nnz={g.nnz}")
    dg = B.graph_load_csr(g.n, g.row_ptr, g.col, B.BD_LAYOUT_AUTO)
    yield g, dg
    dg.free()


def _oracle_plans(g, s, t, eps, L):
    c_B, c_R, _ = BUDGETS["grid1414"]
    op = OP.Policy("scaled", c_B=c_B, c_R=c_R)
    d = g.deg
    return [OP.plan(float(eps[i]), int(L[i]), int(d[s[i]]), int(d[t[i]]), g.d_min, op) for i in range(s.size)]


@pytest.mark.timeout(300)
def test_grid_info(grid):
    g, dg = grid
    info = dg.info()
    assert info["bipartite"] == 1 and info["d_min"] == 1 and info["d_max"] == 4 and info["layout"] == 1
    assert g.n == 1414 * 1414 and g.nnz == 2 * (2 * 1414 * 1413 - round(0.05 * 2 * 1414 * 1413))


def test_grid_planner_parity(grid):
    g, dg = grid
    s, t, eps, L = queries.workload_batch("grid1414", g.n)
    plan = B.bd_plan(dg, s, t, eps, L, budget_policy("grid1414"))
    ref = np.array(_oracle_plans(g, s, t, eps, L), dtype=np.int64)
    assert np.all(plan["status"] == 0)
    got = np.stack([plan["B"], plan["G"], plan["K"], plan["R"]], axis=1).astype(np.int64)
    assert np.array_equal(got, ref)
    W = 2 * ref[:, 2] * ref[:, 3] * L.astype(np.int64)
    assert np.array_equal(plan["walk_steps"], W)
    _say(f"[grid] R {ref[:, 3].min()}..{ref[:, 3].max()}, K {sorted(set(ref[:, 2].tolist()))}, "
         f"{W.sum():.3e} walk steps")


def _sample(eps, L, per=2):
    idx = []
    for e in (0.02, 0.05, 0.1):
        for l in (500, 2000, 5000):
            idx += np.flatnonzero((eps == e) & (L == l))[:per].tolist()
    return np.array(sorted(idx))


@pytest.mark.timeout(600)
def test_grid_full_batch_graph_sampled_parity(grid):
    g, dg = grid
    s, t, eps, L = queries.workload_batch("grid1414", g.n)
    pol = budget_policy("grid1414")
    best, times = B.bd_autotune(dg, s[:2048], t[:2048], eps[:2048], L[:2048], SEED, pol)
    _say(f"[grid] autotune chunk_pairs={best.chunk_pairs} queues={best.queues} "
         f"kernel ms {np.round(times, 1).tolist()}")
    ex = B.exec_cfg("batched", chunk_pairs=best.chunk_pairs, use_graph=True, queues=best.queues)
    res, st = B.bd_query_batch(dg, s, t, eps, L, SEED, pol, ex, with_stats=True)
    assert np.all(res["status"] == 0)
    _say(f"[grid] 65,536 queries: {st['walk_steps']:.3e} steps, kernel {st['walk_kernel_ms']:.0f} ms, "
         f"{st['chunks']} chunks")
    idx = _sample(eps, L)
    plans = _oracle_plans(g, s[idx], t[idx], eps[idx], L[idx])
    ref = E.estimate(g, s[idx], t[idx], L[idx], plans, SEED, uid=idx.astype(np.uint32), threads=16)
    assert np.array_equal(res["beta"][idx], ref), (idx, res["beta"][idx] - ref)
    # the U-statistic is unbiased, not positive: at these walk counts some
    # estimates fall below zero; none is NaN or infinite
    assert np.all(np.isfinite(res["beta"]))


@pytest.mark.timeout(300)
def test_grid_replay_equals_eager_and_plain(grid):
    g, dg = grid
    s, t, eps, L = queries.workload_batch("grid1414", g.n, 2048)
    pol = budget_policy("grid1414")
    eager = B.bd_query_batch(dg, s, t, eps, L, SEED, pol, B.exec_cfg("batched"))
    for rep in range(3):
        r = B.bd_query_batch(dg, s, t, eps, L, SEED, pol, B.exec_cfg("batched", use_graph=True))
        assert np.array_equal(r["beta"], eager["beta"]), rep
        # eager work between replays
        B.bd_query_batch(dg, s[:4], t[:4], eps[:4], L[:4], SEED + rep, pol, B.exec_cfg("batched"))
    for nq in (1, 3, 8):
        r = B.bd_query_batch(dg, s, t, eps, L, SEED, pol, B.exec_cfg("batched", queues=nq, chunk_pairs=2048))
        assert np.array_equal(r["beta"], eager["beta"]), nq
    sub = np.arange(0, 2048, 97)
    plain = B.bd_query_batch(dg, s[sub], t[sub], eps[sub], L[sub], SEED, pol, B.exec_cfg("plain"),
                             uid=sub.astype(np.uint32))
    assert np.array_equal(plain["beta"], eager["beta"][sub])
    dc = B.graph_load_csr(g.n, g.row_ptr, g.col, B.BD_LAYOUT_COMPACT | B.BD_SKIP_VALIDATION)
    try:
        r = B.bd_query_batch(dc, s, t, eps, L, SEED, pol, B.exec_cfg("batched", chunk_pairs=128))
        assert np.array_equal(r["beta"], eager["beta"])
    finally:
        dc.free()


@pytest.mark.timeout(600)
def test_grid_storage_ids_graph_sampled_parity():
    # the benchmark's grid tables: hubs first with the probe on storage ids and
    # the degree-run kernel (blocks of 128 storage ids); autotuned chunking,
    # the whole set from a captured hipGraph, replayed with eager work between;
    # sampled estimates against the oracle on the grid in storage order
    g = graphs.workload_graph("grid1414")
    dg = B.graph_load_csr(g.n, g.row_ptr, g.col,
                          B.BD_LAYOUT_COMPACT | B.BD_RELABEL_DEGREE | B.BD_PROBE_STORAGE_IDS)
    try:
        assert dg.info()["lds_hubs"] == g.n
        gs, _, internal = graphs.storage_order(g)
        s, t, eps, L = queries.workload_batch("grid1414", g.n)
        pol = budget_policy("grid1414")
        best, _ = B.bd_autotune(dg, s[:2048], t[:2048], eps[:2048], L[:2048], SEED, pol)
        ex = B.exec_cfg("batched", chunk_pairs=best.chunk_pairs, use_graph=True, queues=best.queues)
        res = B.bd_query_batch(dg, s, t, eps, L, SEED, pol, ex)
        assert np.all(res["status"] == 0)
        _say(f"[grid] storage ids: chunk_pairs={best.chunk_pairs} queues={best.queues}")
        idx = _sample(eps, L)
        plans = _oracle_plans(gs, internal[s[idx]], internal[t[idx]], eps[idx], L[idx])
        ref = E.estimate(gs, internal[s[idx]], internal[t[idx]], L[idx], plans, SEED, uid=idx.astype(np.uint32),
                         threads=16)
        assert np.array_equal(res["beta"][idx], ref), (idx, res["beta"][idx] - ref)
        sub = slice(0, 4096)
        first = B.bd_query_batch(dg, s[sub], t[sub], eps[sub], L[sub], SEED, pol, ex)
        assert np.array_equal(first["beta"], res["beta"][sub])
        for rep in range(2):
            B.bd_query_batch(dg, s[:4], t[:4], eps[:4], L[:4], SEED + rep, pol, B.exec_cfg("batched"))
            again = B.bd_query_batch(dg, s[sub], t[sub], eps[sub], L[sub], SEED, pol, ex)
            assert np.array_equal(again["beta"], first["beta"]), rep
    finally:
        dg.free()
