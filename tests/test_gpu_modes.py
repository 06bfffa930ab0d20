"""Execution modes on the GPU: split probes, batched work stealing and the
served mode (continuous batching), each checked bit for bit against the
oracle or against another mode (all sums are exact, so every mode must agree
exactly).
"""

import sys
import time

import numpy as np
import pytest

from oracle import estimator as E
from oracle import planner as OP
from paper_2512_05460_amd import binding as B
from synth import graphs, queries

pytestmark = pytest.mark.gpu

SEED = 0x5E12ED


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


_cache = {}


def _graph(key, flags):
    if (key, flags) not in _cache:
        g = graphs.workload_graph(key)
        _cache[(key, flags)] = (g, B.graph_load_csr(g.n, g.row_ptr, g.col, flags))
    return _cache[(key, flags)]


@pytest.mark.parametrize("flags", [B.BD_LAYOUT_COMPACT, B.BD_LAYOUT_CSR | B.BD_RELABEL_DEGREE])
def test_split_probe_parity(flags):
    # R = 5000 > the replica-part size: batched and served launches cut each probe's replicas
    # into parts (2560 + 2440 in batched launches); plain launches keep whole probes.
    g, dg = _graph("ba1k", flags)
    s, t, L = 10, 900, 5
    pol = B.policy("fixed", B=1, R=5000)
    plan = OP.plan(0.1, L, 1, 1, 1, OP.Policy("fixed", B_fixed=1, R_fixed=5000))
    ob, oq, oy = E.estimate(g, [s], [t], L, [plan], SEED, uid=[3], want_q=True, threads=1)
    # batched: automatic kernel choice, forced wave-uniform kernel, general only
    for ex in (B.exec_cfg("batched"), B.exec_cfg("batched", uniform_min_r=48),
               B.exec_cfg("batched", uniform_min_r=-1), B.exec_cfg("batched", uniform_min_r=-1, chunk_pairs=700),
               B.exec_cfg("plain")):
        res, q, y = B.bd_query_probes(dg, s, t, 0.1, L, 3, SEED, pol, ex)
        assert np.array_equal(q, oq), ex.as_dict()
        assert np.array_equal(y, oy) and res["beta"] == ob[0]


def _mixed(g, n, seed, Ls=(0, 3, 20, 100)):
    s, t = queries.uniform_pairs(g.n, n, seed)
    eps, L = queries.mixed_eps_L(n, [0.3, 0.5], list(Ls), seed + 1)
    return s, t, eps, L


def test_batched_equals_plain_with_splits():
    g, dg = _graph("ba1k", B.BD_LAYOUT_COMPACT)
    s, t, eps, L = _mixed(g, 12, 5)
    hubs = np.argsort(g.deg)[::-1][:4].astype(np.int32)
    s = np.concatenate([s, hubs[:2]])
    t = np.concatenate([t, hubs[2:]])
    eps = np.concatenate([eps, [0.5, 0.5]])
    L = np.concatenate([L, [100, 100]]).astype(np.int32)
    pol = B.policy("scaled", c_B=0.02, c_R=0.2)  # R from 2 to > 4096: small-R, whole and split probes
    plan = B.bd_plan(dg, s, t, eps, L, pol)
    _say("R range", plan["R"].min(), plan["R"].max())
    assert plan["R"].max() > 4096 and plan["R"].min() < 48
    a = B.bd_query_batch(dg, s, t, eps, L, SEED, pol, B.exec_cfg("plain"))
    b = B.bd_query_batch(dg, s, t, eps, L, SEED, pol, B.exec_cfg("batched"))
    c = B.bd_query_batch(dg, s, t, eps, L, SEED, pol, B.exec_cfg("batched", grid_wgs=7))
    assert np.array_equal(a["beta"], b["beta"]) and np.array_equal(a["beta"], c["beta"])
    for ex in (B.exec_cfg("batched", uniform_min_r=48), B.exec_cfg("batched", uniform_min_r=1, queues=3),
               B.exec_cfg("batched", uniform_min_r=-1, chunk_pairs=1000)):
        d = B.bd_query_batch(dg, s, t, eps, L, SEED, pol, ex)
        assert np.array_equal(a["beta"], d["beta"]), ex.as_dict()


def test_served_alone_equals_mix():
    g, dg = _graph("ba1k", B.BD_LAYOUT_COMPACT)
    pol = B.policy("scaled", c_B=0.05, c_R=0.005)
    srv = B.Server(dg, pol, max_queries=4096)
    try:
        s, t, eps, L = _mixed(g, 6, 21)
        uid = np.arange(6) + 1000
        rid = srv.submit(s, t, eps, L, SEED, uid=uid)
        alone, lat = srv.wait(rid)
        assert np.all(alone["status"] == 0)
        # the same request again, now among many others submitted around it
        others = []
        for j in range(8):
            so, to, eo, lo = _mixed(g, 1 + 5 * j, 100 + j)
            others.append(srv.submit(so, to, eo, lo, SEED + j, uid=np.arange(so.size) + 50 * j))
            if j == 3:
                rid2 = srv.submit(s, t, eps, L, SEED, uid=uid)
        mixed, lat2 = srv.wait(rid2)
        for r in others:
            out, _ = srv.wait(r)
            assert np.all(out["status"] == 0)
        assert np.array_equal(alone["beta"], mixed["beta"])
        _say(f"[served] latency alone {lat:.1f} ms, in the mix {lat2:.1f} ms")
        # and equal to the batched call with the same uids
        ref = B.bd_query_batch(dg, s, t, eps, L, SEED, pol, uid=uid)
        assert np.array_equal(ref["beta"], alone["beta"])
    finally:
        srv.destroy()


def test_served_many_completions_per_slice():
    # 20,000 one-step queries fit one slice: its completion ring holds more
    # entries than the part copied back after every slice
    g, dg = _graph("ba1k", B.BD_LAYOUT_COMPACT)
    n = 20000
    s, t = queries.uniform_pairs(g.n, n, 404)
    pol = B.policy("fixed", B=1, R=2)
    ref = B.bd_query_batch(dg, s, t, 0.5, 1, SEED, pol, B.exec_cfg("batched"))
    srv = B.Server(dg, pol)
    try:
        out, _ = srv.wait(srv.submit(s, t, 0.5, 1, SEED))
        assert np.all(out["status"] == 0)
        assert np.array_equal(out["beta"], ref["beta"])
        # and in several requests at once
        rids = [srv.submit(s[i::3], t[i::3], 0.5, 1, SEED, uid=np.arange(n)[i::3]) for i in range(3)]
        for i, rid in enumerate(rids):
            o, _ = srv.wait(rid)
            assert np.array_equal(o["beta"], ref["beta"][i::3])
    finally:
        srv.destroy()


def test_served_admission_caps_and_split():
    g, dg = _graph("ba1k", B.BD_LAYOUT_COMPACT)
    pol = B.policy("fixed", B=1, R=4500)  # every probe split into replica parts
    srv = B.Server(dg, pol, max_queries=4)
    try:
        with pytest.raises(B.ProbeWalkError) as ei:
            srv.submit(np.arange(5), np.arange(5) + 10, 0.1, 3, SEED)
        assert ei.value.code == B.BD_E_FULL
        rids, inputs = [], []
        for j in range(5):
            s, t = queries.uniform_pairs(g.n, 3, 300 + j)
            L = np.array([2, 3, 4], dtype=np.int32)
            inputs.append((s, t, L))
            rids.append(srv.submit(s, t, 0.1, L, SEED, uid=np.arange(3) + 10 * j))
        done = set()
        t0 = time.time()
        while len(done) < len(rids) and time.time() - t0 < 60:
            for i, r in enumerate(rids):
                if i in done:
                    continue
                ok, out, lat = srv.poll(r)
                if ok:
                    s, t, L = inputs[i]
                    ref = B.bd_query_batch(dg, s, t, 0.1, L, SEED, pol, uid=np.arange(3) + 10 * i)
                    assert np.array_equal(out["beta"], ref["beta"])
                    done.add(i)
            time.sleep(0.01)
        assert len(done) == len(rids)
    finally:
        srv.destroy()


def test_served_walk_step_admission():
    # walk-budget admission: a request above the cap is refused; requests under
    # it are admitted one at a time when together they exceed it
    g, dg = _graph("ba1k", B.BD_LAYOUT_COMPACT)
    pol = B.policy("fixed", B=2, R=64)
    per_query = 2 * 74 * 64 * 40                      # K = 74, R = 64, L = 40
    srv = B.Server(dg, pol, max_steps=3 * per_query)
    try:
        with pytest.raises(B.ProbeWalkError) as ei:
            srv.submit(np.arange(4), np.arange(4) + 50, 0.1, 40, SEED)
        assert ei.value.code == B.BD_E_FULL
        reqs = [queries.uniform_pairs(g.n, 3, 900 + j) for j in range(4)]
        rids = [srv.submit(s, t, 0.1, 40, SEED, uid=np.arange(3) + 10 * j) for j, (s, t) in enumerate(reqs)]
        for j, rid in enumerate(rids):
            out, _ = srv.wait(rid)
            s, t = reqs[j]
            ref = B.bd_query_batch(dg, s, t, 0.1, 40, SEED, pol, uid=np.arange(3) + 10 * j)
            assert np.array_equal(out["beta"], ref["beta"])
    finally:
        srv.destroy()


def test_served_destroy_with_pending_work():
    g, dg = _graph("ba1k", B.BD_LAYOUT_COMPACT)
    srv = B.Server(dg, B.policy("fixed", B=4, R=256), max_queries=2)
    for j in range(6):
        s, t = queries.uniform_pairs(g.n, 2, 700 + j)
        srv.submit(s, t, 0.1, 50, SEED)
    srv.destroy()  # must return: in-flight slices drain, pending requests are cancelled


def test_graph_replay_matches_eager():
    g, dg = _graph("ba1k", B.BD_LAYOUT_COMPACT)
    pol = B.policy("scaled", c_B=0.05, c_R=0.05)
    ex_graph = B.exec_cfg("batched", use_graph=True)
    ex_eager = B.exec_cfg("batched")
    # fixed endpoints, eps and L keep the launch shape; seeds and uids vary per replay
    s = np.full(16, 7, dtype=np.int32)
    t = np.full(16, 900, dtype=np.int32)
    eps = np.full(16, 0.3)
    L = np.full(16, 100, dtype=np.int32)
    for rep in range(4):
        seed = SEED + 17 * rep
        uid = np.arange(16) + 100 * rep
        got = B.bd_query_batch(dg, s, t, eps, L, seed, pol, ex_graph, uid=uid)
        # eager work in between replays
        other = B.bd_query_batch(dg, s[:3], t[:3] + 1, eps[:3], L[:3], seed + 1, pol, ex_eager)
        assert np.all(other["status"] == 0)
        ref = B.bd_query_batch(dg, s, t, eps, L, seed, pol, ex_eager, uid=uid)
        assert np.array_equal(got["beta"], ref["beta"]), rep
        again = B.bd_query_batch(dg, s, t, eps, L, seed, pol, ex_graph, uid=uid)
        assert np.array_equal(again["beta"], ref["beta"]), rep
    # alternating walk-sharing factors on one batch: each replay matches eager
    for M in (1, 2, 4, 1, 4):
        pm = B.policy("fixed", B=4, R=64, share=M)
        got = B.bd_query_batch(dg, s, t, eps, L, SEED, pm, ex_graph)
        ref = B.bd_query_batch(dg, s, t, eps, L, SEED, pm, ex_eager)
        assert np.array_equal(got["beta"], ref["beta"]), M


def test_autotune():
    g, dg = _graph("ba1k", B.BD_LAYOUT_COMPACT)
    s, t = queries.uniform_pairs(g.n, 8, 77)
    pol = B.policy("scaled", c_B=0.05, c_R=0.05)
    best, times = B.bd_autotune(dg, s, t, 0.3, 100, SEED, pol, "batched")
    _say(f"[autotune] best chunk_pairs={best.chunk_pairs} queues={best.queues} times={np.round(times, 2)}")
    assert len(times) == 9 and best.chunk_pairs in (128, 256, 512, 1024, 2048, 4096, 8192, 16384)
    assert best.queues in (1, 8)
    a = B.bd_query_batch(dg, s, t, 0.3, 100, SEED, pol, best)
    b = B.bd_query_batch(dg, s, t, 0.3, 100, SEED, pol)
    assert np.array_equal(a["beta"], b["beta"])


# ---------------------------------------------------------------------------
# Truncated series, mixing factor, Theorem 3.8's L, stabilization rule
# ---------------------------------------------------------------------------
from oracle import exact as X  # noqa: E402
from oracle import stabilize as OS  # noqa: E402


@pytest.mark.parametrize("key,flags", [("ba1k", B.BD_LAYOUT_COMPACT), ("ba1k", B.BD_LAYOUT_CSR | B.BD_RELABEL_DEGREE),
                                       ("cl100k", B.BD_LAYOUT_COMPACT)])
def test_truncated_beta_vs_oracle(key, flags):
    g, dg = _graph(key, flags)
    s, t = queries.uniform_pairs(g.n, 70, 11)
    for L in ((0, 1, 7, 200) if key == "ba1k" else (50,)):
        got = B.bd_truncated_beta(dg, s, t, L)
        idx = range(70) if key == "ba1k" else range(0, 70, 10)
        for i in idx:
            ref = X.beta_truncated(g, int(s[i]), int(t[i]), L)
            assert got[i] == pytest.approx(ref, rel=1e-11), (L, i)


@pytest.mark.parametrize("maker,lam", [(lambda: graphs.complete_graph(7), 1 / 6),
                                       (lambda: graphs.cycle_graph(9), float(np.cos(np.pi / 9)))])
def test_lambda_closed_forms(maker, lam):
    g = maker()
    dg = B.graph_load_csr(g.n, g.row_ptr, g.col, B.BD_LAYOUT_CSR)
    assert B.bd_graph_lambda(dg, 300, 7) == pytest.approx(lam, rel=1e-8)


def test_lambda_ba1k_and_theorem_L():
    g, dg = _graph("ba1k", B.BD_LAYOUT_COMPACT)
    ref = X.mixing_factor(g)
    lam = B.bd_graph_lambda(dg, 3000, 3)
    _say(f"[lambda] ba1k dense {ref:.8f} power {lam:.8f}")
    assert lam == pytest.approx(ref, rel=1e-4)
    s, t = queries.uniform_pairs(g.n, 20, 4)
    Ls = B.bd_theorem_L(dg, s, t, 0.1, ref)
    for i in range(20):
        assert Ls[i] == OP.theorem_L(g.n, 0.1, ref, int(g.deg[s[i]]), int(g.deg[t[i]]))


def test_stabilized_matches_oracle():
    g, dg = _graph("ba1k", B.BD_LAYOUT_COMPACT)
    s, t = queries.uniform_pairs(g.n, 6, 9)
    pol = B.policy("scaled", c_B=0.05, c_R=0.05)
    opol = OP.Policy("scaled", c_B=0.05, c_R=0.05)
    res, Ls = B.bd_query_stabilized(dg, s, t, 0.3, 64, SEED, pol, uid=np.arange(6))
    for i in range(6):
        ob, oL = OS.stabilized(g, int(s[i]), int(t[i]), 0.3, 64, SEED, i, opol)
        assert Ls[i] == oL and res["beta"][i] == ob, (i, Ls[i], oL)


@pytest.mark.timeout(300)
def test_stabilization_proxy_error():
    # Section 4.3's check of the rule: relative gap between the estimate at
    # L_stop and the estimate at L_max = 256, here on the Chung-Lu n=1e5 graph
    # at eps = 0.1 with its calibrated walk counts
    from paper_2512_05460_amd.budgets import budget_policy
    g, dg = _graph("cl100k", B.BD_LAYOUT_COMPACT | B.BD_RELABEL_DEGREE)
    s, t = queries.uniform_pairs(g.n, 24, 515)
    pol = budget_policy("cl100k")
    eps = 0.1
    res, Ls = B.bd_query_stabilized(dg, s, t, eps, 256, SEED, pol)
    ref = B.bd_query_batch(dg, s, t, eps, 256, SEED, pol)
    assert np.all(res["status"] == 0) and np.all(ref["status"] == 0)
    assert np.all((Ls >= 2) & (Ls <= 256)) and np.all((Ls & (Ls - 1)) == 0)
    proxy = np.abs(res["beta"] - ref["beta"]) / np.abs(ref["beta"])
    _say(f"[stabilize] L_stop {np.bincount(np.log2(Ls).astype(int)).tolist()}, proxy error median "
         f"{np.median(proxy):.4f}, max {proxy.max():.4f}, within eps {(proxy <= eps).mean():.3f}")
    assert np.median(proxy) <= eps
