"""Failure handling forced from the host, with every kernel ending normally:

  * the watchdog deadline (bd_exec.deadline_ms): a batch stopped part-way in
    the batched, plain and hipGraph-replayed launches returns early; the
    queries it abandoned carry BD_E_TIMEOUT and the ones it finished equal an
    unbounded run bit for bit; the next call is unaffected;
  * request cancellation in the server: a queued request finishes at once as
    cancelled; an admitted one keeps the results of the queries that finished
    and the rest are cancelled; requests admitted afterwards into the freed
    slots give the batched results bit for bit.
"""

import time

import numpy as np
import pytest

from paper_2512_05460_amd import binding as B
from synth import graphs, queries

pytestmark = pytest.mark.gpu

SEED = graphs.PHILOX_SEED


@pytest.fixture(scope="module", params=["hubs", "storage-ids"])
def cl(request):
    # compact hubs first, and the storage-id layout with the degree-run kernel
    g = graphs.workload_graph("cl100k")
    flags = B.BD_LAYOUT_COMPACT | B.BD_RELABEL_DEGREE
    if request.param == "storage-ids":
        flags |= B.BD_PROBE_STORAGE_IDS
    dg = B.graph_load_csr(g.n, g.row_ptr, g.col, flags)
    if request.param == "storage-ids":
        assert dg.info()["lds_hubs"] == g.n
    yield g, dg
    dg.free()


POL = B.policy("fixed", B=8, R=2000)  # 296 probes x 2000 replicas per query


@pytest.mark.parametrize("mode,graph", [("batched", False), ("batched", True), ("plain", False)])
def test_deadline_abandons_and_keeps_finished(cl, mode, graph):
    g, dg = cl
    s, t = queries.uniform_pairs(g.n, 48, 123)
    L = np.where(np.arange(48) % 2 == 0, 300, 1000).astype(np.int32)
    full = B.bd_query_batch(dg, s, t, 0.1, L, SEED, POL, B.exec_cfg(mode, use_graph=graph))
    assert np.all(full["status"] == 0)
    t0 = time.perf_counter()
    full2 = B.bd_query_batch(dg, s, t, 0.1, L, SEED, POL, B.exec_cfg(mode, use_graph=graph))
    dt_full = time.perf_counter() - t0
    t0 = time.perf_counter()
    cut = B.bd_query_batch(dg, s, t, 0.1, L, SEED, POL, B.exec_cfg(mode, use_graph=graph, deadline_ms=20.0))
    dt_cut = time.perf_counter() - t0
    st = cut["status"]
    assert set(np.unique(st)) <= {0, B.BD_E_TIMEOUT}
    assert np.any(st == B.BD_E_TIMEOUT), f"nothing abandoned in {dt_cut:.3f} s (unbounded {dt_full:.3f} s)"
    ok = st == 0
    assert np.array_equal(cut["beta"][ok], full["beta"][ok])
    assert np.all(cut["beta"][~ok] == 0.0)
    assert dt_cut < dt_full
    # the workspace and the abort flag are clean for the next call
    again = B.bd_query_batch(dg, s, t, 0.1, L, SEED, POL, B.exec_cfg(mode, use_graph=graph))
    assert np.array_equal(again["beta"], full["beta"]) and np.array_equal(full2["beta"], full["beta"])


def test_server_cancel(cl):
    g, dg = cl
    pol = B.policy("fixed", B=4, R=3000)
    sa, ta = queries.uniform_pairs(g.n, 400, 7)
    sd, td = queries.uniform_pairs(g.n, 300, 8)
    sc, tc = queries.uniform_pairs(g.n, 300, 9)
    ref_a = B.bd_query_batch(dg, sa, ta, 0.1, 600, SEED, pol, uid=np.arange(400))
    ref_c = B.bd_query_batch(dg, sc, tc, 0.1, 600, SEED, pol, uid=np.arange(1000, 1300))
    srv = B.Server(dg, pol, max_queries=500)
    ra = srv.submit(sa, ta, 0.1, 600, SEED, uid=np.arange(400))
    rd = srv.submit(sd, td, 0.1, 600, SEED, uid=np.arange(500, 800))  # queued: 700 > 500 slots
    time.sleep(0.05)
    srv.cancel(rd)
    od, _ = srv.wait(rd, 5000.0)
    assert np.all(od["status"] == B.BD_E_CANCELLED)
    srv.cancel(ra)
    oa, _ = srv.wait(ra, 60000.0)
    sta = oa["status"]
    assert set(np.unique(sta)) <= {0, B.BD_E_CANCELLED}
    ok = sta == 0
    assert np.array_equal(oa["beta"][ok], ref_a["beta"][ok])
    # the freed slots serve a new request correctly (their device state was cleared)
    rc = srv.submit(sc, tc, 0.1, 600, SEED, uid=np.arange(1000, 1300))
    oc, _ = srv.wait(rc, 60000.0)
    assert np.all(oc["status"] == 0)
    assert np.array_equal(oc["beta"], ref_c["beta"])
    with pytest.raises(B.ProbeWalkError) as e:
        srv.cancel(ra)  # collected already
    assert e.value.code == B.BD_E_NOTFOUND
    srv.destroy()
