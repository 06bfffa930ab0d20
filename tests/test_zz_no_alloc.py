"""The allocation-free entry point (bd_query_batch_noalloc) against
bd_query_batch on the same inputs, through the C ABI: identical results bit for
bit, on consecutive calls that share the fixed scratch array (the second one
smaller), in batched mode with split probes and in plain mode; a batch beyond
the array is refused with BD_E_SCRATCH and leaves later calls intact."""

import numpy as np
import pytest

from paper_2512_05460_amd import binding as B
from synth import graphs, queries

pytestmark = pytest.mark.gpu

SEED = graphs.PHILOX_SEED


def _same(a, b):
    for f in ("status", "K", "R", "B", "G", "L", "walk_steps"):
        assert np.array_equal(a[f], b[f]), f
    assert np.array_equal(a["beta"], b["beta"])  # bit for bit (exact sums)


@pytest.fixture(scope="module", params=["hubs", "storage-ids"])
def ba(request):
    # compact hubs first, and the storage-id layout with the degree-run kernel
    g = graphs.workload_graph("ba1k")
    flags = B.BD_LAYOUT_COMPACT | B.BD_RELABEL_DEGREE
    if request.param == "storage-ids":
        flags |= B.BD_PROBE_STORAGE_IDS
    dg = B.graph_load_csr(g.n, g.row_ptr, g.col, flags)
    yield g, dg
    dg.free()


def test_noalloc_matches_batch_consecutive_calls(ba):
    g, dg = ba
    s, t = queries.uniform_pairs(g.n, 48, 31)
    s[5] = t[5]  # one invalid query in the batch
    L = np.where(np.arange(48) % 3 == 0, 0, np.where(np.arange(48) % 3 == 1, 7, 40)).astype(np.int32)
    # R above the split size: batched mode cuts these probes into replica parts
    big = B.policy("fixed", B=1, R=4500)
    ex = B.exec_cfg("batched")
    ref = B.bd_query_batch(dg, s, t, 0.1, L, SEED, big, ex)
    got, st = B.bd_query_batch_noalloc(dg, s, t, 0.1, L, SEED, big, ex, with_stats=True)
    assert got["status"][5] == B.BD_E_INVALID
    _same(got, ref)
    assert st["walk_kernel_ms"] == 0.0 and st["launches"] >= 1 and st["walk_steps"] == ref["walk_steps"][
        ref["status"] == 0].sum()
    # second call, smaller, different budget: the scratch holds the last call's contents
    small = B.policy("scaled", c_B=0.2, c_R=128.0 / 2 ** 14)
    ref2 = B.bd_query_batch(dg, s[:6], t[:6], 0.1, 200, SEED, small, ex, uid=np.arange(100, 106))
    got2 = B.bd_query_batch_noalloc(dg, s[:6], t[:6], 0.1, 200, SEED, small, ex, uid=np.arange(100, 106))
    _same(got2, ref2)
    assert np.all(got2["status"][[0, 1, 2, 3, 4]] == 0)


def test_noalloc_plain_mode(ba):
    g, dg = ba
    s, t = queries.uniform_pairs(g.n, 9, 5)
    pol = B.policy("fixed", B=3, R=70)
    for mode in ("plain", "batched"):
        ex = B.exec_cfg(mode)
        _same(B.bd_query_batch_noalloc(dg, s, t, 0.1, 33, SEED, pol, ex), B.bd_query_batch(dg, s, t, 0.1, 33, SEED, pol, ex))


def test_noalloc_refuses_batch_beyond_scratch(ba):
    g, dg = ba
    # about 650 bytes per query: 120,000 queries need more than the 64 MiB array
    n = 120_000
    s, t = queries.uniform_pairs(g.n, n, 77)
    with pytest.raises(B.ProbeWalkError) as e:
        B.bd_query_batch_noalloc(dg, s, t, 0.5, 1, SEED, B.policy("fixed", B=1, R=2), B.exec_cfg("batched"))
    assert e.value.code == B.BD_E_SCRATCH
    # a following call works and still matches
    pol = B.policy("fixed", B=2, R=64)
    _same(B.bd_query_batch_noalloc(dg, s[:4], t[:4], 0.1, 12, SEED, pol),
          B.bd_query_batch(dg, s[:4], t[:4], 0.1, 12, SEED, pol))
