"""Seeded input generators: canonical CSR form and the workload shapes."""

import numpy as np
import pytest
import scipy.sparse.csgraph as csgraph

from synth import graphs, queries


def _check_canonical(g):
    rp, col = g.row_ptr, g.col
    assert rp.dtype == np.int64 and col.dtype == np.int32
    assert rp[0] == 0 and rp[-1] == col.size
    assert np.all(np.diff(rp) >= 1), "every node has a neighbour"
    rows = np.repeat(np.arange(g.n), np.diff(rp))
    assert np.all(col != rows), "no self-loops"
    for v in range(0, g.n, max(1, g.n // 200)):
        nb = col[rp[v]:rp[v + 1]]
        assert np.all(np.diff(nb) > 0), "sorted, no duplicates"
    A = g.scipy()
    assert (A != A.T).nnz == 0, "symmetric"
    ncomp, _ = csgraph.connected_components(A, directed=False)
    assert ncomp == 1


@pytest.mark.parametrize("maker", [
    lambda: graphs.complete_graph(6), lambda: graphs.cycle_graph(9),
    lambda: graphs.path_graph(7), lambda: graphs.random_connected(40, 0.1, 3),
])
def test_small_graphs_canonical(maker):
    _check_canonical(maker())


def test_ba1k_shape():
    g = graphs.workload_graph("ba1k")
    _check_canonical(g)
    assert g.n == 1000
    assert g.nnz == 2 * (6 + 3 * 996)
    assert g.d_min == 3


def test_cl100k_shape():
    g = graphs.workload_graph("cl100k")
    _check_canonical(g)
    assert 95_000 <= g.n <= 100_000
    assert 9.5 <= g.nnz / g.n <= 10.5
    assert g.d_min == 1 and g.d_max > 500


def test_grid_shape():
    g = graphs.workload_graph("grid1414")
    assert g.n == 1414 * 1414
    assert g.nnz == 2 * (3_995_964 - 199_798)
    ncomp, _ = csgraph.connected_components(g.scipy(), directed=False)
    assert ncomp == 1
    assert g.d_max == 4


def test_generators_deterministic():
    a = graphs.chung_lu(5000, 8.0, 2.5, 11)
    b = graphs.chung_lu(5000, 8.0, 2.5, 11)
    assert np.array_equal(a.row_ptr, b.row_ptr) and np.array_equal(a.col, b.col)


def test_uniform_pairs():
    s, t = queries.uniform_pairs(50, 20000, 1)
    assert np.all(s != t) and s.min() >= 0 and t.max() < 50
    # uniform over ordered pairs: each node appears as t about 20000/50 times
    cnt = np.bincount(t, minlength=50)
    assert abs(cnt.mean() - 400) < 1e-9 and cnt.std() < 60


def test_inverse_cdf_equals_searchsorted():
    rng = np.random.default_rng(3)
    for n, gamma in ((1, 2.5), (7, 2.1), (1000, 2.5), (200_000, 2.3)):
        w = np.arange(1, n + 1, dtype=np.float64) ** (-1.0 / (gamma - 1.0))
        cdf = np.cumsum(w)
        cdf /= cdf[-1]
        first = np.searchsorted(cdf, np.arange(4 * n, dtype=np.float64) / (4 * n), side="right")
        r = rng.random(200_000)
        r[:4] = [0.0, np.nextafter(1.0, 0.0), cdf[n // 2], np.nextafter(cdf[n // 2], 0.0)]
        assert np.array_equal(graphs._inverse_cdf(cdf, r, first, 4 * n),
                              np.searchsorted(cdf, r, side="right"))


def test_largest_component_matches_rebuild():
    # several components: the kept one rebuilt from its edge list is identical
    g = graphs.chung_lu(3000, 1.5, 2.2, 11, lcc=False)
    lc = graphs.largest_component(g)
    import scipy.sparse.csgraph as csgraph
    _, labels = csgraph.connected_components(g.scipy(), directed=False)
    big = np.argmax(np.bincount(labels))
    keep = labels == big
    assert lc.n == keep.sum() < g.n
    new_id = np.cumsum(keep) - 1
    rows = np.repeat(np.arange(g.n), g.deg)
    m = keep[rows]
    ref = graphs.csr_from_edges(lc.n, new_id[rows[m]], new_id[g.col[m]])
    assert np.array_equal(lc.row_ptr, ref.row_ptr) and np.array_equal(lc.col, ref.col)
    assert lc.col.dtype == np.int32


def test_native_chung_lu():
    # canonical CSR, connected, independent of the thread count, degrees near target
    a = graphs.chung_lu_native(50_000, 25.0, 2.2, 3, threads=1)
    b = graphs.chung_lu_native(50_000, 25.0, 2.2, 3, threads=4)
    assert np.array_equal(a.row_ptr, b.row_ptr) and np.array_equal(a.col, b.col)
    assert a.col.dtype == np.int32 and a.row_ptr.dtype == np.int64
    A = a.scipy()
    assert (A != A.T).nnz == 0 and A.diagonal().sum() == 0
    for v in range(0, a.n, 97):
        row = a.col[a.row_ptr[v]:a.row_ptr[v + 1]]
        assert np.all(np.diff(row) > 0)
    import scipy.sparse.csgraph as csgraph
    assert csgraph.connected_components(A, directed=False)[0] == 1
    assert 0.9 * 50_000 < a.n <= 50_000 and 22 < a.nnz / a.n < 26
    c = graphs.chung_lu_native(50_000, 25.0, 2.2, 4, threads=2)
    assert not np.array_equal(a.col[:1000], c.col[:1000])


def test_storage_order():
    # node i of the result is the node of rank i in descending degree (ties by
    # ascending id); each row keeps the given neighbour order, renamed
    g = graphs.barabasi_albert(300, 3, 11)
    gs, order, internal = graphs.storage_order(g)
    assert sorted(order.tolist()) == list(range(g.n))
    assert np.array_equal(internal[order], np.arange(g.n))
    d = g.deg[order]
    assert np.all(np.diff(d) <= 0)
    ties = (d[1:] == d[:-1])
    assert np.all(order[1:][ties] > order[:-1][ties])
    for i in range(g.n):
        v = order[i]
        row = gs.col[gs.row_ptr[i]:gs.row_ptr[i + 1]]
        assert np.array_equal(order[row], g.col[g.row_ptr[v]:g.row_ptr[v + 1]])
