"""Seeded graph generators and the canonical CSR form.

Canonical CSR (the form every consumer receives):
  * undirected, simple: symmetric adjacency, no self-loops, no duplicate edges;
  * neighbours of each node sorted ascending (the neighbour index a walk draws
    is an index into this sorted list, so the order is part of the contract);
  * ``row_ptr`` int64 of length n+1, ``col`` int32 of length nnz = 2|E|.

Generators are deterministic functions of their seed (numpy PCG64), so every
machine that runs them builds the same graph bit for bit.
"""

from __future__ import annotations

import dataclasses
import functools

import numpy as np
import scipy.sparse as sp
import scipy.sparse.csgraph as csgraph


@dataclasses.dataclass
class Csr:
    n: int
    row_ptr: np.ndarray  # int64[n+1]
    col: np.ndarray  # int32[nnz]
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    # degrees are computed once per graph (the arrays are not modified after construction)
    @functools.cached_property
    def deg(self) -> np.ndarray:
        return np.diff(self.row_ptr).astype(np.int64)

    @functools.cached_property
    def d_min(self) -> int:
        return int(self.deg.min())

    @functools.cached_property
    def d_max(self) -> int:
        return int(self.deg.max())

    def footprint_bytes(self) -> int:
        """int32 CSR footprint: 4(n+1) + 4 nnz bytes."""
        return 4 * (self.n + 1) + 4 * self.nnz

    def scipy(self) -> sp.csr_matrix:
        data = np.ones(self.nnz, dtype=np.float64)
        return sp.csr_matrix((data, self.col, self.row_ptr), shape=(self.n, self.n))


def csr_from_edges(n: int, u: np.ndarray, v: np.ndarray, name: str = "") -> Csr:
    """Build the canonical CSR of the undirected simple graph spanned by (u, v)."""
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    keep = u != v
    u, v = u[keep], v[keep]
    a = np.concatenate([u, v])
    b = np.concatenate([v, u])
    key = np.unique(a * np.int64(n) + b)  # sorts by (row, col) and dedupes
    rows = key // n
    cols = (key - rows * n).astype(np.int32)
    counts = np.bincount(rows, minlength=n).astype(np.int64)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return Csr(n=n, row_ptr=row_ptr, col=cols, name=name)


def largest_component(g: Csr, name: str | None = None) -> Csr:
    """Restrict to the largest connected component, keeping relative node order."""
    ncomp, labels = csgraph.connected_components(g.scipy(), directed=False)
    if ncomp == 1:
        if name is not None:
            g.name = name
        return g
    sizes = np.bincount(labels)
    big = int(np.argmax(sizes))
    keep = labels == big
    m = int(keep.sum())
    new_id = np.full(g.n, -1, dtype=np.int64)
    new_id[keep] = np.arange(m, dtype=np.int64)
    # A component is closed under adjacency, so a kept node keeps its whole
    # neighbour list; the renaming is increasing, so rows stay in order and
    # neighbour lists stay sorted: the result is already canonical.
    deg = g.deg
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(deg[keep], out=row_ptr[1:])
    col = new_id[g.col[np.repeat(keep, deg)]].astype(np.int32)
    return Csr(n=m, row_ptr=row_ptr, col=col, name=name if name is not None else g.name)


def relabel(g: Csr, perm: np.ndarray, name: str | None = None) -> Csr:
    """Rename node i to perm[i] and return the canonical CSR of the result."""
    rows = np.repeat(np.arange(g.n, dtype=np.int64), g.deg)
    u = perm[rows]
    v = perm[g.col.astype(np.int64)]
    return csr_from_edges(g.n, u, v, name=name if name is not None else g.name)


def storage_order(g: Csr):
    """The graph as a library that stores nodes in descending-degree order
    (ties by ascending id) holds it: node i of the result is the node of rank
    i, and each row keeps the given neighbour order with the ids renamed (not
    re-sorted). Returns (graph, order, internal): order[i] is the original id
    of node i, internal the inverse permutation."""
    order = np.argsort(-g.deg, kind="stable")
    internal = np.empty(g.n, dtype=np.int64)
    internal[order] = np.arange(g.n)
    deg = g.deg[order]
    rp = np.zeros(g.n + 1, dtype=np.int64)
    np.cumsum(deg, out=rp[1:])
    src = np.repeat(g.row_ptr[:-1][order], deg) + (np.arange(g.nnz) - np.repeat(rp[:-1], deg))
    col = internal[g.col[src]].astype(np.int32)
    return Csr(n=g.n, row_ptr=rp, col=col, name=g.name + "-storage"), order, internal


# --------------------------------------------------------------------------- #
# Small textbook graphs (closed forms for the exact distance exist on these)
# --------------------------------------------------------------------------- #

def complete_graph(n: int) -> Csr:
    i, j = np.triu_indices(n, k=1)
    return csr_from_edges(n, i, j, name=f"K{n}")


def cycle_graph(n: int) -> Csr:
    i = np.arange(n)
    return csr_from_edges(n, i, (i + 1) % n, name=f"C{n}")


def path_graph(n: int) -> Csr:
    i = np.arange(n - 1)
    return csr_from_edges(n, i, i + 1, name=f"P{n}")


def random_connected(n: int, p: float, seed: int) -> Csr:
    """Erdos-Renyi G(n, p) plus a random Hamiltonian path and one triangle.

    The path makes it connected; the triangle on three path-consecutive nodes
    makes it non-bipartite.
    """
    rng = np.random.default_rng(seed)
    i, j = np.triu_indices(n, k=1)
    pick = rng.random(i.size) < p
    order = rng.permutation(n)
    u = np.concatenate([i[pick], order[:-1], order[:1]])
    v = np.concatenate([j[pick], order[1:], order[2:3]])
    return csr_from_edges(n, u, v, name=f"G({n},{p})#{seed}")


# --------------------------------------------------------------------------- #
# Workload generators
# --------------------------------------------------------------------------- #

def barabasi_albert(n: int, m: int, seed: int) -> Csr:
    """Preferential attachment grown from the complete graph on m+1 nodes.

    Each new node v attaches to m distinct existing nodes, each drawn with
    probability proportional to its current degree (uniform draws from the
    list of edge endpoints, repeats rejected).
    """
    rng = np.random.default_rng(seed)
    m0 = m + 1
    us, vs = [], []
    endpoints: list[int] = []
    for a in range(m0):
        for b in range(a + 1, m0):
            us.append(a)
            vs.append(b)
            endpoints += [a, b]
    for v in range(m0, n):
        targets: set[int] = set()
        while len(targets) < m:
            targets.add(endpoints[int(rng.integers(len(endpoints)))])
        for t in sorted(targets):
            us.append(v)
            vs.append(t)
            endpoints += [v, t]
    return csr_from_edges(n, np.array(us), np.array(vs), name=f"BA(n={n},m={m})")


def _inverse_cdf(cdf: np.ndarray, r: np.ndarray, first: np.ndarray, buckets: int) -> np.ndarray:
    """np.searchsorted(cdf, r, side="right") for nondecreasing ``cdf``, by a
    bucket table: ``first[j]`` counts the entries <= j / buckets, so the answer
    for r is at least ``first[j]`` with j / buckets <= r, and is reached by
    stepping forward while cdf[idx] <= r (a few steps per draw)."""
    j = np.floor(r * buckets).astype(np.int64) - 1
    np.clip(j, 0, buckets - 1, out=j)
    idx = first[j]
    active = np.arange(r.size)
    n = cdf.size
    while active.size:
        ia = idx[active]
        step = ia < n
        step[step] = cdf[ia[step]] <= r[active[step]]
        active = active[step]
        idx[active] += 1
    return idx


def chung_lu(n: int, mean_deg: float, gamma: float, seed: int,
             lcc: bool = True, chunk: int = 1 << 24) -> Csr:
    """Chung-Lu power-law graph by weighted endpoint sampling.

    Weights w_i proportional to (i+1)^(-1/(gamma-1)), scaled to mean
    ``mean_deg`` and capped at sqrt(sum w). round(n*mean_deg/2) edges are
    drawn, both endpoints independently with probability proportional to w;
    self-loops and repeated edges are dropped. Node ids are then shuffled so
    that ids carry no degree information, and the largest connected
    component is kept when ``lcc``.
    """
    rng = np.random.default_rng(seed)
    w = np.arange(1, n + 1, dtype=np.float64) ** (-1.0 / (gamma - 1.0))
    w *= mean_deg * n / w.sum()
    w = np.minimum(w, np.sqrt(w.sum()))
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    m = int(round(n * mean_deg / 2.0))
    buckets = 4 * n
    first = np.searchsorted(cdf, np.arange(buckets, dtype=np.float64) / buckets, side="right")
    keys = []
    left = m
    while left > 0:
        c = min(chunk, left)
        a = _inverse_cdf(cdf, rng.random(c), first, buckets)
        b = _inverse_cdf(cdf, rng.random(c), first, buckets)
        np.minimum(a, n - 1, out=a)
        np.minimum(b, n - 1, out=b)
        lo = np.minimum(a, b)
        hi = np.maximum(a, b)
        ok = lo != hi
        keys.append(np.unique(lo[ok].astype(np.int64) * n + hi[ok]))
        left -= c
    key = np.unique(np.concatenate(keys)) if len(keys) > 1 else keys[0]
    u = key // n
    v = key - u * n
    perm = rng.permutation(n).astype(np.int64)
    g = csr_from_edges(n, perm[u], perm[v], name=f"CL(n={n},d={mean_deg},g={gamma})")
    if lcc:
        g = largest_component(g, name=g.name + "/LCC")
    return g


_clgen = None


def _clgen_lib():
    global _clgen
    if _clgen is None:
        import ctypes
        import os

        from synth import build as _sbuild
        if not os.path.exists(_sbuild.LIB):
            _sbuild.build()
        L = ctypes.CDLL(_sbuild.LIB)
        L.clg_generate.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_double, ctypes.c_uint64,
                                   ctypes.c_int, ctypes.c_int]
        L.clg_generate.restype = ctypes.c_void_p
        L.clg_n.argtypes = [ctypes.c_void_p]
        L.clg_n.restype = ctypes.c_int64
        L.clg_nnz.argtypes = [ctypes.c_void_p]
        L.clg_nnz.restype = ctypes.c_int64
        L.clg_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.clg_copy.restype = None
        L.clg_free.argtypes = [ctypes.c_void_p]
        L.clg_free.restype = None
        _clgen = L
    return _clgen


def chung_lu_native(n: int, mean_deg: float, gamma: float, seed: int, lcc: bool = True,
                    threads: int = 16) -> Csr:
    """The Chung-Lu model of ``chung_lu`` from the native generator (synth/clgen.cpp):
    same weights, cap and edge count, a counter-based random stream so that the
    graph does not depend on the thread count, and the canonical CSR built in
    O(nnz) memory. Used for the workload too large for the numpy generator."""
    import ctypes
    import os

    L = _clgen_lib()
    threads = max(1, min(threads, len(os.sched_getaffinity(0))))
    h = L.clg_generate(n, mean_deg, gamma, seed & (2 ** 64 - 1), threads, 1 if lcc else 0)
    if not h:
        raise ValueError("clg_generate: invalid arguments")
    try:
        m = int(L.clg_n(h))
        nnz = int(L.clg_nnz(h))
        rp = np.empty(m + 1, dtype=np.int64)
        col = np.empty(nnz, dtype=np.int32)
        L.clg_copy(h, rp.ctypes.data_as(ctypes.c_void_p), col.ctypes.data_as(ctypes.c_void_p))
    finally:
        L.clg_free(h)
    return Csr(n=m, row_ptr=rp, col=col, name=f"CLn(n={n},d={mean_deg},g={gamma})" + ("/LCC" if lcc else ""))


def grid_minus_edges(side: int, frac: float, seed: int) -> Csr:
    """side x side grid with round(frac * |E|) random edges removed, connected.

    A spanning tree (minimum spanning tree under i.i.d. uniform edge weights)
    is protected; the removed edges are drawn uniformly from the rest.
    """
    rng = np.random.default_rng(seed)
    n = side * side
    idx = np.arange(n, dtype=np.int64).reshape(side, side)
    hu, hv = idx[:, :-1].ravel(), idx[:, 1:].ravel()
    vu, vv = idx[:-1, :].ravel(), idx[1:, :].ravel()
    u = np.concatenate([hu, vu])
    v = np.concatenate([hv, vv])
    e = u.size
    wts = rng.random(e) + 1e-9
    mat = sp.csr_matrix((wts, (u, v)), shape=(n, n))
    tree = csgraph.minimum_spanning_tree(mat).tocoo()
    tkey = np.minimum(tree.row, tree.col).astype(np.int64) * n + np.maximum(tree.row, tree.col)
    ekey = u * n + v
    in_tree = np.isin(ekey, tkey)
    cand = np.flatnonzero(~in_tree)
    nremove = int(round(frac * e))
    drop = rng.choice(cand, size=nremove, replace=False)
    keep = np.ones(e, dtype=bool)
    keep[drop] = False
    return csr_from_edges(n, u[keep], v[keep], name=f"grid({side}x{side})-{frac:g}")


GRAPH_SEED = 0x5EED0000
QUERY_SEED_OFFSET = 0x100
PHILOX_SEED = 0x0B1A5ED5EED
# Philox key of the walk-count calibration runs; no test or benchmark uses it
CALIBRATION_SEED = 0x0CA11B7A7E5E

# The five workload graphs. Key -> (builder, description).
WORKLOADS = {
    "ba1k": (lambda: barabasi_albert(1000, 3, GRAPH_SEED + 0),
             "Barabasi-Albert n=1,000, m=3 (grown from K4)"),
    "cl100k": (lambda: chung_lu(100_000, 10.0, 2.5, GRAPH_SEED + 1),
               "Chung-Lu n=100,000, mean degree 10, exponent 2.5, LCC"),
    "grid1414": (lambda: grid_minus_edges(1414, 0.05, GRAPH_SEED + 2),
                 "1,414 x 1,414 grid, 5% of edges removed, connected"),
    "cl10m": (lambda: chung_lu(10_000_000, 10.0, 2.3, GRAPH_SEED + 3),
              "Chung-Lu n=10,000,000, mean degree 10, exponent 2.3, LCC"),
    "cl40m": (lambda: chung_lu_native(40_000_000, 25.0, 2.2, GRAPH_SEED + 4),
              "Chung-Lu n=40,000,000, mean degree 25, exponent 2.2, LCC (native generator)"),
}

WORKLOAD_INDEX = {"ba1k": 0, "cl100k": 1, "grid1414": 2, "cl10m": 3, "cl40m": 4}

_cache: dict[str, Csr] = {}


def workload_graph(key: str) -> Csr:
    if key not in _cache:
        builder, desc = WORKLOADS[key]
        g = builder()
        g.name = key
        _cache[key] = g
    return _cache[key]
