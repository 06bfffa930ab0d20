"""Device memory through PyTorch (the boundary's ownership model):

  * with PyTorch's caching allocator installed (the binding's default) the
    graph tables and work buffers come from torch's pool: torch's allocated
    bytes grow by at least the graph's device bytes at load and return to where
    they were after graph_free;
  * a CSR held in torch tensors on the device loads through the C ABI
    (BD_DEVICE_PTRS) and gives the oracle's estimates bit for bit, in every
    layout; host arrays passed with the flag are refused;
  * switching back to the library's own allocation gives the same bits.
"""

import ctypes

import numpy as np
import pytest
import torch

from oracle import estimator as E
from oracle import planner as OP
from paper_2512_05460_amd import binding as B
from synth import graphs, queries

pytestmark = pytest.mark.gpu

SEED = graphs.PHILOX_SEED
LAYOUTS = [B.BD_LAYOUT_CSR, B.BD_LAYOUT_FAT | B.BD_RELABEL_DEGREE, B.BD_LAYOUT_COMPACT,
           B.BD_LAYOUT_COMPACT | B.BD_RELABEL_DEGREE, B.BD_LAYOUT_COMPACT | B.BD_RELABEL_DEGREE | B.BD_WIDE_IDS,
           B.BD_LAYOUT_COMPACT | B.BD_RELABEL_DEGREE | B.BD_PROBE_STORAGE_IDS]


def _oracle(g, s, t, L, b, r):
    plans = [OP.plan(0.1, L, 1, 1, 1, OP.Policy("fixed", B_fixed=b, R_fixed=r))] * len(s)
    return E.estimate(g, s, t, L, plans, SEED, threads=8)


@pytest.mark.parametrize("flags", LAYOUTS)
def test_device_csr_through_torch_memory(flags):
    B.use_torch_allocator(True)
    g = graphs.workload_graph("ba1k")
    rp = torch.from_numpy(g.row_ptr.astype(np.int64)).cuda()
    col = torch.from_numpy(g.col.astype(np.int32)).cuda()
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    dg = B.graph_load_csr_device(g.n, rp, col, flags)
    info = dg.info()
    assert torch.cuda.memory_allocated() - before >= info["device_bytes"]
    s, t = queries.uniform_pairs(g.n, 12, 99)
    pol = B.policy("fixed", B=2, R=80)
    res = B.bd_query_batch(dg, s, t, 0.1, 30, SEED, pol)
    assert np.all(res["status"] == 0)
    if flags & B.BD_PROBE_STORAGE_IDS:  # Algorithm 1 on the graph in storage order
        gs, _, internal = graphs.storage_order(g)
        assert np.array_equal(res["beta"], _oracle(gs, internal[s], internal[t], 30, 2, 80))
    else:
        assert np.array_equal(res["beta"], _oracle(g, s, t, 30, 2, 80))
    dg.free()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == before


def test_host_arrays_with_device_flag_are_refused():
    g = graphs.workload_graph("ba1k")
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(g.col, dtype=np.int32)
    h = ctypes.c_void_p()
    rc = B.lib().graph_load_csr(g.n, rp.ctypes.data_as(ctypes.c_void_p), col.ctypes.data_as(ctypes.c_void_p),
                                B.BD_DEVICE_PTRS, None, ctypes.byref(h))
    assert rc == B.BD_E_INVALID


def test_library_allocation_gives_the_same_bits():
    g = graphs.workload_graph("cl100k")
    s, t = queries.uniform_pairs(g.n, 6, 5)
    pol = B.policy("fixed", B=1, R=5000)  # split probes in batched mode: accumulators in the workspace
    out = []
    for torch_mem in (True, False):
        B.use_torch_allocator(torch_mem)
        try:
            dg = B.graph_load_csr(g.n, g.row_ptr, g.col, B.BD_LAYOUT_AUTO)
            out.append(B.bd_query_batch(dg, s, t, 0.1, 20, SEED, pol)["beta"])
            srv = B.Server(dg, pol)
            o, _ = srv.wait(srv.submit(s, t, 0.1, 20, SEED))
            srv.destroy()
            assert np.array_equal(o["beta"], out[-1])
            dg.free()
        finally:
            B.use_torch_allocator(True)
    assert np.array_equal(out[0], out[1])
