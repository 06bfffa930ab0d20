"""The C ABI library loads and exports what include/probewalk.h declares, and its
host-side graph checks reject bad input before any device work (CPU only)."""

import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2512_05460_amd import binding
from synth import graphs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "probewalk.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return set(re.findall(r"^\s*(?:int|void|const char\*)\s+\**(\w+)\s*\(", text, flags=re.M))


def test_header_symbols_exported():
    names = _declared()
    assert "graph_load_csr" in names and "bd_query_batch" in names
    lib = ctypes.CDLL(binding.LIB_PATH)
    for name in names:
        assert hasattr(lib, name), name
    assert names == set(binding.EXPORTS)


def test_strerror():
    assert binding.strerror(0) == "ok"
    assert "graph" in binding.strerror(binding.BD_E_GRAPH)
    assert binding.strerror(12345) == "unknown error"


def _load(n, rp, col):
    h = ctypes.c_void_p()
    rp = np.ascontiguousarray(rp, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    return binding.lib().graph_load_csr(n, rp.ctypes.data_as(ctypes.c_void_p),
                                        col.ctypes.data_as(ctypes.c_void_p), 0, None, ctypes.byref(h))


def test_graph_checks_reject_bad_input():
    # asymmetric: 0->1 without 1->0
    assert _load(3, [0, 2, 3, 4], [1, 2, 2, 0]) == binding.BD_E_GRAPH
    # self-loop
    assert _load(2, [0, 2, 3], [0, 1, 0]) == binding.BD_E_GRAPH
    # unsorted row
    g = graphs.complete_graph(4)
    col = g.col.copy()
    col[0], col[1] = col[1], col[0]
    assert _load(4, g.row_ptr, col) == binding.BD_E_GRAPH
    # duplicate edge
    assert _load(2, [0, 2, 4], [1, 1, 0, 0]) == binding.BD_E_GRAPH
    # disconnected: two separate edges
    assert _load(4, [0, 1, 2, 3, 4], [1, 0, 3, 2]) == binding.BD_E_GRAPH
    # isolated node
    assert _load(3, [0, 1, 2, 2], [1, 0]) == binding.BD_E_GRAPH
    # out-of-range id
    assert _load(2, [0, 1, 2], [5, 0]) == binding.BD_E_GRAPH
    # sizes
    assert _load(1, [0, 0], []) == binding.BD_E_RANGE
    # the compact layouts exclude the fat layout; the automatic choice excludes both
    g = graphs.complete_graph(4)
    h = ctypes.c_void_p()
    for bad in (binding.BD_LAYOUT_COMPACT | binding.BD_LAYOUT_FAT,
                binding.BD_LAYOUT_COMPACT | binding.BD_LAYOUT_FAT | binding.BD_RELABEL_DEGREE,
                binding.BD_LAYOUT_AUTO | binding.BD_LAYOUT_FAT, binding.BD_LAYOUT_AUTO | binding.BD_LAYOUT_COMPACT,
                binding.BD_LAYOUT_AUTO | binding.BD_WIDE_IDS):
        rc = binding.lib().graph_load_csr(4, g.row_ptr.ctypes.data_as(ctypes.c_void_p),
                                          g.col.ctypes.data_as(ctypes.c_void_p), bad, None, ctypes.byref(h))
        assert rc == binding.BD_E_INVALID


def test_result_layout_matches_header(tmp_path):
    # the ctypes mirrors against the C header as a C compiler lays it out
    src = tmp_path / "sizes.c"
    src.write_text('#include <stdio.h>\n#include "probewalk.h"\n'
                   'int main(void) { printf("%zu %zu %zu %zu %zu %zu %zu\\n", sizeof(bd_result), '
                   'sizeof(bd_policy), sizeof(bd_exec), sizeof(bd_stats), sizeof(bd_server_cfg), '
                   'sizeof(bd_graph_info), sizeof(bd_roofline)); return 0; }\n')
    exe = tmp_path / "sizes"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    sizes = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True,
                                            check=True).stdout.split()]
    assert sizes == [binding.RESULT_DTYPE.itemsize, ctypes.sizeof(binding.BdPolicy),
                     ctypes.sizeof(binding.BdExec), ctypes.sizeof(binding.BdStats),
                     ctypes.sizeof(binding.BdServerCfg), ctypes.sizeof(binding.BdGraphInfo),
                     ctypes.sizeof(binding.BdRoofline)]
    assert ctypes.sizeof(binding.BdExec) == 40
    assert ctypes.sizeof(binding.BdAllocator) == 3 * ctypes.sizeof(ctypes.c_void_p)


def test_binding_has_no_fallback(monkeypatch, tmp_path):
    monkeypatch.setattr(binding, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(binding, "_lib", None)
    with pytest.raises(ImportError):
        binding.lib()


def test_storage_probe_flag_combinations():
    # BD_PROBE_STORAGE_IDS needs BD_LAYOUT_COMPACT | BD_RELABEL_DEGREE and takes
    # neither BD_WIDE_IDS nor BD_LAYOUT_AUTO; checked before any device work
    g = graphs.workload_graph("ba1k")
    full = binding.BD_LAYOUT_COMPACT | binding.BD_RELABEL_DEGREE | binding.BD_PROBE_STORAGE_IDS
    for bad in (binding.BD_PROBE_STORAGE_IDS, binding.BD_PROBE_STORAGE_IDS | binding.BD_LAYOUT_COMPACT,
                full | binding.BD_WIDE_IDS, binding.BD_PROBE_STORAGE_IDS | binding.BD_LAYOUT_AUTO,
                binding.BD_PROBE_STORAGE_IDS | binding.BD_LAYOUT_FAT | binding.BD_RELABEL_DEGREE,
                binding.BD_LAYOUT_COMPACT | binding.BD_RELABEL_DEGREE | binding.BD_DIRECT_HUBS,
                binding.BD_LAYOUT_COMPACT | binding.BD_RELABEL_DEGREE | binding.BD_NARROW_HUBS,
                binding.BD_LAYOUT_COMPACT | binding.BD_RELABEL_DEGREE | binding.BD_WIDE_HUBS,
                full | binding.BD_WIDE_HUBS | binding.BD_NARROW_HUBS):
        h = ctypes.c_void_p()
        rc = binding.lib().graph_load_csr(g.n, g.row_ptr.ctypes.data_as(ctypes.c_void_p),
                                          g.col.ctypes.data_as(ctypes.c_void_p), bad, None, ctypes.byref(h))
        assert rc == binding.BD_E_INVALID, bad
