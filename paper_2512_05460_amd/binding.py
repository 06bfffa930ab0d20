"""ctypes binding of ``include/probewalk.h``: argument marshalling only.

Every function here has the name of the C entry point it calls and does
nothing but convert numpy arrays / torch streams into pointers and back; all
of the estimator runs in the HIP library. Streams come from PyTorch
(``torch.cuda.current_stream()`` by default).

The library must have been built (``python -m paper_2512_05460_amd.build``);
there is no fallback of any kind when it is missing.

PyTorch ships its own HIP runtime under the same SONAME as the system one.
``lib()`` imports torch before loading ``libprobewalk.so`` so that the
library binds to the runtime torch already loaded: one HIP runtime per
process, in which torch's streams and our calls live together.

Device memory: ``lib()`` installs PyTorch's caching allocator as the library's
allocator (``bd_set_allocator``), so graph tables, work buffers and server
arenas come from torch's pool and show in ``torch.cuda.memory_allocated()``.
``use_torch_allocator(False)`` switches back to the library's own hipMalloc for
buffers allocated afterwards. Objects still alive at interpreter exit are freed
by an exit hook while torch is still usable.
"""

from __future__ import annotations

import atexit
import ctypes
import os
import weakref

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libprobewalk.so")

BD_OK = 0
BD_E_INVALID = -1
BD_E_GRAPH = -2
BD_E_RANGE = -3
BD_E_BUDGET = -4
BD_E_HIP = -5
BD_E_NOMEM = -6
BD_E_NODEVICE = -7
BD_E_NOTFOUND = -8
BD_E_FULL = -9
BD_E_CANCELLED = -10
BD_E_TIMEOUT = -11
BD_E_SCRATCH = -12
NOALLOC_SCRATCH_BYTES = 64 << 20

BD_LAYOUT_CSR = 0
BD_LAYOUT_FAT = 1
BD_SKIP_VALIDATION = 2
BD_RELABEL_DEGREE = 4
BD_LAYOUT_COMPACT = 8
BD_WIDE_IDS = 16
BD_LAYOUT_AUTO = 32
BD_DEVICE_PTRS = 64
BD_PROBE_STORAGE_IDS = 128
BD_NONTEMPORAL = 256
BD_TEMPORAL = 512
BD_NARROW_HUBS = 1024
BD_DIRECT_HUBS = 2048
BD_WIDE_HUBS = 4096

BD_POLICY_PAPER = 0
BD_POLICY_SCALED = 1
BD_POLICY_FIXED = 2

BD_MODE_PLAIN = 0
BD_MODE_BATCHED = 1

# Symbols declared in include/probewalk.h.
EXPORTS = ("graph_load_csr", "graph_free", "bd_graph_get_info", "bd_plan", "bd_query_batch",
           "bd_walk_trace", "bd_probe_eval", "bd_query_probes", "bd_server_create",
           "bd_server_submit", "bd_server_poll", "bd_server_wait", "bd_server_destroy",
           "bd_strerror", "bd_device_info", "bd_gather_roofline", "bd_autotune",
           "bd_query_stabilized", "bd_truncated_beta", "bd_graph_lambda", "bd_theorem_L",
           "bd_query_batch_noalloc", "bd_set_allocator", "bd_server_cancel")


class BdPolicy(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("c_B", ctypes.c_double), ("c_R", ctypes.c_double),
                ("delta", ctypes.c_double), ("B_fixed", ctypes.c_int64), ("R_fixed", ctypes.c_int64),
                ("max_steps_per_query", ctypes.c_uint64), ("share", ctypes.c_int32)]


class BdExec(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_uint32), ("chunk_probes", ctypes.c_int32),
                ("grid_wgs", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("chunk_pairs", ctypes.c_int32), ("queues", ctypes.c_int32),
                ("uniform_min_r", ctypes.c_int32), ("deadline_ms", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class BdStats(ctypes.Structure):
    _fields_ = [("walk_kernel_ms", ctypes.c_double), ("total_ms", ctypes.c_double),
                ("launches", ctypes.c_int64), ("chunks", ctypes.c_int64),
                ("walk_steps", ctypes.c_int64), ("walk_pairs", ctypes.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class BdGraphInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("d_min", ctypes.c_int32),
                ("d_max", ctypes.c_int32), ("bipartite", ctypes.c_int32), ("layout", ctypes.c_int32),
                ("device_bytes", ctypes.c_int64), ("nontemporal", ctypes.c_int32), ("lds_hubs", ctypes.c_int32)]


class BdRoofline(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double), ("steps_per_s", ctypes.c_double),
                ("gathers_per_s", ctypes.c_double), ("steps", ctypes.c_int64),
                ("chains_per_lane", ctypes.c_int32), ("work_groups", ctypes.c_int32)]


class BdServerCfg(ctypes.Structure):
    _fields_ = [("policy", BdPolicy), ("max_queries_inflight", ctypes.c_int64),
                ("max_steps_inflight", ctypes.c_uint64), ("chunk_probes", ctypes.c_int32),
                ("slice_ms", ctypes.c_double), ("small_first", ctypes.c_double)]


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)


class BdAllocator(ctypes.Structure):
    _fields_ = [("ctx", ctypes.c_void_p), ("alloc", _ALLOC_FN), ("free", _FREE_FN)]


RESULT_DTYPE = np.dtype([("beta", "f8"), ("K", "i8"), ("R", "i8"), ("B", "i4"), ("G", "i4"),
                         ("L", "i4"), ("status", "i4"), ("walk_steps", "i8")], align=True)
assert RESULT_DTYPE.itemsize == 48

_lib = None
_P = ctypes.c_void_p


class ProbeWalkError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {strerror(code)} ({code})")


def lib():
    """Load libprobewalk.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2512_05460_amd.build`")
        import torch  # noqa: F401  (bind to the HIP runtime torch loads)

        L = ctypes.CDLL(LIB_PATH)
        i32, i64, u32, u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64
        sig = {
            "graph_load_csr": (ctypes.c_int, [i64, _P, _P, u32, _P, ctypes.POINTER(_P)]),
            "graph_free": (None, [_P]),
            "bd_graph_get_info": (ctypes.c_int, [_P, ctypes.POINTER(BdGraphInfo)]),
            "bd_plan": (ctypes.c_int, [_P, i64, _P, _P, _P, _P, ctypes.POINTER(BdPolicy), _P]),
            "bd_query_batch": (ctypes.c_int, [_P, i64, _P, _P, _P, _P, _P, u64, ctypes.POINTER(BdPolicy),
                                              ctypes.POINTER(BdExec), _P, _P, ctypes.POINTER(BdStats)]),
            "bd_query_batch_noalloc": (ctypes.c_int, [_P, i64, _P, _P, _P, _P, _P, u64, ctypes.POINTER(BdPolicy),
                                                      ctypes.POINTER(BdExec), _P, _P, ctypes.POINTER(BdStats)]),
            "bd_walk_trace": (ctypes.c_int, [_P, i64, _P, _P, _P, _P, _P, i32, u64, _P, _P, _P]),
            "bd_probe_eval": (ctypes.c_int, [_P, u64, u32, u32, i64, _P, _P, _P, _P]),
            "bd_query_probes": (ctypes.c_int, [_P, i32, i32, ctypes.c_double, i32, u32, u64,
                                               ctypes.POINTER(BdPolicy), ctypes.POINTER(BdExec), _P,
                                               _P, _P, _P]),
            "bd_server_create": (ctypes.c_int, [_P, ctypes.POINTER(BdServerCfg), ctypes.POINTER(_P)]),
            "bd_server_submit": (ctypes.c_int, [_P, i64, _P, _P, _P, _P, _P, u64, ctypes.POINTER(u64)]),
            "bd_server_poll": (ctypes.c_int, [_P, u64, _P, ctypes.POINTER(ctypes.c_int),
                                              ctypes.POINTER(ctypes.c_double)]),
            "bd_server_wait": (ctypes.c_int, [_P, u64, ctypes.c_double, _P, ctypes.POINTER(ctypes.c_double)]),
            "bd_server_destroy": (None, [_P]),
            "bd_server_cancel": (ctypes.c_int, [_P, u64]),
            "bd_strerror": (ctypes.c_char_p, [ctypes.c_int]),
            "bd_device_info": (ctypes.c_int, [ctypes.c_char_p, ctypes.c_size_t]),
            "bd_gather_roofline": (ctypes.c_int, [_P, i32, i32, i32, _P, ctypes.POINTER(BdRoofline)]),
            "bd_truncated_beta": (ctypes.c_int, [_P, i64, _P, _P, i32, _P, _P]),
            "bd_graph_lambda": (ctypes.c_int, [_P, i32, u64, _P, ctypes.POINTER(ctypes.c_double)]),
            "bd_theorem_L": (ctypes.c_int, [_P, i64, _P, _P, _P, ctypes.c_double, _P]),
            "bd_query_stabilized": (ctypes.c_int, [_P, i64, _P, _P, _P, i32, _P, u64, ctypes.POINTER(BdPolicy),
                                                   ctypes.POINTER(BdExec), _P, _P, _P]),
            "bd_autotune": (ctypes.c_int, [_P, i64, _P, _P, _P, _P, u64, ctypes.POINTER(BdPolicy), u32, _P,
                                           ctypes.POINTER(BdExec), _P, ctypes.POINTER(i32)]),
        }
        sig["bd_set_allocator"] = (ctypes.c_int, [ctypes.POINTER(BdAllocator)])
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
        use_torch_allocator(True)
        # registered after torch's import, so it runs before torch's own exit hooks
        atexit.register(_free_live_objects)
    return _lib


# --- device memory from PyTorch's caching allocator ------------------------------
def _torch_alloc(ctx, nbytes, stream):
    import torch
    try:
        return torch.cuda.caching_allocator_alloc(int(nbytes), device=torch.cuda.current_device(),
                                                  stream=stream if stream else None)
    except Exception:  # reported to the library as a failed allocation (BD_E_NOMEM)
        return None


def _torch_free(ctx, ptr, nbytes, stream):
    import torch
    torch.cuda.caching_allocator_delete(ptr)


_TORCH_ALLOCATOR = BdAllocator(None, _ALLOC_FN(_torch_alloc), _FREE_FN(_torch_free))
_live = weakref.WeakSet()  # graphs and servers, freed at exit while torch still works
_torch_alloc_on = False


def use_torch_allocator(enable: bool = True):
    """Take the library's device buffers allocated from now on from PyTorch's
    caching allocator (True) or from the library's own hipMalloc (False)."""
    global _torch_alloc_on
    L = _lib if _lib is not None else lib()
    _check(L.bd_set_allocator(ctypes.byref(_TORCH_ALLOCATOR) if enable else None), "bd_set_allocator")
    _torch_alloc_on = enable


def _free_live_objects():
    for obj in [o for o in list(_live) if isinstance(o, Server)] + [o for o in list(_live) if isinstance(o, Graph)]:
        try:
            obj.free() if isinstance(obj, Graph) else obj.destroy()
        except Exception:
            pass


def strerror(code: int) -> str:
    return lib().bd_strerror(code).decode()


def _check(rc: int, where: str):
    if rc != BD_OK:
        raise ProbeWalkError(rc, where)


def _arr(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_P)


def _stream(stream):
    """hipStream_t handle: an int, a torch stream, or torch's current stream."""
    if stream is None:
        import torch
        if torch.cuda.is_available():
            return torch.cuda.current_stream().cuda_stream
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def policy(kind="paper", c_B=448.0, c_R=128.0, delta=0.01, B=0, R=0, max_steps=0, share=1) -> BdPolicy:
    k = {"paper": BD_POLICY_PAPER, "scaled": BD_POLICY_SCALED, "fixed": BD_POLICY_FIXED}[kind]
    return BdPolicy(k, c_B, c_R, delta, B, R, max_steps, share)


def exec_cfg(mode="batched", chunk_probes=0, grid_wgs=0, use_graph=False, chunk_pairs=0, queues=0,
             uniform_min_r=0, deadline_ms=0.0) -> BdExec:
    m = {"plain": BD_MODE_PLAIN, "batched": BD_MODE_BATCHED}[mode]
    return BdExec(m, chunk_probes, grid_wgs, 1 if use_graph else 0, chunk_pairs, queues, uniform_min_r,
                  deadline_ms)


class Graph:
    """Owning wrapper of a ``bd_graph*`` handle."""

    def __init__(self, handle):
        self._h = handle
        _live.add(self)

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("graph was freed")
        return self._h

    def info(self) -> dict:
        return bd_graph_get_info(self)

    def free(self):
        if self._h is not None:
            lib().graph_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def graph_load_csr(n: int, row_ptr, col_idx, flags: int = BD_LAYOUT_CSR, stream=None) -> Graph:
    rp = _arr(row_ptr, np.int64)
    col = _arr(col_idx, np.int32)
    if rp.size != n + 1:
        raise ValueError("row_ptr must have n+1 entries")
    h = _P()
    _check(lib().graph_load_csr(n, _ptr(rp), _ptr(col), flags, _stream(stream), ctypes.byref(h)),
           "graph_load_csr")
    return Graph(h)


def graph_load_csr_device(n: int, row_ptr, col_idx, flags: int = BD_LAYOUT_CSR, stream=None) -> Graph:
    """graph_load_csr with BD_DEVICE_PTRS: row_ptr (int64, n+1) and col_idx
    (int32) are torch tensors on the current device."""
    import torch
    if row_ptr.dtype != torch.int64 or col_idx.dtype != torch.int32:
        raise TypeError("row_ptr must be int64 and col_idx int32")
    if not (row_ptr.is_cuda and col_idx.is_cuda):
        raise ValueError("row_ptr and col_idx must be device tensors")
    rp, col = row_ptr.contiguous(), col_idx.contiguous()
    if rp.numel() != n + 1:
        raise ValueError("row_ptr must have n+1 entries")
    h = _P()
    _check(lib().graph_load_csr(n, rp.data_ptr(), col.data_ptr(), flags | BD_DEVICE_PTRS, _stream(stream),
                                ctypes.byref(h)), "graph_load_csr")
    return Graph(h)


def graph_free(g: Graph):
    g.free()


def bd_graph_get_info(g: Graph) -> dict:
    info = BdGraphInfo()
    _check(lib().bd_graph_get_info(g.handle, ctypes.byref(info)), "bd_graph_get_info")
    return {f: getattr(info, f) for f, _ in info._fields_}


def bd_plan(g: Graph, s, t, eps, L, pol: BdPolicy | None = None) -> np.ndarray:
    s, t = _arr(s, np.int32), _arr(t, np.int32)
    eps = _arr(np.broadcast_to(eps, s.shape), np.float64)
    L = _arr(np.broadcast_to(L, s.shape), np.int32)
    out = np.zeros(s.size, dtype=RESULT_DTYPE)
    _check(lib().bd_plan(g.handle, s.size, _ptr(s), _ptr(t), _ptr(eps), _ptr(L),
                         None if pol is None else ctypes.byref(pol), _ptr(out)), "bd_plan")
    return out


def bd_query_batch(g: Graph, s, t, eps, L, seed: int, pol: BdPolicy | None = None,
                   ex: BdExec | None = None, uid=None, stream=None, with_stats: bool = False):
    s, t = _arr(s, np.int32), _arr(t, np.int32)
    eps = _arr(np.broadcast_to(eps, s.shape), np.float64)
    L = _arr(np.broadcast_to(L, s.shape), np.int32)
    u = None if uid is None else _arr(uid, np.uint32)
    out = np.zeros(s.size, dtype=RESULT_DTYPE)
    st = BdStats()
    _check(lib().bd_query_batch(g.handle, s.size, _ptr(s), _ptr(t), _ptr(eps), _ptr(L), _ptr(u),
                                seed & (2 ** 64 - 1), None if pol is None else ctypes.byref(pol),
                                None if ex is None else ctypes.byref(ex), _stream(stream), _ptr(out),
                                ctypes.byref(st)), "bd_query_batch")
    return (out, st.as_dict()) if with_stats else out


def bd_query_batch_noalloc(g: Graph, s, t, eps, L, seed: int, pol: BdPolicy | None = None,
                           ex: BdExec | None = None, uid=None, stream=None, with_stats: bool = False):
    """bd_query_batch with the library's fixed scratch array (no device allocation)."""
    s, t = _arr(s, np.int32), _arr(t, np.int32)
    eps = _arr(np.broadcast_to(eps, s.shape), np.float64)
    L = _arr(np.broadcast_to(L, s.shape), np.int32)
    u = None if uid is None else _arr(uid, np.uint32)
    out = np.zeros(s.size, dtype=RESULT_DTYPE)
    st = BdStats()
    _check(lib().bd_query_batch_noalloc(g.handle, s.size, _ptr(s), _ptr(t), _ptr(eps), _ptr(L), _ptr(u),
                                        seed & (2 ** 64 - 1), None if pol is None else ctypes.byref(pol),
                                        None if ex is None else ctypes.byref(ex), _stream(stream), _ptr(out),
                                        ctypes.byref(st)), "bd_query_batch_noalloc")
    return (out, st.as_dict()) if with_stats else out


def bd_query_probes(g: Graph, s: int, t: int, eps: float, L: int, uid: int, seed: int,
                    pol: BdPolicy | None = None, ex: BdExec | None = None, stream=None):
    """Returns (result, Q per probe, block means)."""
    plan = bd_plan(g, [s], [t], [eps], [L], pol)[0]
    if plan["status"] != BD_OK:
        raise ProbeWalkError(int(plan["status"]), "bd_query_probes")
    q = np.zeros(int(plan["K"]), dtype=np.float64)
    y = np.zeros(int(plan["G"]), dtype=np.float64)
    out = np.zeros(1, dtype=RESULT_DTYPE)
    _check(lib().bd_query_probes(g.handle, s, t, eps, L, uid, seed & (2 ** 64 - 1),
                                 None if pol is None else ctypes.byref(pol),
                                 None if ex is None else ctypes.byref(ex), _stream(stream),
                                 _ptr(q), _ptr(y), _ptr(out)), "bd_query_probes")
    return out[0], q, y


def bd_walk_trace(g: Graph, start, uid, k, p, side, L: int, seed: int, stream=None):
    start = _arr(start, np.int32)
    n = start.size
    uid = _arr(np.broadcast_to(uid, (n,)), np.uint32)
    k = _arr(np.broadcast_to(k, (n,)), np.uint32)
    p = _arr(np.broadcast_to(p, (n,)), np.uint32)
    side = _arr(np.broadcast_to(side, (n,)), np.uint32)
    trace = np.zeros((n, L + 1), dtype=np.int32)
    acc = np.zeros(n, dtype=np.float32)
    _check(lib().bd_walk_trace(g.handle, n, _ptr(start), _ptr(uid), _ptr(k), _ptr(p), _ptr(side), L,
                               seed & (2 ** 64 - 1), _stream(stream), _ptr(trace), _ptr(acc)),
           "bd_walk_trace")
    return trace, acc


def bd_probe_eval(g: Graph, seed: int, uid: int, k: int, nodes, stream=None):
    nodes = _arr(nodes, np.uint32)
    pi = np.zeros(nodes.size, dtype=np.uint32)
    z = np.zeros(nodes.size, dtype=np.int8)
    _check(lib().bd_probe_eval(g.handle, seed & (2 ** 64 - 1), uid, k, nodes.size, _ptr(nodes),
                               _stream(stream), _ptr(pi), _ptr(z)), "bd_probe_eval")
    return pi, z


class Server:
    """Owning wrapper of a ``bd_server*`` (served mode, continuous batching)."""

    def __init__(self, g: Graph, pol: BdPolicy, max_queries: int = 0, max_steps: int = 0,
                 chunk_probes: int = 0, slice_ms: float = 0.0, small_first: float = 0.0):
        self.graph = g  # the graph must outlive the server
        cfg = BdServerCfg(pol, max_queries, max_steps, chunk_probes, slice_ms, small_first)
        h = _P()
        _check(lib().bd_server_create(g.handle, ctypes.byref(cfg), ctypes.byref(h)), "bd_server_create")
        self._h = h
        self._sizes = {}
        _live.add(self)

    def submit(self, s, t, eps, L, seed: int, uid=None) -> int:
        s, t = _arr(s, np.int32), _arr(t, np.int32)
        eps = _arr(np.broadcast_to(eps, s.shape), np.float64)
        L = _arr(np.broadcast_to(L, s.shape), np.int32)
        u = None if uid is None else _arr(uid, np.uint32)
        rid = ctypes.c_uint64()
        _check(lib().bd_server_submit(self._h, s.size, _ptr(s), _ptr(t), _ptr(eps), _ptr(L), _ptr(u),
                                      seed & (2 ** 64 - 1), ctypes.byref(rid)), "bd_server_submit")
        self._sizes[rid.value] = s.size
        return rid.value

    def poll(self, rid: int):
        """(done, results or None, latency_ms or None)."""
        out = np.zeros(self._sizes[rid], dtype=RESULT_DTYPE)
        done = ctypes.c_int()
        lat = ctypes.c_double()
        _check(lib().bd_server_poll(self._h, rid, _ptr(out), ctypes.byref(done), ctypes.byref(lat)),
               "bd_server_poll")
        if done.value:
            del self._sizes[rid]
            return True, out, lat.value
        return False, None, None

    def wait(self, rid: int, timeout_ms: float = 0.0):
        out = np.zeros(self._sizes[rid], dtype=RESULT_DTYPE)
        lat = ctypes.c_double()
        _check(lib().bd_server_wait(self._h, rid, timeout_ms, _ptr(out), ctypes.byref(lat)),
               "bd_server_wait")
        del self._sizes[rid]
        return out, lat.value

    def cancel(self, rid: int):
        """bd_server_cancel: collect the request with poll/wait afterwards."""
        _check(lib().bd_server_cancel(self._h, rid), "bd_server_cancel")

    def destroy(self):
        if self._h is not None:
            lib().bd_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def bd_server_create(g: Graph, pol: BdPolicy, **kw) -> Server:
    return Server(g, pol, **kw)


def bd_device_info() -> str:
    buf = ctypes.create_string_buffer(512)
    rc = lib().bd_device_info(buf, 512)
    _check(rc, "bd_device_info")
    return buf.value.decode()


def bd_gather_roofline(g: Graph, chains_per_lane: int = 4, steps: int = 2000, work_groups: int = 0,
                       stream=None) -> dict:
    r = BdRoofline()
    _check(lib().bd_gather_roofline(g.handle, chains_per_lane, steps, work_groups, _stream(stream),
                                    ctypes.byref(r)), "bd_gather_roofline")
    return {f: getattr(r, f) for f, _ in r._fields_}


def bd_autotune(g: Graph, s, t, eps, L, seed: int, pol: BdPolicy | None = None, mode: str = "batched",
                stream=None):
    """Returns (best BdExec, kernel ms per candidate)."""
    s, t = _arr(s, np.int32), _arr(t, np.int32)
    eps = _arr(np.broadcast_to(eps, s.shape), np.float64)
    L = _arr(np.broadcast_to(L, s.shape), np.int32)
    best = BdExec()
    times = np.zeros(16, dtype=np.float64)
    n = ctypes.c_int32()
    m = {"plain": BD_MODE_PLAIN, "batched": BD_MODE_BATCHED}[mode]
    _check(lib().bd_autotune(g.handle, s.size, _ptr(s), _ptr(t), _ptr(eps), _ptr(L), seed & (2 ** 64 - 1),
                             None if pol is None else ctypes.byref(pol), m, _stream(stream), ctypes.byref(best),
                             _ptr(times), ctypes.byref(n)), "bd_autotune")
    return best, times[:n.value]


def bd_query_stabilized(g: Graph, s, t, eps, L_max: int, seed: int, pol: BdPolicy | None = None,
                        ex: BdExec | None = None, uid=None, stream=None):
    """Returns (results, L_stop) -- the stabilization rule of section 4.3."""
    s, t = _arr(s, np.int32), _arr(t, np.int32)
    eps = _arr(np.broadcast_to(eps, s.shape), np.float64)
    u = None if uid is None else _arr(uid, np.uint32)
    out = np.zeros(s.size, dtype=RESULT_DTYPE)
    Ls = np.zeros(s.size, dtype=np.int32)
    _check(lib().bd_query_stabilized(g.handle, s.size, _ptr(s), _ptr(t), _ptr(eps), L_max, _ptr(u),
                                     seed & (2 ** 64 - 1), None if pol is None else ctypes.byref(pol),
                                     None if ex is None else ctypes.byref(ex), _stream(stream), _ptr(out),
                                     _ptr(Ls)), "bd_query_stabilized")
    return out, Ls


def bd_truncated_beta(g: Graph, s, t, L: int, stream=None) -> np.ndarray:
    s, t = _arr(s, np.int32), _arr(t, np.int32)
    out = np.zeros(s.size, dtype=np.float64)
    _check(lib().bd_truncated_beta(g.handle, s.size, _ptr(s), _ptr(t), L, _stream(stream), _ptr(out)),
           "bd_truncated_beta")
    return out


def bd_graph_lambda(g: Graph, iters: int = 500, seed: int = 1, stream=None) -> float:
    lam = ctypes.c_double()
    _check(lib().bd_graph_lambda(g.handle, iters, seed, _stream(stream), ctypes.byref(lam)), "bd_graph_lambda")
    return lam.value


def bd_theorem_L(g: Graph, s, t, eps, lam: float) -> np.ndarray:
    s, t = _arr(s, np.int32), _arr(t, np.int32)
    eps = _arr(np.broadcast_to(eps, s.shape), np.float64)
    out = np.zeros(s.size, dtype=np.int32)
    _check(lib().bd_theorem_L(g.handle, s.size, _ptr(s), _ptr(t), _ptr(eps), lam, _ptr(out)), "bd_theorem_L")
    return out
