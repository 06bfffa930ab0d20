"""ctypes driver for the C oracle (``pw_oracle.c``).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

_lib = None

_P = ctypes.c_void_p


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        L.pwo_philox.argtypes = [_P, _P, _P]
        L.pwo_philox.restype = None
        L.pwo_probe_eval.argtypes = [ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint32,
                                     ctypes.c_uint32, ctypes.c_int64, _P, _P, _P, _P]
        L.pwo_probe_eval.restype = None
        L.pwo_walk_trace.argtypes = [ctypes.c_uint32, _P, _P, ctypes.c_uint32, ctypes.c_int32,
                                     ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                     ctypes.c_uint32, ctypes.c_uint32, _P, _P]
        L.pwo_walk_trace.restype = None
        L.pwo_estimate.argtypes = [ctypes.c_uint32, _P, _P, ctypes.c_int64, _P, _P, _P, _P,
                                   _P, _P, _P, _P, _P, _P, ctypes.c_uint64, ctypes.c_int,
                                   _P, _P, _P]
        L.pwo_estimate.restype = ctypes.c_int
        L.pwo_replicas.argtypes = [ctypes.c_uint32, _P, _P, ctypes.c_int32, ctypes.c_int32,
                                   ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint32,
                                   ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64, _P]
        L.pwo_replicas.restype = None
        L.pwo_q_from_u.argtypes = [ctypes.c_int64, _P]
        L.pwo_q_from_u.restype = ctypes.c_double
        L.pwo_probe_q.argtypes = [ctypes.c_uint32, _P, _P, ctypes.c_int32, ctypes.c_int32,
                                  ctypes.c_int32, ctypes.c_uint32, ctypes.c_int64, ctypes.c_int64,
                                  ctypes.c_int64, ctypes.c_uint64, ctypes.c_int64, _P, ctypes.c_int, _P]
        L.pwo_probe_q.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def philox(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().pwo_philox(_ptr(c), _ptr(k), _ptr(out))
    return out


def probe(n: int, seed: int, uid: int, k: int, nodes=None):
    """Return (pi_k(nodes), z^(k)(nodes), params[K0..K5, a, b, r])."""
    if nodes is None:
        nodes = np.arange(n, dtype=np.uint32)
    nodes = np.ascontiguousarray(nodes, dtype=np.uint32)
    pi = np.zeros(nodes.size, dtype=np.uint32)
    z = np.zeros(nodes.size, dtype=np.int8)
    params = np.zeros(9, dtype=np.uint32)
    lib().pwo_probe_eval(n, seed, uid, k, nodes.size, _ptr(nodes), _ptr(pi), _ptr(z), _ptr(params))
    return pi, z, params


def walk_trace(g, start: int, L: int, seed: int, uid: int, k: int, p: int, side: int):
    """Node sequence X_0..X_L of one walk, and its binary32 sum of z/d."""
    trace = np.zeros(L + 1, dtype=np.int32)
    acc = np.zeros(1, dtype=np.float32)
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(g.col, dtype=np.int32)
    lib().pwo_walk_trace(g.n, _ptr(rp), _ptr(col), start, L, seed, uid, k, p, side,
                         _ptr(trace), _ptr(acc))
    return trace, float(acc[0])


def replicas(g, s: int, t: int, L: int, uid: int, k: int, p_begin: int, count: int, seed: int):
    """U_p = a - b for p in [p_begin, p_begin + count) at probe k."""
    out = np.zeros(count, dtype=np.float32)
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(g.col, dtype=np.int32)
    lib().pwo_replicas(g.n, _ptr(rp), _ptr(col), s, t, L, uid, k, p_begin, count, seed, _ptr(out))
    return out


def q_from_u(U) -> float:
    U = np.ascontiguousarray(U, dtype=np.float32)
    return float(lib().pwo_q_from_u(U.size, _ptr(U)))


def estimate(g, s, t, L, plans, seed: int, uid=None, threads: int = 1,
             k_end=None, want_q: bool = False, share=1):
    """Run Algorithm 1 for each query.

    ``plans`` is a sequence of (B, G, K, R) tuples, one per query. ``share``
    (scalar or per query) is the walk-sharing group size M; 1 is Algorithm 1.
    Returns beta-hat per query, and (when ``want_q``) the per-probe Q and the
    G block means of query 0.
    """
    s = np.ascontiguousarray(s, dtype=np.int32)
    t = np.ascontiguousarray(t, dtype=np.int32)
    L = np.ascontiguousarray(np.broadcast_to(L, s.shape), dtype=np.int32)
    nq = s.size
    plans = list(plans)
    B = np.array([p[0] for p in plans], dtype=np.int64)
    G = np.array([p[1] for p in plans], dtype=np.int64)
    K = np.array([p[2] for p in plans], dtype=np.int64)
    R = np.array([p[3] for p in plans], dtype=np.int64)
    M = np.ascontiguousarray(np.broadcast_to(np.asarray(share, dtype=np.int64), s.shape))
    uid_a = None if uid is None else np.ascontiguousarray(uid, dtype=np.uint32)
    kend = None if k_end is None else np.ascontiguousarray(k_end, dtype=np.int64)
    beta = np.zeros(nq, dtype=np.float64)
    q0 = np.zeros(int(K[0]), dtype=np.float64) if want_q else None
    y0 = np.zeros(int(G[0]), dtype=np.float64) if want_q else None
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(g.col, dtype=np.int32)
    rc = lib().pwo_estimate(
        g.n, _ptr(rp), _ptr(col), nq, _ptr(s), _ptr(t), _ptr(L),
        None if uid_a is None else _ptr(uid_a), _ptr(K), _ptr(R), _ptr(B), _ptr(G), _ptr(M),
        None if kend is None else _ptr(kend), seed, threads, _ptr(beta),
        None if q0 is None else _ptr(q0), None if y0 is None else _ptr(y0))
    if rc != 0:
        raise RuntimeError(f"oracle estimate failed: {rc}")
    if want_q:
        return beta, q0, y0
    return beta


def probe_q(g, s: int, t: int, L: int, uid: int, R: int, seed: int, ks, threads: int = 1,
            B: int = 1, share: int = 1):
    """Q_R(z^(k)) for each probe index in ``ks`` (threads over probes). With walk
    sharing (group size ``share`` inside blocks of ``B`` probes) probe k is
    scored on the walks of its group."""
    ks = np.ascontiguousarray(ks, dtype=np.uint32)
    out = np.zeros(ks.size, dtype=np.float64)
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(g.col, dtype=np.int32)
    lib().pwo_probe_q(g.n, _ptr(rp), _ptr(col), s, t, L, uid, R, B, share, seed, ks.size, _ptr(ks),
                      threads, _ptr(out))
    return out
