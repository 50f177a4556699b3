"""CPU oracle for the Seraph vertex programs (arXiv 1806.00762).

TEST INFRASTRUCTURE ONLY: only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package. The product path
never does. It shares no code with the GPU library.

Plain definitions in FP64 / 64-bit integers, written in ``oracle.c``:
  * SSSP: Dijkstra (indexed binary heap); Bellman-Ford as a cross-check.
  * BFS: FIFO queue.
  * CC: union-find; label = smallest vertex id of the component (Section 4.1);
    synchronous label propagation over OpenMP threads (the multi-core CPU
    baseline), pinned to union-find.
  * PageRank / personalized PageRank: Jacobi power iteration,
    x = (1-d) t + d (P^T x + D t), D = dangling mass (the paper names PageRank
    in Section 4.3 but does not define it; this is the textbook form).
  * Certificates for SSSP/BFS and CC; the PageRank residual bound.
  * Predictive vertex updating reference semantics: Table I thresholds and the
    Fig. 6 weak state machine as the Section 4.3 text describes it.
``build()`` compiles ``oracle.c`` with gcc -O2 into ``liboracle.so``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

INF = 0xFFFFFFFF

_p = ctypes.c_void_p
_i32, _i64, _u32, _dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_double


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=False)
    lib = ctypes.CDLL(_LIB_PATH)
    sig = {
        "or_sssp_dijkstra": [_i32, _p, _p, _p, _i32, _p],
        "or_sssp_bellman_ford": [_i32, _p, _p, _p, _i32, _p, _p],
        "or_bfs": [_i32, _p, _p, _i32, _p],
        "or_cc_union_find": [_i32, _p, _p, _p],
        "or_cc_labelprop_sync": [_i32, _p, _p, _i32, _p, _p, _p],
        "or_cc_labelprop_parallel": [_i32, _p, _p, _i32, _p, _p, _p],
        "or_pagerank": [_i32, _p, _p, _dbl, _i32, _dbl, _i32, _p, _p, _p],
        "or_pagerank_partial": [_i32, _p, _p, _dbl, _i32, _i32, _p],
        "or_pagerank_residual": [_i32, _p, _p, _dbl, _i32, _p, _p],
        "or_sssp_certificate": [_i32, _p, _p, _p, _i32, _p, _p],
        "or_cc_check": [_i32, _p, _p, _p, _p],
        "or_strong_threshold_sssp": [_i32, _p, _p],
        "or_strong_threshold_cc": [_i32, _p, _p],
        "or_weak_next": [_i32, _i32, _i32, _u32, _p, _p],
        "or_weak_default_diagram": [_p, _p, _p, _p, _p],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.or_strong_threshold_sssp.restype = _u32
    lib.or_strong_threshold_cc.restype = _u32
    lib.or_strong_threshold_bfs.argtypes = [_i32]
    lib.or_strong_threshold_bfs.restype = _u32
    lib.or_weak_next.restype = _i32
    lib.or_weak_default_diagram.restype = None
    _lib = lib
    return lib


def _csr(g):
    off = np.ascontiguousarray(g.offsets, dtype=np.int64)
    col = np.ascontiguousarray(g.col, dtype=np.int32)
    w = None if getattr(g, "weights", None) is None else np.ascontiguousarray(g.weights, dtype=np.uint32)
    return off, col, w


def _ptr(a):
    return None if a is None else a.ctypes.data


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def sssp(g, src: int, weights=True) -> np.ndarray:
    """Dijkstra distances (uint32, INF = 0xFFFFFFFF). weights=False uses unit weights."""
    off, col, w = _csr(g)
    out = np.empty(g.n, dtype=np.uint32)
    _check(_load().or_sssp_dijkstra(g.n, _ptr(off), _ptr(col), _ptr(w) if weights else None, src,
                                    _ptr(out)), "dijkstra")
    return out


def sssp_bellman_ford(g, src: int, weights=True):
    off, col, w = _csr(g)
    out = np.empty(g.n, dtype=np.uint32)
    rounds = ctypes.c_int32()
    _check(_load().or_sssp_bellman_ford(g.n, _ptr(off), _ptr(col), _ptr(w) if weights else None,
                                        src, _ptr(out), ctypes.byref(rounds)), "bellman-ford")
    return out, rounds.value


def bfs(g, src: int) -> np.ndarray:
    off, col, _ = _csr(g)
    out = np.empty(g.n, dtype=np.uint32)
    _check(_load().or_bfs(g.n, _ptr(off), _ptr(col), src, _ptr(out)), "bfs")
    return out


def cc(g) -> np.ndarray:
    off, col, _ = _csr(g)
    out = np.empty(g.n, dtype=np.uint32)
    _check(_load().or_cc_union_find(g.n, _ptr(off), _ptr(col), _ptr(out)), "union-find")
    return out


def cc_labelprop_sync(g, iters: int):
    """Synchronous min-label propagation; returns (labels, history[iters, n], changed_iters)."""
    off, col, _ = _csr(g)
    lab = np.empty(g.n, dtype=np.uint32)
    hist = np.empty((iters, g.n), dtype=np.uint32)
    nch = ctypes.c_int32()
    _check(_load().or_cc_labelprop_sync(g.n, _ptr(off), _ptr(col), iters, _ptr(lab), _ptr(hist),
                                        ctypes.byref(nch)), "labelprop")
    return lab, hist, nch.value


def cc_labelprop_parallel(g, threads: int = 0):
    """Synchronous min-label propagation to the fixed point over `threads`
    OpenMP threads (0 = all); g must be symmetric. Returns (labels, iterations,
    threads used)."""
    off, col, _ = _csr(g)
    lab = np.empty(g.n, dtype=np.uint32)
    it = ctypes.c_int32(); tu = ctypes.c_int32()
    _check(_load().or_cc_labelprop_parallel(g.n, _ptr(off), _ptr(col), threads, _ptr(lab), ctypes.byref(it),
                                            ctypes.byref(tu)), "parallel labelprop")
    return lab, it.value, tu.value


def pagerank(g, damping=0.85, seed: int = -1, tol=1e-13, max_iter=100000):
    """FP64 power iteration; seed >= 0 gives personalized PageRank with t = e_seed.
    Returns (x, iterations, last L1 change)."""
    off, col, _ = _csr(g)
    x = np.empty(g.n, dtype=np.float64)
    it = ctypes.c_int32(); l1 = ctypes.c_double()
    _check(_load().or_pagerank(g.n, _ptr(off), _ptr(col), damping, seed, tol, max_iter, _ptr(x),
                               ctypes.byref(it), ctypes.byref(l1)), "pagerank")
    return x, it.value, l1.value


def pagerank_partial(g, k: int, damping=0.85, seed: int = -1) -> np.ndarray:
    """The first k terms of the PageRank series (k steps from x0 = 0): the
    state of residual propagation after k synchronous passes."""
    off, col, _ = _csr(g)
    x = np.empty(g.n, dtype=np.float64)
    _check(_load().or_pagerank_partial(g.n, _ptr(off), _ptr(col), damping, seed, k, _ptr(x)), "pagerank_partial")
    return x


def pagerank_residual(g, x, damping=0.85, seed: int = -1) -> float:
    off, col, _ = _csr(g)
    xx = np.ascontiguousarray(x, dtype=np.float64)
    r = ctypes.c_double()
    _check(_load().or_pagerank_residual(g.n, _ptr(off), _ptr(col), damping, seed, _ptr(xx),
                                        ctypes.byref(r)), "residual")
    return r.value


def sssp_certificate(g, src: int, dist, weights=True):
    """0 if dist passes the exactness certificate, else (code, witness)."""
    off, col, w = _csr(g)
    d = np.ascontiguousarray(dist, dtype=np.uint32)
    bad = ctypes.c_int64(-1)
    rc = _load().or_sssp_certificate(g.n, _ptr(off), _ptr(col), _ptr(w) if weights else None, src,
                                     _ptr(d), ctypes.byref(bad))
    return 0 if rc == 0 else (rc, bad.value)


def cc_check(g, labels):
    off, col, _ = _csr(g)
    lab = np.ascontiguousarray(labels, dtype=np.uint32)
    bad = ctypes.c_int64(-1)
    rc = _load().or_cc_check(g.n, _ptr(off), _ptr(col), _ptr(lab), ctypes.byref(bad))
    return 0 if rc == 0 else (rc, bad.value)


def strong_threshold_bfs(k: int) -> int:
    return int(_load().or_strong_threshold_bfs(k))


def strong_threshold_sssp(prev, cur) -> int:
    p = np.ascontiguousarray(prev, dtype=np.uint32); c = np.ascontiguousarray(cur, dtype=np.uint32)
    return int(_load().or_strong_threshold_sssp(p.size, _ptr(p), _ptr(c)))


def strong_threshold_cc(prev, cur) -> int:
    p = np.ascontiguousarray(prev, dtype=np.uint32); c = np.ascontiguousarray(cur, dtype=np.uint32)
    return int(_load().or_strong_threshold_cc(p.size, _ptr(p), _ptr(c)))


def weak_default_diagram():
    """(num_states, initial, attempt_mask, on_success[8], on_fail[8]) of the Fig. 6 reading."""
    ns = ctypes.c_int32(); ini = ctypes.c_int32(); mask = ctypes.c_uint32()
    succ = (ctypes.c_uint8 * 8)(); fail = (ctypes.c_uint8 * 8)()
    _load().or_weak_default_diagram(ctypes.byref(ns), ctypes.byref(ini), ctypes.byref(mask), succ, fail)
    return ns.value, ini.value, mask.value, list(succ), list(fail)


def weak_next(state: int, changed: bool, diagram=None) -> int:
    ns, _, mask, succ, fail = diagram if diagram is not None else weak_default_diagram()
    s = (ctypes.c_uint8 * 8)(*succ); f = (ctypes.c_uint8 * 8)(*fail)
    return int(_load().or_weak_next(state, 1 if changed else 0, ns, mask, s, f))
