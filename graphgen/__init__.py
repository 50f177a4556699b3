"""Seeded synthetic graph inputs shared by the CPU oracle and the GPU library.

Input generation only (no graph algorithm lives here): R-MAT and uniform edge
lists drawn from a counter-based SplitMix64 stream, uint32 weights from Lemire
bounded draws, cleaned (self-loops dropped, optional symmetrization, duplicate
edges removed keeping the smallest weight) into a sorted out-edge CSR.
The C++ source is ``graphgen.cpp``; ``build()`` compiles it with g++/OpenMP.

Workload recipes (R-MAT parameters a=0.57, b=0.19, c=0.19, d=0.05 as in the
evaluated R-MAT family, Section 5, Table III) are collected in ``recipes``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.cpp")
_LIB_PATH = os.path.join(_HERE, "libgraphgen.so")
_lib = None

RMAT, UNIFORM = 0, 1


def build(force: bool = True) -> str:
    """Compile libgraphgen.so next to this file (g++ -O3 -fopenmp)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["g++", "-O3", "-march=x86-64-v2", "-std=c++17", "-fopenmp", "-fPIC", "-shared",
               _SRC, "-o", tmp]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=False)
    lib = ctypes.CDLL(_LIB_PATH)
    lib.gg_generate.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int64, ctypes.c_double,
                                ctypes.c_double, ctypes.c_double, ctypes.c_uint64, ctypes.c_int,
                                ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int,
                                ctypes.c_int, ctypes.POINTER(ctypes.c_void_p)]
    lib.gg_generate.restype = ctypes.c_int
    lib.gg_info.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32),
                            ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32)]
    lib.gg_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    lib.gg_free.argtypes = [ctypes.c_void_p]
    lib.gg_splitmix64_draw.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
    lib.gg_splitmix64_draw.restype = ctypes.c_uint64
    lib.gg_bounded_draws.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64,
                                     ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p]
    _lib = lib
    return lib


@dataclass
class Graph:
    """Out-edge CSR: row ``u`` lists the heads ``col[offsets[u]:offsets[u+1]]``."""
    n: int
    offsets: np.ndarray            # int64[n+1]
    col: np.ndarray                # int32[m]
    weights: Optional[np.ndarray]  # uint32[m] or None
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.offsets[-1])

    def outdeg(self) -> np.ndarray:
        return np.diff(self.offsets)


def generate(kind: int, scale: int, nedges: int, *, a=0.57, b=0.19, c=0.19, seed: int = 1,
             weights: Optional[tuple] = None, symmetrize: bool = False, nthreads: int = 0,
             name: str = "") -> Graph:
    """Generate a cleaned graph with 2**scale vertices from ``nedges`` draws.

    ``weights`` = (lo, hi, wseed) draws uint32 weights uniformly in [lo, hi].
    """
    lib = _load()
    h = ctypes.c_void_p()
    wlo, whi, wseed = (weights if weights is not None else (0, 0, 0))
    rc = lib.gg_generate(kind, scale, nedges, a, b, c, seed, 1 if weights else 0, wseed, wlo, whi,
                         1 if symmetrize else 0, nthreads, ctypes.byref(h))
    if rc != 0:
        raise ValueError(f"gg_generate failed with {rc}")
    try:
        n = ctypes.c_int32(); m = ctypes.c_int64(); wt = ctypes.c_int32()
        lib.gg_info(h, ctypes.byref(n), ctypes.byref(m), ctypes.byref(wt))
        offsets = np.empty(n.value + 1, dtype=np.int64)
        col = np.empty(max(m.value, 0), dtype=np.int32)
        w = np.empty(m.value, dtype=np.uint32) if wt.value else None
        lib.gg_copy(h, offsets.ctypes.data, col.ctypes.data, w.ctypes.data if w is not None else None)
    finally:
        lib.gg_free(h)
    return Graph(n.value, offsets, col, w, name)


def rmat(scale: int, edge_factor: int, seed: int, *, weights=None, symmetrize=False,
         a=0.57, b=0.19, c=0.19, nthreads=0, name="") -> Graph:
    return generate(RMAT, scale, edge_factor << scale, a=a, b=b, c=c, seed=seed, weights=weights,
                    symmetrize=symmetrize, nthreads=nthreads,
                    name=name or f"rmat{scale}_ef{edge_factor}_s{seed}")


def uniform(scale: int, nedges: int, seed: int, *, weights=None, symmetrize=False, nthreads=0,
            name="") -> Graph:
    return generate(UNIFORM, scale, nedges, seed=seed, weights=weights, symmetrize=symmetrize,
                    nthreads=nthreads, name=name or f"uniform{scale}_m{nedges}_s{seed}")


def splitmix64_draw(key: int, k: int) -> int:
    return int(_load().gg_splitmix64_draw(key, k))


def bounded_draws(seed: int, stream: int, count: int, lo: int, hi: int) -> np.ndarray:
    """``count`` seeded uint32 integers uniform in [lo, hi]."""
    out = np.empty(count, dtype=np.uint32)
    if count:
        _load().gg_bounded_draws(seed, stream, count, lo, hi, out.ctypes.data)
    return out


def from_edges(n: int, src, dst, w=None, *, symmetrize=False, drop_self_loops=True,
               dedup=True, name="") -> Graph:
    """Small hand-made graphs: build a cleaned, sorted out-CSR from edge arrays."""
    src = np.asarray(src, dtype=np.int64).ravel()
    dst = np.asarray(dst, dtype=np.int64).ravel()
    ww = None if w is None else np.asarray(w, dtype=np.uint64).ravel()
    if src.size and (src.min() < 0 or src.max() >= n or dst.min() < 0 or dst.max() >= n):
        raise ValueError("edge endpoint out of range")
    if symmetrize:
        src, dst = np.concatenate([src, dst]), np.concatenate([dst, src])
        if ww is not None:
            ww = np.concatenate([ww, ww])
    if drop_self_loops:
        keep = src != dst
        src, dst = src[keep], dst[keep]
        if ww is not None:
            ww = ww[keep]
    if ww is None:
        order = np.lexsort((dst, src))
    else:
        order = np.lexsort((ww, dst, src))
    src, dst = src[order], dst[order]
    if ww is not None:
        ww = ww[order]
    if dedup and src.size:
        first = np.ones(src.size, dtype=bool)
        first[1:] = (src[1:] != src[:-1]) | (dst[1:] != dst[:-1])
        src, dst = src[first], dst[first]
        if ww is not None:
            ww = ww[first]
    offsets = np.zeros(n + 1, dtype=np.int64)
    np.add.at(offsets, src + 1, 1)
    offsets = np.cumsum(offsets)
    return Graph(n, offsets, dst.astype(np.int32),
                 None if ww is None else ww.astype(np.uint32), name)


def grid(rows: int, cols: int, *, weights=None, name="") -> Graph:
    """2-D lattice with row-major ids and arcs both ways between 4-neighbours:
    a high-diameter graph with locality (page-level skipping has work to save).
    ``weights`` = (lo, hi, seed) draws one weight per arc."""
    n = rows * cols
    ids = np.arange(n, dtype=np.int64).reshape(rows, cols)
    right = (ids[:, :-1].ravel(), ids[:, 1:].ravel())
    down = (ids[:-1, :].ravel(), ids[1:, :].ravel())
    src = np.concatenate([right[0], right[1], down[0], down[1]])
    dst = np.concatenate([right[1], right[0], down[1], down[0]])
    w = None
    if weights is not None:
        lo, hi, seed = weights
        w = bounded_draws(seed, 3, src.size, lo, hi)
    return from_edges(n, src, dst, w, name=name or f"grid{rows}x{cols}")


# --- workload recipes -------------------------------------------------------
# Seeds and shapes of the synthetic workloads; each returns a Graph.

class recipes:
    @staticmethod
    def pagerank_s16() -> Graph:
        """R-MAT scale 16, edge factor 16, directed, cleaned (PageRank workload)."""
        return rmat(16, 16, seed=16, name="rmat16_ef16")

    @staticmethod
    def sssp_s22() -> Graph:
        """R-MAT scale 22, edge factor 16, directed, uint32 weights in [1,255]."""
        return rmat(22, 16, seed=22, weights=(1, 255, 122), name="rmat22_ef16_w")

    @staticmethod
    def cc_rmat_s24() -> Graph:
        """R-MAT scale 24, edge factor 32, symmetrized (connected components)."""
        return rmat(24, 32, seed=24, symmetrize=True, name="rmat24_ef32_sym")

    @staticmethod
    def cc_uniform_s24() -> Graph:
        """Uniform twin of the scale-24 R-MAT: 2^24 vertices, 2^29 uniform pairs, symmetrized."""
        return uniform(24, 32 << 24, seed=124, symmetrize=True, name="uniform24_m2^29_sym")

    @staticmethod
    def batched_graph(i: int) -> Graph:
        """Graph i of the 32-graph batched personalized-PageRank set (scales 12-20)."""
        scale = 12 + (9 * i) // 32
        ef = 8 << (i % 3)
        return rmat(scale, ef, seed=1000 + i, name=f"batch{i}_rmat{scale}_ef{ef}")

    @staticmethod
    def serving_graph(scale: int) -> Graph:
        """Resident serving graphs: R-MAT scale 20/22/23, ef 16, uint32 weights in [1,255]."""
        return rmat(scale, 16, seed=300 + scale, weights=(1, 255, 400 + scale),
                    name=f"serve_rmat{scale}_ef16_w")


def sources_with_outedges(g: Graph, count: int, seed: int, stream: int = 7) -> np.ndarray:
    """Seeded sources drawn uniformly from the vertices with out-degree >= 1."""
    cand = np.nonzero(np.diff(g.offsets) > 0)[0].astype(np.int64)
    if cand.size == 0:
        raise ValueError("graph has no vertex with an out-edge")
    idx = bounded_draws(seed, stream, count, 0, cand.size - 1)
    return cand[idx.astype(np.int64)].astype(np.int32)


def poisson_arrivals(rate_per_s: float, count: int, seed: int) -> np.ndarray:
    """Arrival times (s) of a Poisson process: exponential gaps from seeded uniforms."""
    u = bounded_draws(seed, 11, count, 0, 0xFFFFFFFE).astype(np.float64)
    u = (u + 0.5) / 4294967296.0                      # (0, 1)
    return np.cumsum(-np.log(u) / rate_per_s)
