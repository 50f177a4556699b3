"""Python binding of libseraph (include/seraph.h): an MI355X engine for
Seraph's streamed, predictively-updated subgraph iteration (arXiv 1806.00762).

Argument marshalling only: every step of the computation runs in the HIP
library. There is no fallback; if ``libseraph.so`` has not been built, any
use raises immediately.

Low-level names mirror the C ABI (``sr_ctx_create``, ``sr_run`` ...); the
``Context`` / ``Graph`` classes wrap them for tests and benchmarks.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libseraph.so")

# --- enums / flags (seraph.h) ------------------------------------------------
SR_OK, SR_EINVAL, SR_ENOMEM, SR_EBUDGET, SR_EDEVICE, SR_ENOTCONV, SR_ESTATE, SR_EBUSY = 0, -1, -2, -3, -4, -5, -6, -7
SR_BFS, SR_SSSP, SR_CC, SR_PAGERANK, SR_PPR = 0, 1, 2, 3, 4
SR_PVU_OFF, SR_PVU_STRONG, SR_PVU_WEAK, SR_PVU_DEFAULT = 0, 1, 2, 3
SR_LOAD_SYMMETRIZE = 0x1
SR_LOAD_SYMMETRIC = 0x2
SR_LOAD_REORDER = 0x4
SR_RUN_AUDIT_PVU, SR_RUN_FORCE_STREAM, SR_RUN_RESUME, SR_RUN_FIXED_INNER, SR_RUN_HETERO = 0x1, 0x2, 0x4, 0x8, 0x10
SR_RUN_SKIP_CLEAN = 0x20
SR_RUN_NO_EARLY_BREAK = 0x40
SR_RUN_WIDE_PAGES = 0x80
SR_RUN_SPLIT_PAGES = 0x100
SR_RUN_DETERMINISTIC = 0x200
SR_RUN_PR_DELTA = 0x400
SR_PART_EQUAL_EDGES = 0x1
SR_STOP_CONVERGED, SR_STOP_FP32_FLOOR, SR_STOP_MAX_PASSES = 1, 2, 3
SR_INF = 0xFFFFFFFF

ALGOS = {"bfs": SR_BFS, "sssp": SR_SSSP, "cc": SR_CC, "pagerank": SR_PAGERANK, "pr": SR_PAGERANK,
         "ppr": SR_PPR}
PVUS = {"off": SR_PVU_OFF, "strong": SR_PVU_STRONG, "weak": SR_PVU_WEAK, "default": SR_PVU_DEFAULT}
_STATUS_NAMES = {0: "SR_OK", -1: "SR_EINVAL", -2: "SR_ENOMEM", -3: "SR_EBUDGET", -4: "SR_EDEVICE",
                 -5: "SR_ENOTCONV", -6: "SR_ESTATE", -7: "SR_EBUSY"}


class sr_graph_info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int64), ("weighted", ctypes.c_int32),
                ("symmetric", ctypes.c_int32), ("num_parts", ctypes.c_int32),
                ("num_slots", ctypes.c_int32), ("graph_bytes", ctypes.c_uint64),
                ("page_bytes_total", ctypes.c_uint64), ("max_page_bytes", ctypes.c_uint64),
                ("resident", ctypes.c_int32), ("reordered", ctypes.c_int32)]


class sr_page_view(ctypes.Structure):
    _fields_ = [("v_begin", ctypes.c_int32), ("v_end", ctypes.c_int32), ("num_edges", ctypes.c_int64),
                ("offsets", ctypes.POINTER(ctypes.c_int32)), ("src", ctypes.POINTER(ctypes.c_uint32)),
                ("weights", ctypes.POINTER(ctypes.c_uint32)), ("src_packed", ctypes.c_int32),
                ("bytes", ctypes.c_uint64), ("stream_bytes", ctypes.c_uint64)]


class sr_pvu_diagram(ctypes.Structure):
    _fields_ = [("num_states", ctypes.c_uint8), ("initial_state", ctypes.c_uint8),
                ("attempt_mask", ctypes.c_uint8), ("on_success", ctypes.c_uint8 * 8),
                ("on_fail", ctypes.c_uint8 * 8)]


class sr_run_params(ctypes.Structure):
    _fields_ = [("algo", ctypes.c_int), ("source", ctypes.c_int32), ("damping", ctypes.c_double),
                ("tol_l1", ctypes.c_double), ("max_passes", ctypes.c_int32),
                ("max_inner_iters", ctypes.c_int32), ("pvu", ctypes.c_int),
                ("diagram", ctypes.POINTER(sr_pvu_diagram)), ("pr_change_eps", ctypes.c_float),
                ("flags", ctypes.c_uint32), ("copy_depth", ctypes.c_int32), ("sparse_switch", ctypes.c_int32),
                ("sparse_return", ctypes.c_int32)]


class sr_run_stats(ctypes.Structure):
    _fields_ = [("passes", ctypes.c_int32), ("sweeps", ctypes.c_int32), ("verify_passes", ctypes.c_int32),
                ("converged", ctypes.c_int32), ("stop_reason", ctypes.c_int32),
                ("edges_scanned", ctypes.c_int64), ("vertices_attempted", ctypes.c_int64),
                ("vertices_skipped", ctypes.c_int64), ("mispredicted", ctypes.c_int64),
                ("h2d_bytes", ctypes.c_uint64), ("kernel_ms", ctypes.c_double),
                ("h2d_ms", ctypes.c_double), ("wall_ms", ctypes.c_double),
                ("final_l1", ctypes.c_double), ("state_hist", ctypes.c_int64 * 8),
                ("algo_bytes", ctypes.c_uint64), ("sparse_stage", ctypes.c_int32),
                ("sparse_rounds", ctypes.c_int32), ("sparse_frontier", ctypes.c_int64),
                ("sparse_relaxations", ctypes.c_int64), ("sparse_ms", ctypes.c_double),
                ("pages_skipped", ctypes.c_int64), ("sweep_kernel_ms", ctypes.c_double),
                ("edges_narrow", ctypes.c_int64), ("sparse_entries", ctypes.c_int32),
                ("sparse_returns", ctypes.c_int32), ("pr_delta_passes", ctypes.c_int32),
                ("sweep_launches", ctypes.c_int32), ("sparse_copy_bytes", ctypes.c_uint64)]

    def as_dict(self) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["state_hist"] = list(self.state_hist)
        return d


class sr_sweep_record(ctypes.Structure):
    _fields_ = [("pass_", ctypes.c_int32), ("phase", ctypes.c_int32), ("changed", ctypes.c_int64),
                ("attempted", ctypes.c_int64), ("skipped", ctypes.c_int64), ("edges", ctypes.c_int64),
                ("state_hist", ctypes.c_int64 * 8), ("l1", ctypes.c_double)]


_P = ctypes.c_void_p
_SIGNATURES = {
    "sr_ctx_create": (ctypes.c_int, [ctypes.c_int, ctypes.c_uint64, ctypes.POINTER(_P)]),
    "sr_ctx_destroy": (None, [_P]),
    "sr_ctx_last_error": (ctypes.c_char_p, [_P]),
    "sr_ctx_set_streams": (ctypes.c_int, [_P, _P, _P]),
    "sr_ctx_set_allocator": (ctypes.c_int, [_P, _P, _P, _P]),
    "sr_ctx_memory": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64)]),
    "sr_graph_load_csr": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int64, _P, _P, _P, ctypes.c_uint32,
                                         ctypes.POINTER(_P)]),
    "sr_graph_partition": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32]),
    "sr_graph_partition_ex": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint32]),
    "sr_graph_info_get": (ctypes.c_int, [_P, ctypes.POINTER(sr_graph_info)]),
    "sr_graph_page": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(sr_page_view)]),
    "sr_graph_order": (ctypes.c_int, [_P, _P, _P]),
    "sr_graph_destroy": (None, [_P]),
    "sr_pvu_default_diagram": (ctypes.c_int, [ctypes.POINTER(sr_pvu_diagram)]),
    "sr_run": (ctypes.c_int, [_P, ctypes.POINTER(sr_run_params), ctypes.POINTER(sr_run_stats)]),
    "sr_run_noalloc": (ctypes.c_int, [_P, ctypes.POINTER(sr_run_params), _P, _P, ctypes.POINTER(sr_run_stats)]),
    "sr_read_values": (ctypes.c_int, [_P, _P, ctypes.c_uint64]),
    "sr_run_sweeps": (ctypes.c_int, [_P, ctypes.POINTER(sr_sweep_record), ctypes.c_int32,
                                     ctypes.POINTER(ctypes.c_int32)]),
}
class sr_instance(ctypes.Structure):
    _fields_ = [("g", ctypes.c_void_p), ("algo", ctypes.c_int), ("source", ctypes.c_int32)]


class sr_batch_stats(ctypes.Structure):
    _fields_ = [("sweeps", ctypes.c_int32), ("groups", ctypes.c_int32), ("group_width", ctypes.c_int32),
                ("grid_blocks", ctypes.c_int32), ("grab", ctypes.c_int32), ("tuned", ctypes.c_int32),
                ("kernel_ms", ctypes.c_double), ("wall_ms", ctypes.c_double), ("algo_bytes", ctypes.c_uint64),
                ("rounds", ctypes.c_int32), ("width_candidates", ctypes.c_int32)]


class sr_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("sweeps", ctypes.c_uint64),
                ("slots_per_graph", ctypes.c_int32 * 8), ("busy_ms", ctypes.c_double),
                ("narrow_fallbacks", ctypes.c_uint64), ("kernel_ms", ctypes.c_double),
                ("algo_bytes", ctypes.c_uint64)]


EXTRA_SIGNATURES: dict = {
    "sr_batch_run": (ctypes.c_int, [_P, ctypes.POINTER(sr_instance), ctypes.c_int32, ctypes.POINTER(sr_run_params),
                                    ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(sr_run_stats),
                                    ctypes.POINTER(sr_batch_stats)]),
    "sr_server_create": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32, ctypes.c_uint64,
                                        ctypes.c_int32, ctypes.POINTER(_P)]),
    "sr_server_submit": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int, ctypes.c_int32,
                                        ctypes.POINTER(ctypes.c_uint64)]),
    "sr_server_poll": (ctypes.c_int, [_P, ctypes.c_uint64, _P, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int),
                                      ctypes.POINTER(ctypes.c_double)]),
    "sr_server_stats_get": (ctypes.c_int, [_P, ctypes.POINTER(sr_server_stats)]),
    "sr_server_destroy": (ctypes.c_int, [_P]),
    "sr_probe_gather": (ctypes.c_int, [_P, _P, ctypes.c_int64, ctypes.c_uint32, _P,
                                       ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_uint64)]),
}

_lib = None


def torch_hip_runtime() -> Optional[str]:
    """Path of the HIP runtime that PyTorch's ROCm build ships in its own lib
    folder (None when torch is not installed or brings none), found without
    importing torch."""
    import importlib.util
    try:
        spec = importlib.util.find_spec("torch")
    except (ImportError, ValueError):
        return None
    if spec is None or not spec.origin:
        return None
    p = os.path.join(os.path.dirname(spec.origin), "lib", "libamdhip64.so")
    return p if os.path.exists(p) else None


def lib():
    """Load libseraph.so (raises if it has not been built: no fallback exists).

    A process must hold one HIP runtime: PyTorch's ROCm build ships its own
    copy (with its own HSA runtime), and a second copy loaded beside it finds
    no device once the first has opened it, and could not take torch's streams
    or memory anyway. So when torch is installed its runtime is loaded first,
    globally, and libseraph's references to libamdhip64.so.7 bind to it
    (same soname); otherwise the system's ROCm runtime serves."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libseraph.so not built at {LIB_PATH}; run __graft_entry__.build()")
    rt = torch_hip_runtime()
    if rt is not None:
        ctypes.CDLL(rt, mode=os.RTLD_NOW | os.RTLD_GLOBAL)
    l = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in {**_SIGNATURES, **EXTRA_SIGNATURES}.items():
        fn = getattr(l, name)
        fn.restype = res
        fn.argtypes = args
    _lib = l
    return l


def exported_symbols() -> list:
    return sorted(set(_SIGNATURES) | set(EXTRA_SIGNATURES))


# sr_alloc_fn / sr_release_fn
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
RELEASE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class SeraphError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _check(rc: int, ctx_ptr=None):
    if rc != SR_OK:
        msg = lib().sr_ctx_last_error(ctx_ptr)
        raise SeraphError(rc, msg.decode() if msg else "")


def default_diagram() -> sr_pvu_diagram:
    d = sr_pvu_diagram()
    _check(lib().sr_pvu_default_diagram(ctypes.byref(d)))
    return d


def make_diagram(num_states, initial, attempt_states, on_success, on_fail) -> sr_pvu_diagram:
    d = sr_pvu_diagram()
    d.num_states = num_states
    d.initial_state = initial
    d.attempt_mask = sum(1 << s for s in attempt_states)
    for i in range(8):
        d.on_success[i] = on_success[i] if i < len(on_success) else 0
        d.on_fail[i] = on_fail[i] if i < len(on_fail) else 0
    return d


class Context:
    """A device (or host-only, device=-1) context with a device-memory budget."""

    def __init__(self, device: int = 0, budget_bytes: int = 0):
        h = _P()
        rc = lib().sr_ctx_create(device, budget_bytes, ctypes.byref(h))
        _check(rc, None)
        self.h = h
        self.device = device

    def close(self):
        if self.h:
            lib().sr_ctx_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def set_streams(self, compute: int = 0, copy: int = 0):
        """hipStream_t handles as integers (e.g. torch.cuda.Stream().cuda_stream)."""
        _check(lib().sr_ctx_set_streams(self.h, _P(compute or None), _P(copy or None)), self.h)

    def set_allocator(self, alloc=None, release=None):
        """Device memory from the caller (sr_ctx_set_allocator): alloc(nbytes) -> device
        address (int, 0 = out of memory), release(address). None restores hipMalloc.
        The callbacks stay referenced by the context object."""
        if alloc is None:
            self._alloc_cb = self._release_cb = None
            _check(lib().sr_ctx_set_allocator(self.h, None, None, None), self.h)
            return

        def _a(nbytes, _user):
            try:
                return int(alloc(int(nbytes))) or None
            except Exception:
                return None

        def _r(ptr, _user):
            release(int(ptr))

        self._alloc_cb, self._release_cb = ALLOC_FN(_a), RELEASE_FN(_r)
        _check(lib().sr_ctx_set_allocator(self.h, ctypes.cast(self._alloc_cb, _P),
                                          ctypes.cast(self._release_cb, _P), None), self.h)

    def set_torch_allocator(self, stream=None):
        """Device memory from PyTorch's caching allocator on the context's device
        (blocks are associated with `stream`, default the current stream)."""
        import torch
        dev = self.device
        st = stream if stream is not None else torch.cuda.current_stream(dev)

        def _alloc(nbytes):
            return torch.cuda.caching_allocator_alloc(nbytes, dev, st)

        def _release(ptr):
            torch.cuda.caching_allocator_delete(ptr)

        self.set_allocator(_alloc, _release)

    def memory(self):
        u, b = ctypes.c_uint64(), ctypes.c_uint64()
        _check(lib().sr_ctx_memory(self.h, ctypes.byref(u), ctypes.byref(b)), self.h)
        return u.value, b.value

    def load(self, g, symmetrize: bool = False, weights: Optional[bool] = None, symmetric: bool = False,
             reorder: bool = False) -> "Graph":
        return Graph(self, g, symmetrize=symmetrize, weights=weights, symmetric=symmetric, reorder=reorder)


class Graph:
    """A graph loaded into a context (C handle sr_graph)."""

    def __init__(self, ctx: Context, g, symmetrize=False, weights=None, symmetric=False, reorder=False):
        self.ctx = ctx
        off = np.ascontiguousarray(g.offsets, dtype=np.int64)
        col = np.ascontiguousarray(g.col, dtype=np.int32)
        w = getattr(g, "weights", None)
        if weights is False:
            w = None
        if w is not None:
            w = np.ascontiguousarray(w, dtype=np.uint32)
        h = _P()
        rc = lib().sr_graph_load_csr(ctx.h, int(g.n), int(off[-1]), off.ctypes.data, col.ctypes.data,
                                     None if w is None else w.ctypes.data,
                                     (SR_LOAD_SYMMETRIZE if symmetrize else 0) | (SR_LOAD_SYMMETRIC if symmetric else 0)
                                     | (SR_LOAD_REORDER if reorder else 0),
                                     ctypes.byref(h))
        _check(rc, ctx.h)
        self.h = h
        self.n = int(g.n)

    def close(self):
        if self.h:
            lib().sr_graph_destroy(self.h)
            self.h = None

    def partition(self, num_parts: int = 0, num_slots: int = 0, equal_edges: bool = False):
        """Cut into pages: equal streamed bytes (default) or equal in-edge counts."""
        _check(lib().sr_graph_partition_ex(self.h, num_parts, num_slots,
                                           SR_PART_EQUAL_EDGES if equal_edges else 0), self.ctx.h)

    def info(self) -> dict:
        i = sr_graph_info()
        _check(lib().sr_graph_info_get(self.h, ctypes.byref(i)), self.ctx.h)
        return {k: getattr(i, k) for k, _ in i._fields_}

    def order(self):
        """(internal_of, caller_of) vertex maps of a graph loaded with reorder=True."""
        a = np.empty(self.n, dtype=np.int32)
        b = np.empty(self.n, dtype=np.int32)
        _check(lib().sr_graph_order(self.h, a.ctypes.data, b.ctypes.data), self.ctx.h)
        return a, b

    def page(self, p: int) -> dict:
        v = sr_page_view()
        _check(lib().sr_graph_page(self.h, p, ctypes.byref(v)), self.ctx.h)
        npv = v.v_end - v.v_begin
        off = np.ctypeslib.as_array(v.offsets, shape=(npv + 1,)).copy()
        ne = int(v.num_edges)
        words = np.ctypeslib.as_array(v.src, shape=(ne,)).copy() if ne else np.zeros(0, np.uint32)
        w = None
        if v.src_packed:
            src = (words & 0xFFFFFF).astype(np.int32)
            w = (words >> 24).astype(np.uint32)
        else:
            src = words.view(np.int32)
            if v.weights and ne:
                w = np.ctypeslib.as_array(v.weights, shape=(ne,)).copy()
        return {"v_begin": v.v_begin, "v_end": v.v_end, "offsets": off, "src": src, "weights": w,
                "src_packed": bool(v.src_packed), "bytes": int(v.bytes), "stream_bytes": int(v.stream_bytes)}

    @staticmethod
    def _params(algo, source: int = 0, pvu="default", damping: float = 0.85, tol_l1: float = 1e-9,
                max_passes: int = 0, max_inner_iters: int = 0, diagram: Optional[sr_pvu_diagram] = None,
                pr_change_eps: float = 0.0, audit: bool = False, force_stream: bool = False,
                resume: bool = False, fixed_inner: bool = False, copy_depth: int = 0, hetero: bool = False,
                sparse_switch: int = 0, sparse_return: int = 0, skip_clean: bool = False,
                early_break: bool = True,
                wide_pages: bool = False, split_pages: bool = False, deterministic: bool = False,
                pr_delta: bool = False) -> sr_run_params:
        p = sr_run_params()
        p.algo = ALGOS[algo] if isinstance(algo, str) else int(algo)
        p.source = source
        p.damping = damping
        p.tol_l1 = tol_l1
        p.max_passes = max_passes
        p.max_inner_iters = max_inner_iters
        p.pvu = PVUS[pvu] if isinstance(pvu, str) else int(pvu)
        p.diagram = ctypes.pointer(diagram) if diagram is not None else None
        p.pr_change_eps = pr_change_eps
        p.flags = ((SR_RUN_AUDIT_PVU if audit else 0) | (SR_RUN_FORCE_STREAM if force_stream else 0)
                   | (SR_RUN_RESUME if resume else 0) | (SR_RUN_FIXED_INNER if fixed_inner else 0)
                   | (SR_RUN_HETERO if hetero else 0) | (SR_RUN_SKIP_CLEAN if skip_clean else 0)
                   | (0 if early_break else SR_RUN_NO_EARLY_BREAK)
                   | (SR_RUN_WIDE_PAGES if wide_pages else 0) | (SR_RUN_SPLIT_PAGES if split_pages else 0)
                   | (SR_RUN_DETERMINISTIC if deterministic else 0) | (SR_RUN_PR_DELTA if pr_delta else 0))
        p.copy_depth = copy_depth
        p.sparse_switch = sparse_switch
        p.sparse_return = sparse_return
        return p

    def run(self, algo, check: bool = True, **kw) -> dict:
        """sr_run: keyword arguments as the fields and flags of sr_run_params
        (see _params); returns the run statistics as a dict."""
        p = self._params(algo, **kw)
        st = sr_run_stats()
        rc = lib().sr_run(self.h, ctypes.byref(p), ctypes.byref(st))
        d = st.as_dict()
        d["status"] = rc
        if check and rc not in (SR_OK,):
            _check(rc, self.ctx.h)
        return d

    def run_noalloc(self, algo, values_dev: int, status_dev: int = 0, check: bool = True, **kw) -> dict:
        """sr_run_noalloc: the allocation-free solve on a resident graph, values
        written to the caller's device buffer at address values_dev (4n bytes),
        weak predictor states to status_dev (n bytes, or 0 when not weak)."""
        p = self._params(algo, **kw)
        st = sr_run_stats()
        rc = lib().sr_run_noalloc(self.h, ctypes.byref(p), ctypes.c_void_p(values_dev),
                                  ctypes.c_void_p(status_dev or None), ctypes.byref(st))
        d = st.as_dict()
        d["status"] = rc
        if check and rc not in (SR_OK,):
            _check(rc, self.ctx.h)
        return d

    def sweeps(self) -> list:
        """Per-sweep trace of the last run: pass, phase, changed/attempted/skipped vertices,
        scanned edges, weak-predictor state histogram, PageRank L1."""
        cnt = ctypes.c_int32()
        _check(lib().sr_run_sweeps(self.h, None, 0, ctypes.byref(cnt)), self.ctx.h)
        arr = (sr_sweep_record * max(cnt.value, 1))()
        _check(lib().sr_run_sweeps(self.h, arr, cnt.value, ctypes.byref(cnt)), self.ctx.h)
        out = []
        for i in range(cnt.value):
            r = arr[i]
            out.append({"pass": r.pass_, "phase": r.phase, "changed": r.changed, "attempted": r.attempted,
                        "skipped": r.skipped, "edges": r.edges, "state_hist": list(r.state_hist), "l1": r.l1})
        return out

    def values(self, dtype=None) -> np.ndarray:
        out = np.empty(self.n, dtype=np.uint32)
        _check(lib().sr_read_values(self.h, out.ctypes.data, out.nbytes), self.ctx.h)
        if dtype is not None:
            return out.view(dtype)
        return out


def probe_gather(ctx: Context, words, src_mask: int, values, repeats: int = 10):
    """Gather-rate probe (sr_probe_gather): u32 edge words and u32 values
    (host arrays). Returns (ms per launch, checksum)."""
    w = np.ascontiguousarray(words, dtype=np.uint32)
    v = np.ascontiguousarray(values, dtype=np.uint32)
    ms = ctypes.c_double()
    cs = ctypes.c_uint64()
    _check(lib().sr_probe_gather(ctx.h, w.ctypes.data if w.size else None, int(w.size), src_mask,
                                 v.ctypes.data if v.size else None, int(v.size), repeats,
                                 ctypes.byref(ms), ctypes.byref(cs)), ctx.h)
    return ms.value, cs.value


def batch_run(ctx: Context, instances, damping: float = 0.85, tol_l1: float = 1e-9, max_sweeps: int = 0,
              pvu="default", check: bool = True):
    """Run [(Graph, algo, source), ...] to convergence in one batched call.
    Returns (list of value arrays, list of per-instance stats, batch stats)."""
    cnt = len(instances)
    arr = (sr_instance * cnt)()
    outs = []
    for i, (G, algo, src) in enumerate(instances):
        arr[i].g = G.h.value if isinstance(G.h, ctypes.c_void_p) else G.h
        arr[i].algo = ALGOS[algo] if isinstance(algo, str) else int(algo)
        arr[i].source = int(src)
        outs.append(np.empty(G.n, dtype=np.uint32))
    dsts = (ctypes.c_void_p * cnt)(*[o.ctypes.data for o in outs])
    p = sr_run_params()
    p.damping = damping
    p.tol_l1 = tol_l1
    p.max_passes = max_sweeps
    p.pvu = PVUS[pvu] if isinstance(pvu, str) else int(pvu)
    per = (sr_run_stats * cnt)()
    bs = sr_batch_stats()
    rc = lib().sr_batch_run(ctx.h, arr, cnt, ctypes.byref(p), dsts, per, ctypes.byref(bs))
    if check and rc != SR_OK:
        _check(rc, ctx.h)
    return outs, [per[i].as_dict() for i in range(cnt)], {k: getattr(bs, k) for k, _ in bs._fields_}


class Server:
    """Continuous-batching SSSP/BFS query server over resident graphs."""

    def __init__(self, ctx: Context, graphs, state_budget_bytes: int = 0, slots: int = 16):
        self.ctx = ctx
        self.graphs = list(graphs)
        arr = (ctypes.c_void_p * len(self.graphs))(*[G.h.value if isinstance(G.h, ctypes.c_void_p) else G.h
                                                     for G in self.graphs])
        h = _P()
        _check(lib().sr_server_create(ctx.h, arr, len(self.graphs), state_budget_bytes, slots, ctypes.byref(h)),
               ctx.h)
        self.h = h

    def submit(self, graph: int, algo, source: int) -> int:
        t = ctypes.c_uint64()
        rc = lib().sr_server_submit(self.h, graph, ALGOS[algo] if isinstance(algo, str) else int(algo), source,
                                    ctypes.byref(t))
        if rc != SR_OK:
            raise SeraphError(rc, "submit failed")
        return t.value

    def poll(self, ticket: int, out: Optional[np.ndarray] = None):
        """(done, latency_ms); fills `out` (uint32[n]) when done."""
        done = ctypes.c_int(0)
        lat = ctypes.c_double(0.0)
        ptr = out.ctypes.data if out is not None else None
        nbytes = out.nbytes if out is not None else 0
        rc = lib().sr_server_poll(self.h, ticket, ptr, nbytes, ctypes.byref(done), ctypes.byref(lat))
        if rc != SR_OK:
            raise SeraphError(rc, "poll failed")
        return bool(done.value), lat.value

    def stats(self) -> dict:
        s = sr_server_stats()
        _check(lib().sr_server_stats_get(self.h, ctypes.byref(s)), self.ctx.h)
        d = {k: getattr(s, k) for k, _ in s._fields_}
        d["slots_per_graph"] = list(s.slots_per_graph)[:len(self.graphs)]
        return d

    def close(self):
        if self.h:
            rc = lib().sr_server_destroy(self.h)
            self.h = None
            if rc != SR_OK:
                raise SeraphError(rc, "server ended with an error")
