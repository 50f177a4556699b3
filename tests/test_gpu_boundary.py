"""Boundary features on the device: caller-provided streams and device memory
(PyTorch's streams and caching allocator behind sr_ctx_set_streams and
sr_ctx_set_allocator), bit-reproducible PageRank (SR_RUN_DETERMINISTIC), and
the equal-edge page split. Every result is checked against the oracle:
integer programs bit-exact, PageRank within 1e-6 max-abs of the FP64 fixed
point."""
import sys

import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def sr():
    import paper_1806_00762_amd as sr
    sr.lib()
    return sr


@pytest.fixture(scope="module")
def torch():
    import torch
    torch.cuda.init()
    return torch


def test_torch_streams_and_allocator(sr, torch):
    """Streamed SSSP and PageRank with torch streams for compute and copies and
    every device byte from torch's caching allocator: results match the
    oracle, torch accounts for the library's memory while the context holds
    it, and gets it all back when the context is destroyed."""
    g = graphgen.rmat(14, 16, seed=14, weights=(1, 255, 114))
    ref_d = oracle.sssp(g, 0)
    ref_x, _, _ = oracle.pagerank(g, tol=1e-13)
    base = torch.cuda.memory_allocated(0)
    compute, copy = torch.cuda.Stream(0), torch.cuda.Stream(0)
    # a quarter of the graph bytes for the page slots, plus the vertex state
    # of both programs (values, predictor states, PageRank terms)
    budget = (4 * (g.n + 1) + 8 * g.m) // 4 + 16 * g.n + (1 << 20)
    ctx = sr.Context(0, budget)
    ctx.set_streams(compute.cuda_stream, copy.cuda_stream)
    ctx.set_torch_allocator(stream=compute)
    G = ctx.load(g, reorder=True)
    G.partition(0, 4)
    st = G.run("sssp", source=0, pvu="strong", max_inner_iters=4, force_stream=True, copy_depth=2)
    assert st["h2d_bytes"] > 0
    assert np.array_equal(G.values(), ref_d)
    used, _ = ctx.memory()
    held = torch.cuda.memory_allocated(0) - base
    say(f"torch allocator: library charged {used} B, torch holds {held} B more")
    assert held >= used > 0
    st = G.run("pagerank", pvu="off", max_inner_iters=2, force_stream=True)
    x = G.values(np.float32).astype(np.float64)
    assert float(np.max(np.abs(x - ref_x))) <= 1e-6
    # the caller's streams carried the work: the library synchronised them,
    # and torch's own view of them is idle
    assert compute.query() and copy.query()
    G.close()
    ctx.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated(0) == base


@pytest.mark.parametrize("algo,seed", [("pagerank", -1), ("ppr", 5)])
@pytest.mark.parametrize("stream", [False, True])
def test_deterministic_pagerank_bit_identical(sr, algo, seed, stream):
    """Two deterministic runs give the same FP32 bits, resident (every page
    in one sweep) and streamed (4 pages through 2 slots, up to 4 sweeps per
    window); both within 1e-6 max-abs of the FP64 oracle."""
    g = graphgen.recipes.pagerank_s16()
    ref, _, _ = oracle.pagerank(g, seed=seed, tol=1e-13)
    src = seed if seed >= 0 else 0
    with sr.Context(0, 0) as ctx:
        G = ctx.load(g)
        G.partition(4, 2)
        outs = []
        for rep in range(2):
            st = G.run(algo, source=src, pvu="off", max_inner_iters=4, force_stream=stream,
                       deterministic=True)
            assert st["stop_reason"] in (1, 2)
            outs.append(G.values())
        x = outs[0].view(np.float32).astype(np.float64)
        err = float(np.max(np.abs(x - ref)))
        say(f"deterministic {algo} stream={stream}: sweeps {st['sweeps']} max-abs {err:.2e}")
        assert np.array_equal(outs[0], outs[1])
        assert err <= 1e-6
        G.close()


def test_deterministic_weak_pagerank(sr):
    """Weak prediction with a change tolerance under the deterministic flag:
    bit-identical twice, and the fixed point within 1e-6."""
    g = graphgen.rmat(14, 16, seed=3)
    ref, _, _ = oracle.pagerank(g, tol=1e-13)
    with sr.Context(0, 0) as ctx:
        G = ctx.load(g, reorder=True)
        G.partition(3, 4)
        outs = [None, None]
        for rep in range(2):
            G.run("pagerank", pvu="weak", pr_change_eps=1e-9, max_inner_iters=3, force_stream=True,
                  deterministic=True)
            outs[rep] = G.values()
        assert np.array_equal(outs[0], outs[1])
        assert float(np.max(np.abs(outs[0].view(np.float32).astype(np.float64) - ref))) <= 1e-6
        G.close()


def test_equal_edge_pagerank_s16(sr):
    """The scale-16 PageRank workload on 4 equal-edge pages, up to 4 in-GPU
    sweeps per page per pass, one page resident at a time: within 1e-6
    max-abs of the FP64 oracle (and far closer)."""
    g = graphgen.recipes.pagerank_s16()
    ref, _, _ = oracle.pagerank(g, tol=1e-13)
    with sr.Context(0, 0) as ctx:
        G = ctx.load(g)
        G.partition(4, 2, equal_edges=True)
        assert G.info()["num_parts"] == 4
        for pvu in ("off", "weak"):
            st = G.run("pagerank", pvu=pvu, max_inner_iters=4, force_stream=True, tol_l1=1e-9)
            x = G.values(np.float32).astype(np.float64)
            err = float(np.max(np.abs(x - ref)))
            say(f"equal-edge pagerank {pvu}: passes {st['passes']} max-abs {err:.2e}")
            assert st["stop_reason"] in (1, 2)
            assert err <= 1e-8
        G.close()
