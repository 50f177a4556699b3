"""Degree-ordered internal numbering (SR_LOAD_REORDER): every program must
return the oracle's result in the caller's ids, on every schedule."""
import sys

import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sr():
    import paper_1806_00762_amd as sr
    sr.lib()
    return sr


@pytest.fixture(scope="module")
def ctx(sr):
    c = sr.Context(0, 0)
    yield c
    c.close()


GRAPHS = {
    "rmat14w": lambda: graphgen.rmat(14, 16, seed=14, weights=(1, 255, 5)),
    "uniform12w": lambda: graphgen.uniform(12, 1 << 15, seed=9, weights=(1, 255, 7)),
}
SCHED = {"resident": (1, 4, False, 0), "s4p7d2": (7, 4, True, 2), "s3p3": (3, 3, True, 1)}


@pytest.mark.parametrize("gname", list(GRAPHS))
@pytest.mark.parametrize("sched", list(SCHED))
def test_reorder_min_programs(sr, ctx, gname, sched):
    g = GRAPHS[gname]()
    parts, slots, force, depth = SCHED[sched]
    src = int(np.argmax(np.diff(g.offsets)))
    for algo, ref, sym in (("sssp", oracle.sssp(g, src), False), ("bfs", oracle.bfs(g, src), False),
                           ("cc", oracle.cc(g), True)):
        G = ctx.load(g, symmetrize=sym, reorder=True)
        try:
            G.partition(parts, slots)
            for pvu in ("strong", "weak"):
                say(f"case reorder {gname} {sched} {algo} {pvu}")
                st = G.run(algo, source=src, pvu=pvu, max_inner_iters=4, force_stream=force, copy_depth=depth)
                assert st["converged"] == 1
                got = G.values()
                assert np.array_equal(got, ref), f"{algo} {pvu}: {np.sum(got != ref)} mismatches"
            # with the host sparse stage and page skipping (internal ids end to end)
            st = G.run(algo, source=src, pvu="strong", force_stream=force, copy_depth=depth, hetero=True,
                       skip_clean=force, sparse_switch=256)
            assert np.array_equal(G.values(), ref)
        finally:
            G.close()


@pytest.mark.parametrize("sched", ["resident", "s4p7d2"])
def test_reorder_pagerank(sr, ctx, sched):
    g = GRAPHS["rmat14w"]()
    parts, slots, force, depth = SCHED[sched]
    ref, _, _ = oracle.pagerank(g, tol=1e-13)
    seed = int(graphgen.sources_with_outedges(g, 1, seed=77)[0])
    pref, _, _ = oracle.pagerank(g, seed=seed, tol=1e-13)
    G = ctx.load(g, reorder=True)
    try:
        G.partition(parts, slots)
        G.run("pagerank", pvu="weak", force_stream=force, copy_depth=depth)
        x = G.values().view(np.float32).astype(np.float64)
        assert np.max(np.abs(x - ref)) <= 1e-6
        G.run("ppr", source=seed, pvu="weak", force_stream=force, copy_depth=depth)
        x = G.values().view(np.float32).astype(np.float64)
        assert np.max(np.abs(x - pref)) <= 1e-6
    finally:
        G.close()


def test_reorder_batch_and_server(sr, ctx):
    """Batched and served queries take sources and return values in the
    caller's ids on a reordered graph."""
    import time
    g = GRAPHS["rmat14w"]()
    G = ctx.load(g, reorder=True)
    try:
        srcs = [int(s) for s in graphgen.sources_with_outedges(g, 10, seed=31)]
        outs, _, _ = sr.batch_run(ctx, [(G, "sssp" if i % 2 else "bfs", s) for i, s in enumerate(srcs)])
        for i, (s, x) in enumerate(zip(srcs, outs)):
            ref = oracle.sssp(g, s) if i % 2 else oracle.bfs(g, s)
            assert np.array_equal(x, ref), (i, s)
        outs, _, _ = sr.batch_run(ctx, [(G, "ppr", s) for s in srcs[:4]])
        for s, x in zip(srcs[:4], outs):
            ref, _, _ = oracle.pagerank(g, seed=s, tol=1e-13)
            assert np.max(np.abs(x.view(np.float32).astype(np.float64) - ref)) <= 1e-6
        srv = sr.Server(ctx, [G], slots=32)
        tickets = [srv.submit(0, "sssp", s) for s in srcs]
        res = {}
        t0 = time.time()
        while len(res) < len(tickets) and time.time() - t0 < 60:
            for t, s in zip(tickets, srcs):
                if t in res:
                    continue
                buf = np.empty(g.n, dtype=np.uint32)
                done, _ = srv.poll(t, buf)
                if done:
                    res[t] = buf
            time.sleep(0.001)
        srv.close()
        for t, s in zip(tickets, srcs):
            assert np.array_equal(res[t], oracle.sssp(g, s)), s
    finally:
        G.close()
