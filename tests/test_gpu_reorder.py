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


def test_reorder_refused_by_batch_and_server(sr, ctx):
    g = GRAPHS["rmat14w"]()
    G = ctx.load(g, reorder=True)
    try:
        with pytest.raises(sr.SeraphError) as e:
            sr.batch_run(ctx, [(G, "sssp", 0)])
        assert e.value.status == sr.SR_EINVAL
        with pytest.raises(sr.SeraphError) as e:
            sr.Server(ctx, [G], slots=8)
        assert e.value.status == sr.SR_EINVAL
    finally:
        G.close()
