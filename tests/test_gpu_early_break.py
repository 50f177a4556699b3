"""BFS early break in the dense pull (strong prediction): a vertex whose first
in-neighbour sits on the threshold level k takes level k + 1 without reading
its other in-edges. Levels must equal the oracle's exactly, with and without
the break, on every schedule; the break must read fewer edges where first
in-neighbours are hubs (degree numbering), in tiles and in heavy chunks."""
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


def star(leaves):
    """Undirected star: centre 0, leaves 1..leaves (the centre's in-degree
    exceeds the heavy-vertex bound, so its pull runs in chunks)."""
    src = np.zeros(leaves, dtype=np.int64)
    dst = np.arange(1, leaves + 1, dtype=np.int64)
    return graphgen.from_edges(leaves + 1, src, dst, symmetrize=True)


GRAPHS = {
    "rmat14": lambda: graphgen.rmat(14, 16, seed=14),
    "uniform12": lambda: graphgen.uniform(12, 1 << 15, seed=9),
    "star5000": lambda: star(5000),
    "grid64": lambda: graphgen.grid(64, 64),
}
SCHED = {"resident": (1, 4, False, 0), "s4p7d2": (7, 4, True, 2), "s3p3": (3, 3, True, 1)}
_cache = {}


def graph(name):
    if name not in _cache:
        _cache[name] = GRAPHS[name]()
    return _cache[name]


@pytest.mark.parametrize("sched", list(SCHED))
@pytest.mark.parametrize("gname", list(GRAPHS))
@pytest.mark.parametrize("reorder", [False, True])
def test_early_break_levels_exact(sr, ctx, gname, sched, reorder):
    g = graph(gname)
    parts, slots, stream, depth = SCHED[sched]
    G = ctx.load(g, reorder=reorder)
    try:
        G.partition(parts, slots)
        srcs = [0, 1] + [int(s) for s in graphgen.sources_with_outedges(g, 2, seed=3)]
        for s in srcs:
            say(f"case {gname} {sched} reorder={reorder} source {s}")
            ref = oracle.bfs(g, s)
            kw = dict(source=s, pvu="strong", force_stream=stream, copy_depth=depth)
            on = G.run("bfs", **kw)
            a = G.values()
            off = G.run("bfs", early_break=False, **kw)
            b = G.values()
            assert np.array_equal(a, ref), (gname, sched, s)
            assert np.array_equal(b, ref), (gname, sched, s)
            say(f"  edges read: break {on['edges_scanned']} full {off['edges_scanned']}")
    finally:
        G.close()


def test_early_break_reads_fewer_edges(sr, ctx):
    """Resident BFS on a degree-numbered R-MAT graph from its hub: each sweep
    closes a pass, so level k + 1 vertices mostly stop at their first
    in-neighbour."""
    g = graphgen.rmat(16, 16, seed=16)
    G = ctx.load(g, reorder=True)
    try:
        G.partition(1, 4)
        on = G.run("bfs", source=0, pvu="strong")
        a = G.values()
        off = G.run("bfs", source=0, pvu="strong", early_break=False)
        assert np.array_equal(a, oracle.bfs(g, 0))
        assert np.array_equal(G.values(), a)
        say(f"edges read: break {on['edges_scanned']} full {off['edges_scanned']}")
        assert on["edges_scanned"] < 0.6 * off["edges_scanned"]
    finally:
        G.close()


def test_early_break_heavy_chunks(sr, ctx):
    """The star's centre (in-degree 5000) is pulled in chunks, and its first
    in-neighbour is leaf 1: from leaf 1 every chunk stops at the probe, from
    the other sources the chunks read their edges; levels stay exact."""
    g = star(5000)
    G = ctx.load(g)
    try:
        G.partition(1, 4)
        for s in (1, 2, 4999, 5000, 0):
            G.run("bfs", source=s, pvu="strong")
            assert np.array_equal(G.values(), oracle.bfs(g, s)), s
    finally:
        G.close()


def test_early_break_only_under_strong_prediction(sr, ctx):
    """Without prediction every resident sweep reads every in-edge (the break
    needs Table I's threshold); weak prediction's levels match too."""
    g = graph("rmat14")
    G = ctx.load(g, reorder=True)
    try:
        G.partition(1, 4)
        ref = oracle.bfs(g, 0)
        st = G.run("bfs", source=0, pvu="off")
        assert np.array_equal(G.values(), ref)
        assert st["edges_scanned"] == st["sweeps"] * G.info()["m"]
        G.run("bfs", source=0, pvu="weak")
        assert np.array_equal(G.values(), ref)
    finally:
        G.close()
