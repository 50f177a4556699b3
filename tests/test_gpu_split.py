"""Split-width streamed pages: a streamed BFS/SSSP/CC run copies page images
whose in-edges from source ids below 2^16 are u16 ids (u8 weights) ahead of
the wide ones. Results must equal the oracle's exactly with split and with
full-width pages, on graphs where both parts are present (n above 2^16), on
graphs whose ids are all narrow, with degree numbering, in tiles and in
heavy chunks (forced with split_pages, since the default takes them only
when they are smaller); the default must take them on a degree-numbered
R-MAT graph and carry fewer bytes over the host link."""
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


def star(leaves, weights=None):
    """Undirected star, centre 0: the centre's in-edges span narrow and wide
    ids (leaves above 2^16 - 1) and are pulled in heavy chunks."""
    src = np.zeros(leaves, dtype=np.int64)
    dst = np.arange(1, leaves + 1, dtype=np.int64)
    w = None
    if weights:
        w = (np.arange(leaves, dtype=np.int64) * 7919 % 200 + 1).astype(np.uint32)
    return graphgen.from_edges(leaves + 1, src, dst, w, symmetrize=True)


GRAPHS = {  # builder, programs, load keywords
    "rmat18w": (lambda: graphgen.rmat(18, 8, seed=18, weights=(1, 255, 7)), ("bfs", "sssp"), {}),
    "rmat18u_sym": (lambda: graphgen.rmat(18, 8, seed=5, symmetrize=True), ("bfs", "cc"),
                    {"symmetric": True}),
    "uniform13w": (lambda: graphgen.uniform(13, 1 << 16, seed=13, weights=(1, 255, 3)), ("bfs", "sssp"),
                   {}),
    "star70000w": (lambda: star(70000, weights=True), ("bfs", "sssp", "cc"), {"symmetric": True}),
    # unweighted: the wide ids of the images are 3 bytes (tiles and heavy chunks)
    "star70000u": (lambda: star(70000), ("bfs", "cc"), {"symmetric": True}),
}
SCHED = {"s4p7d2": (7, 4, 2), "s3p3d1": (3, 3, 1)}
_cache = {}


def graph(name):
    if name not in _cache:
        _cache[name] = GRAPHS[name][0]()
    return _cache[name]


def ref(algo, g, s):
    if algo == "bfs":
        return oracle.bfs(g, s)
    if algo == "sssp":
        return oracle.sssp(g, s)
    return oracle.cc(g)


@pytest.mark.parametrize("sched", list(SCHED))
@pytest.mark.parametrize("gname", list(GRAPHS))
@pytest.mark.parametrize("reorder", [False, True])
def test_split_pages_exact(sr, ctx, gname, sched, reorder):
    g = graph(gname)
    _, progs, lkw = GRAPHS[gname]
    parts, slots, depth = SCHED[sched]
    G = ctx.load(g, reorder=reorder, **lkw)
    try:
        G.partition(parts, slots)
        srcs = [0] + [int(s) for s in graphgen.sources_with_outedges(g, 2, seed=11)]
        for algo in progs:
            for s in (srcs if algo != "cc" else [0]):
                say(f"case {gname} {sched} reorder={reorder} {algo} source {s}")
                want = ref(algo, g, s)
                kw = dict(source=s, force_stream=True, copy_depth=depth)
                a = G.run(algo, split_pages=True, **kw)
                va = G.values()
                b = G.run(algo, wide_pages=True, **kw)
                vb = G.values()
                assert np.array_equal(va, want), (gname, sched, algo, s)
                assert np.array_equal(vb, want), (gname, sched, algo, s)
                assert b["edges_narrow"] == 0
                assert 0 < a["edges_narrow"] <= a["edges_scanned"], (a["edges_narrow"], a["edges_scanned"])
                say(f"  narrow {a['edges_narrow']} of {a['edges_scanned']}; "
                    f"h2d split {a['h2d_bytes']} wide {b['h2d_bytes']}")
    finally:
        G.close()


def test_split_pages_carry_fewer_bytes(sr, ctx):
    """Without prediction every pass copies every page and reads every edge:
    same passes, so the split run (taken by default here) moves fewer bytes
    over the link and reads part of its edges as u16 ids."""
    g = graphgen.rmat(18, 16, seed=7)
    G = ctx.load(g, reorder=True)
    try:
        G.partition(6, 4)
        a = G.run("bfs", source=0, pvu="off", force_stream=True, copy_depth=2, max_inner_iters=1)
        assert a["edges_narrow"] > 0
        va = G.values()
        b = G.run("bfs", source=0, pvu="off", force_stream=True, copy_depth=2, max_inner_iters=1,
                  wide_pages=True)
        assert np.array_equal(va, oracle.bfs(g, 0))
        assert np.array_equal(G.values(), va)
        say(f"passes {a['passes']} / {b['passes']}; h2d {a['h2d_bytes']} / {b['h2d_bytes']}; "
            f"algo bytes {a['algo_bytes']} / {b['algo_bytes']}")
        if a["passes"] == b["passes"] and a["sweeps"] == b["sweeps"]:
            assert a["h2d_bytes"] < b["h2d_bytes"]
            assert a["edges_scanned"] == b["edges_scanned"]
            assert a["algo_bytes"] < b["algo_bytes"]
            frac = a["edges_narrow"] / a["edges_scanned"]
            assert 0.0 < frac < 1.0
    finally:
        G.close()


def test_split_not_for_resident_or_pagerank(sr, ctx):
    """Resident runs and PageRank read the full-width pages."""
    g = graphgen.rmat(14, 16, seed=3, weights=(1, 255, 7))
    G = ctx.load(g)
    try:
        G.partition(1, 4)
        st = G.run("sssp", source=0)
        assert st["edges_narrow"] == 0
        assert np.array_equal(G.values(), oracle.sssp(g, 0))
        G.partition(5, 3)
        st = G.run("pagerank", force_stream=True, copy_depth=1)
        assert st["edges_narrow"] == 0
        st = G.run("sssp", source=0, force_stream=True, copy_depth=1, split_pages=True)
        assert st["edges_narrow"] > 0
        assert np.array_equal(G.values(), oracle.sssp(g, 0))
        for kw in (dict(wide_pages=True, split_pages=True), dict(algo="pagerank", split_pages=True)):
            algo = kw.pop("algo", "sssp")
            st = G.run(algo, source=0, force_stream=True, copy_depth=1, check=False, **kw)
            assert st["status"] == sr.SR_EINVAL, (algo, kw)
        G.partition(1, 4)
        st = G.run("sssp", source=0, split_pages=True, check=False)
        assert st["status"] == sr.SR_EINVAL
    finally:
        G.close()


def boundary_graph():
    """Sources on both sides of the narrow limit (65534..65537) and at the
    ends of the id range, into: a chain that needs many passes, a vertex with
    exactly the heavy bound of in-edges (2048: still in a tile), one just
    above it (2049: two chunks) and one with 5000, each mixing narrow and
    wide sources; plus a 4096-edge tile of 2048 + 2048 in-edges."""
    n = 70000
    rng = np.random.default_rng(65536)
    src, dst = [], []
    for a, b in ((0, 65534), (65534, 65535), (65535, 65536), (65536, 65537), (65537, 69999),
                 (69999, 1), (1, 65535), (65536, 2)):
        src.append(a); dst.append(b)
    for v, d in ((3, 2048), (4, 2049), (5, 5000), (6, 2048), (7, 2048)):
        s = rng.choice(np.arange(8, n), size=d, replace=False)
        src.extend(s.tolist()); dst.extend([v] * d)
    # every vertex gets three in-edges from random sources
    t = np.arange(8, n)
    for _ in range(3):
        src.extend(rng.integers(0, n, size=t.size).tolist()); dst.extend(t.tolist())
    src = np.array(src); dst = np.array(dst)
    w = rng.integers(1, 256, size=src.size).astype(np.uint32)
    return graphgen.from_edges(n, src, dst, w)


@pytest.mark.parametrize("parts,slots,depth", [(3, 3, 1), (6, 4, 2)])
@pytest.mark.parametrize("reorder", [False, True])
def test_split_pages_boundaries(sr, ctx, parts, slots, depth, reorder):
    g = boundary_graph()
    G = ctx.load(g, reorder=reorder)
    try:
        G.partition(parts, slots)
        for algo in ("bfs", "sssp"):
            for s in (0, 65535, 65536, 69999):
                say(f"case boundary parts={parts} reorder={reorder} {algo} source {s}")
                want = ref(algo, g, s)
                for pvu in ("strong", "off"):
                    kw = dict(source=s, pvu=pvu, force_stream=True, copy_depth=depth)
                    st = G.run(algo, split_pages=True, **kw)
                    assert np.array_equal(G.values(), want), (algo, s, pvu)
                    assert st["edges_narrow"] > 0
                    G.run(algo, wide_pages=True, **kw)
                    assert np.array_equal(G.values(), want), (algo, s, pvu)
    finally:
        G.close()
