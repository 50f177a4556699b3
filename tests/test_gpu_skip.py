"""Page skipping on streamed passes: a pass copies and sweeps only the pages
an edge from a vertex changed in the previous pass enters. Results must stay
exact; on a lattice (locality, high diameter) most page visits are skipped."""
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


def solve(ctx, g, algo, parts, slots, sym=False, source=0, **kw):
    G = ctx.load(g, symmetrize=sym)
    try:
        G.partition(parts, slots)
        st = G.run(algo, source=source, max_inner_iters=4, force_stream=True, max_passes=20000, **kw)
        return G.values(), st
    finally:
        G.close()


@pytest.mark.parametrize("layout", [(6, 3, 1), (9, 4, 2)])
def test_skip_lattice_exact_and_saves_copies(sr, ctx, layout):
    parts, slots, depth = layout
    g = graphgen.grid(96, 96, weights=(1, 9, 11))
    for algo, ref, sym in (("sssp", oracle.sssp(g, 0), False), ("bfs", oracle.bfs(g, 0), False),
                           ("cc", oracle.cc(g), True)):
        for pvu in ("strong", "off"):
            got, st = solve(ctx, g, algo, parts, slots, sym=sym, pvu=pvu, copy_depth=depth, skip_clean=True)
            base_vals, base = solve(ctx, g, algo, parts, slots, sym=sym, pvu=pvu, copy_depth=depth)
            say(f"case skip lattice {layout} {algo} {pvu}: passes {st['passes']} vs {base['passes']}, "
                f"skipped {st['pages_skipped']}, h2d {st['h2d_bytes']} vs {base['h2d_bytes']}")
            assert np.array_equal(got, ref), f"{algo} {pvu}: {np.sum(got != ref)} mismatches"
            assert np.array_equal(base_vals, ref)
            assert st["converged"] == 1
            if algo != "cc":
                assert st["pages_skipped"] > 0
                assert st["h2d_bytes"] < base["h2d_bytes"]


@pytest.mark.parametrize("det", [False, True])
def test_skip_rmat_exact(sr, ctx, det):
    g = graphgen.rmat(14, 16, seed=14, weights=(1, 255, 5))
    src = int(np.argmax(np.diff(g.offsets)))
    for algo, ref, sym in (("sssp", oracle.sssp(g, src), False), ("bfs", oracle.bfs(g, src), False),
                           ("cc", oracle.cc(g), True)):
        got, st = solve(ctx, g, algo, 7, 4, sym=sym, source=src, pvu="strong", copy_depth=2, skip_clean=True,
                        deterministic=det)
        say(f"case skip rmat14 det={det} {algo}: passes {st['passes']} skipped {st['pages_skipped']}")
        assert np.array_equal(got, ref)


def test_skip_with_sparse_stage(sr, ctx):
    g = graphgen.grid(64, 64, weights=(1, 9, 12))
    got, st = solve(ctx, g, "sssp", 6, 3, pvu="strong", skip_clean=True, hetero=True, sparse_switch=256)
    assert np.array_equal(got, oracle.sssp(g, 0))
    assert st["sparse_stage"] == 1


def test_skip_refused_and_resident(sr, ctx):
    g = graphgen.grid(32, 32, weights=(1, 9, 13))
    G = ctx.load(g)
    try:
        G.partition(4, 3)
        for algo, pvu in (("sssp", "weak"), ("pagerank", "weak")):
            with pytest.raises(sr.SeraphError) as e:
                G.run(algo, source=0, pvu=pvu, force_stream=True, skip_clean=True)
            assert e.value.status == sr.SR_EINVAL
        st = G.run("sssp", source=0, force_stream=True, skip_clean=True)  # default prediction: strong
        assert np.array_equal(G.values(), oracle.sssp(g, 0))
        G.partition(1, 4)
        st = G.run("sssp", source=0, pvu="strong", skip_clean=True)  # resident: nothing to skip
        assert st["pages_skipped"] == 0
        assert np.array_equal(G.values(), oracle.sssp(g, 0))
    finally:
        G.close()
