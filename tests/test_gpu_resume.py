"""SR_RUN_RESUME: a run stopped by max_passes (SR_ENOTCONV, partial values
readable) continues from its values and predictor states to the same result
as a run from scratch: bit-exact for the min programs, within 1e-6 of the
FP64 oracle for PageRank (whose rank and dangling sums are taken from the
resumed ranks)."""
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


@pytest.mark.parametrize("stream", [False, True])
@pytest.mark.parametrize("algo,pvu", [("sssp", "strong"), ("sssp", "weak"), ("bfs", "strong"), ("cc", "strong")])
def test_resume_min_programs(sr, ctx, algo, pvu, stream):
    g = graphgen.rmat(13, 16, seed=91, weights=(1, 255, 92), symmetrize=(algo == "cc"))
    G = ctx.load(g, symmetric=(algo == "cc"))
    try:
        G.partition(5 if stream else 1, 3)
        s = 0 if algo == "cc" else int(graphgen.sources_with_outedges(g, 1, seed=93)[0])
        ref = oracle.cc(g) if algo == "cc" else (oracle.sssp(g, s) if algo == "sssp" else oracle.bfs(g, s))
        say(f"case resume {algo} {pvu} stream={stream}")
        kw = dict(source=s, pvu=pvu, force_stream=stream, max_inner_iters=1)
        st = G.run(algo, max_passes=1, check=False, **kw)
        part = G.values()
        assert st["passes"] >= 1
        st2 = G.run(algo, resume=True, **kw)
        assert np.array_equal(G.values(), ref)
        if st["converged"] == 0:
            # the first pass left work for the resumed run
            assert not np.array_equal(part, ref) or st2["passes"] >= 1
    finally:
        G.close()


@pytest.mark.parametrize("algo", ["pagerank", "ppr"])
def test_resume_pagerank(sr, ctx, algo):
    g = graphgen.rmat(13, 16, seed=94)
    G = ctx.load(g)
    try:
        G.partition(4, 4)
        s = int(graphgen.sources_with_outedges(g, 1, seed=95)[0])
        ref, _, _ = oracle.pagerank(g, seed=(s if algo == "ppr" else -1), tol=1e-13)
        st = G.run(algo, source=s, pvu="off", max_passes=3, check=False)
        assert st["converged"] == 0
        x3 = G.values().view(np.float32).astype(np.float64)
        assert np.max(np.abs(x3 - ref)) > 1e-6
        G.run(algo, source=s, pvu="off", resume=True)
        x = G.values().view(np.float32).astype(np.float64)
        err = float(np.max(np.abs(x - ref)))
        say(f"case resume {algo}: max-abs {err:.2e}")
        assert err <= 1e-6
        assert abs(x.sum() - 1.0) < 1e-5
    finally:
        G.close()


def test_resume_needs_a_run_of_the_same_program(sr, ctx):
    g = graphgen.rmat(10, 8, seed=96, weights=(1, 255, 97))
    G = ctx.load(g)
    try:
        with pytest.raises(sr.SeraphError):
            G.run("sssp", source=0, resume=True)
        G.run("bfs", source=0)
        with pytest.raises(sr.SeraphError):
            G.run("sssp", source=0, resume=True)
    finally:
        G.close()
