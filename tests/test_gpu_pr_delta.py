"""PageRank-delta (SR_RUN_PR_DELTA): the data-driven form of Section 4.3 as
residual propagation, then the rank-form verification passes. The residual
phase alone is pinned against the oracle's partial sums of the PageRank
series (k synchronous passes reach the first k terms); whole runs end at the
PageRank fixed point within 1e-6 max-abs of the FP64 oracle (and 1e-8 on the
scale-16 workload, where the mean rank is 1.5e-5)."""
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
def ctx(sr):
    c = sr.Context(0, 0)
    yield c
    c.close()


_g = {}


def graph(name):
    if name not in _g:
        _g[name] = {"s16": graphgen.recipes.pagerank_s16, "r12": lambda: graphgen.rmat(12, 8, seed=12),
                    "u11": lambda: graphgen.uniform(11, 1 << 13, seed=5)}[name]()
    return _g[name]


@pytest.mark.parametrize("gname", ["r12", "u11"])
@pytest.mark.parametrize("seed", [-1, 3])
@pytest.mark.parametrize("stream", [False, True])
def test_residual_phase_is_the_partial_sum(sr, ctx, gname, seed, stream):
    """With prediction off and no send threshold, k passes of the residual
    phase give the first k terms of the series: stop after k passes and
    compare the ranks with the oracle's partial sum."""
    g = graph(gname)
    G = ctx.load(g)
    try:
        G.partition(3, 2)
        for k in (1, 2, 5, 12):
            st = G.run("ppr" if seed >= 0 else "pagerank", source=max(seed, 0), pvu="off", pr_delta=True,
                       max_passes=k, force_stream=stream, max_inner_iters=4, check=False)
            assert st["status"] == sr.SR_ENOTCONV and st["pr_delta_passes"] == k
            x = G.values(np.float32).astype(np.float64)
            ref = oracle.pagerank_partial(g, k, seed=seed)
            err = float(np.max(np.abs(x - ref)))
            tol = 2e-7 * max(float(ref.max()), 1e-30) * k + 1e-12
            say(f"case partial {gname} seed={seed} stream={stream} k={k}: max-abs {err:.2e} (tol {tol:.2e})")
            assert err <= tol
    finally:
        G.close()


@pytest.mark.parametrize("pvu,eps", [("off", 0.0), ("weak", 0.0), ("weak", 1e-9), ("off", 1e-8)])
@pytest.mark.parametrize("sched", ["resident", "four_pages"])
def test_pagerank_delta_s16(sr, ctx, pvu, eps, sched):
    """The scale-16 PageRank workload (4 equal-edge pages, up to 4 sweeps per
    window outside the residual phase): the FP64 fixed point within 1e-8."""
    g = graph("s16")
    ref, _, _ = oracle.pagerank(g, tol=1e-13)
    G = ctx.load(g)
    try:
        G.partition(4, 2 if sched == "four_pages" else 0, equal_edges=True)
        st = G.run("pagerank", pvu=pvu, pr_delta=True, pr_change_eps=eps, max_inner_iters=4,
                   force_stream=sched == "four_pages", tol_l1=1e-9)
        x = G.values(np.float32).astype(np.float64)
        err = float(np.max(np.abs(x - ref)))
        say(f"case delta s16 {sched} {pvu} eps={eps}: delta passes {st['pr_delta_passes']} passes {st['passes']} "
            f"verify {st['verify_passes']} sweeps {st['sweeps']} pulls {st['vertices_attempted']} max-abs {err:.2e}")
        assert st["stop_reason"] in (1, 2)
        assert st["pr_delta_passes"] > 0 and st["verify_passes"] >= 1
        assert err <= 1e-6
        assert err <= 1e-8
    finally:
        G.close()


@pytest.mark.parametrize("gname", ["r12", "u11"])
def test_ppr_delta(sr, ctx, gname):
    g = graph(gname)
    for s in (0, 17):
        ref, _, _ = oracle.pagerank(g, seed=s, tol=1e-13)
        G = ctx.load(g, reorder=True)
        try:
            G.partition(3, 4)
            for pvu in ("off", "weak"):
                st = G.run("ppr", source=s, pvu=pvu, pr_delta=True, pr_change_eps=1e-9, force_stream=True)
                x = G.values(np.float32).astype(np.float64)
                assert float(np.max(np.abs(x - ref))) <= 1e-6
                assert st["pr_delta_passes"] > 0
        finally:
            G.close()


def test_pagerank_delta_refused(sr, ctx):
    g = graphgen.rmat(10, 8, seed=3, weights=(1, 9, 3))
    G = ctx.load(g)
    try:
        for algo, kw in (("pagerank", dict(pvu="strong")), ("pagerank", dict(pvu="off", deterministic=True)),
                         ("pagerank", dict(pvu="off", audit=True)), ("sssp", dict(pvu="off")),
                         ("bfs", dict(pvu="off"))):
            with pytest.raises(sr.SeraphError) as e:
                G.run(algo, pr_delta=True, **kw)
            assert e.value.status == sr.SR_EINVAL
        G.run("pagerank", pvu="off")
        with pytest.raises(sr.SeraphError) as e:
            G.run("pagerank", pvu="off", pr_delta=True, resume=True)
        assert e.value.status == sr.SR_EINVAL
    finally:
        G.close()
