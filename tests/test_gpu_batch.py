"""Batched multi-instance runs through sr_batch_run: every instance equals
its oracle (PPR within 1e-6 max-abs, SSSP/BFS bit-exact) and its solo run."""
import sys

import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


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


def test_batched_ppr_uneven_graphs(sr, ctx):
    graphs = [graphgen.rmat(s, ef, seed=500 + s) for s, ef in ((10, 8), (12, 16), (13, 32), (11, 8))]
    Gs = [ctx.load(g) for g in graphs]
    insts = []
    for gi, g in enumerate(graphs):
        # 11 instances on some graphs: one full group of 8 and a partial group
        k = 11 if gi % 2 == 0 else 5
        for s in graphgen.sources_with_outedges(g, k, seed=2000 + gi):
            insts.append((gi, int(s)))
    say(f"case batched ppr {len(insts)} instances over {len(graphs)} graphs")
    outs, per, bs = sr.batch_run(ctx, [(Gs[gi], "ppr", s) for gi, s in insts])
    say(f"  batch stats {bs}")
    worst = 0.0
    for (gi, s), x, st in zip(insts, outs, per):
        ref, _, _ = oracle.pagerank(graphs[gi], seed=s, tol=1e-13)
        err = float(np.max(np.abs(x.view(np.float32).astype(np.float64) - ref)))
        worst = max(worst, err)
        assert st["converged"] == 1
        assert err <= 1e-6, (gi, s, err)
    say(f"  worst max-abs {worst:.3e}")
    for G in Gs:
        G.close()


def test_batched_sssp_bfs_mix_matches_oracle_and_solo(sr, ctx):
    graphs = [graphgen.rmat(12, 16, seed=61, weights=(1, 255, 62)), graphgen.rmat(14, 8, seed=63, weights=(1, 255, 64))]
    Gs = [ctx.load(g) for g in graphs]
    insts = []
    for gi, g in enumerate(graphs):
        for j, s in enumerate(graphgen.sources_with_outedges(g, 10, seed=3000 + gi)):
            insts.append((gi, "sssp" if j % 2 == 0 else "bfs", int(s)))
    say(f"case batched sssp/bfs {len(insts)}")
    outs, per, bs = sr.batch_run(ctx, [(Gs[gi], a, s) for gi, a, s in insts])
    for (gi, a, s), x, st in zip(insts, outs, per):
        ref = oracle.sssp(graphs[gi], s) if a == "sssp" else oracle.bfs(graphs[gi], s)
        assert np.array_equal(x, ref), (gi, a, s, int(np.sum(x != ref)))
    # solo runs agree bit-for-bit
    for gi, a, s in insts[:4]:
        Gs[gi].run(a, source=s)
        assert np.array_equal(Gs[gi].values(), outs[insts.index((gi, a, s))])
    for G in Gs:
        G.close()


def test_batched_pvu_off_equals_strong(sr, ctx):
    g = graphgen.rmat(12, 16, seed=71, weights=(1, 255, 72))
    G = ctx.load(g)
    srcs = [int(s) for s in graphgen.sources_with_outedges(g, 8, seed=9)]
    a, _, _ = sr.batch_run(ctx, [(G, "sssp", s) for s in srcs], pvu="off")
    b, _, _ = sr.batch_run(ctx, [(G, "sssp", s) for s in srcs], pvu="strong")
    for x, y, s in zip(a, b, srcs):
        assert np.array_equal(x, y)
        assert np.array_equal(x, oracle.sssp(g, s))
    G.close()


def test_batched_interleaved_graphs_and_sizes(sr, ctx):
    """Instances listed alternately over graphs of different sizes (results
    are extracted one group at a time; every instance must still get its own
    column of its own graph)."""
    graphs = [graphgen.rmat(13, 8, seed=81, weights=(1, 255, 82)), graphgen.uniform(11, 1 << 14, seed=83,
                                                                                   weights=(1, 255, 84))]
    Gs = [ctx.load(g, reorder=(gi == 1)) for gi, g in enumerate(graphs)]
    srcs = [[int(s) for s in graphgen.sources_with_outedges(g, 11, seed=85 + gi)] for gi, g in enumerate(graphs)]
    insts = []
    for j in range(11):
        for gi in (0, 1):
            insts.append((gi, "sssp" if (j + gi) % 2 == 0 else "bfs", srcs[gi][j]))
    say(f"case batched interleaved {len(insts)}")
    outs, _, _ = sr.batch_run(ctx, [(Gs[gi], a, s) for gi, a, s in insts])
    for (gi, a, s), x in zip(insts, outs):
        ref = oracle.sssp(graphs[gi], s) if a == "sssp" else oracle.bfs(graphs[gi], s)
        assert np.array_equal(x, ref), (gi, a, s)
    outs, _, _ = sr.batch_run(ctx, [(Gs[gi], "ppr", s) for gi, _, s in insts[:10]])
    for (gi, _, s), x in zip(insts[:10], outs):
        ref, _, _ = oracle.pagerank(graphs[gi], seed=s, tol=1e-13)
        assert np.max(np.abs(x.view(np.float32).astype(np.float64) - ref)) <= 1e-6, (gi, s)
    for G in Gs:
        G.close()


@pytest.mark.parametrize("family,K,rounds", [("ppr", 8, 2), ("ppr", 16, 8), ("ppr", 16, 4),
                                             ("min", 8, 8), ("min", 16, 2), ("min", 32, 4), ("min", 32, 8)])
def test_batched_schedule_widths_and_rounds(sr, ctx, family, K, rounds, monkeypatch):
    """Every group width and vertex-rounds choice the autotuner can pick gives
    the oracle's results: PPR within 1e-6 max-abs, SSSP/BFS bit-exact
    (SR_BATCH_SCHEDULE fixes K and rounds; grid and grab are still tuned)."""
    monkeypatch.setenv("SR_BATCH_SCHEDULE", f"{K},{rounds}")
    graphs = [graphgen.rmat(11, 16, seed=71, weights=(1, 255, 72)), graphgen.rmat(13, 8, seed=73, weights=(1, 255, 74))]
    Gs = [ctx.load(g, reorder=gi == 1) for gi, g in enumerate(graphs)]
    insts = []
    for gi, g in enumerate(graphs):
        for j, s in enumerate(graphgen.sources_with_outedges(g, 19, seed=3000 + gi)):
            algo = "ppr" if family == "ppr" else ("sssp" if j % 2 == 0 else "bfs")
            insts.append((gi, algo, int(s)))
    say(f"case batched schedule {family} K={K} rounds={rounds}")
    outs, per, bs = sr.batch_run(ctx, [(Gs[gi], a, s) for gi, a, s in insts])
    assert bs["group_width"] == K and bs["rounds"] == rounds
    for (gi, a, s), x, st in zip(insts, outs, per):
        assert st["converged"] == 1
        if a == "ppr":
            ref, _, _ = oracle.pagerank(graphs[gi], seed=s, tol=1e-13)
            assert float(np.max(np.abs(x.view(np.float32).astype(np.float64) - ref))) <= 1e-6
        else:
            ref = oracle.sssp(graphs[gi], s) if a == "sssp" else oracle.bfs(graphs[gi], s)
            assert np.array_equal(x, ref), (gi, a, s)
    for G in Gs:
        G.close()


def test_batched_autotuner_times_every_width(sr, ctx, monkeypatch):
    """Without a fixed schedule the first call times every group width (a
    fresh workload signature), picks one, and a repeat call takes it from the
    cache; results stay bit-exact."""
    monkeypatch.delenv("SR_BATCH_SCHEDULE", raising=False)
    g = graphgen.rmat(12, 12, seed=81, weights=(1, 255, 82))
    G = ctx.load(g)
    srcs = [int(s) for s in graphgen.sources_with_outedges(g, 32, seed=3100)]
    outs, per, bs = sr.batch_run(ctx, [(G, "sssp", s) for s in srcs])
    say(f"  first call schedule {bs}")
    assert bs["width_candidates"] == 3 and bs["tuned"] == 1
    assert bs["group_width"] in (8, 16, 32) and bs["rounds"] in (2, 4, 8)
    outs2, _, bs2 = sr.batch_run(ctx, [(G, "sssp", s) for s in srcs])
    assert bs2["width_candidates"] == 1 and bs2["tuned"] == 0
    assert (bs2["group_width"], bs2["rounds"], bs2["grid_blocks"], bs2["grab"]) == \
        (bs["group_width"], bs["rounds"], bs["grid_blocks"], bs["grab"])
    for s, x, x2 in zip(srcs, outs, outs2):
        ref = oracle.sssp(g, s)
        assert np.array_equal(x, ref) and np.array_equal(x2, ref)
    G.close()
