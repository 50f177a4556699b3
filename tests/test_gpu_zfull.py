"""Full-size workloads: PageRank on R-MAT scale 16 (4 equal-edge pages, up to
4 in-GPU sweeps per page per pass), streamed SSSP on R-MAT scale 22 under a
device budget of 1/4 of the graph bytes, streamed CC on R-MAT scale 24 /
edge factor 32 and its uniform twin (the benchmark's headline workload), the
256-instance batched PPR set, and a Poisson serving stream. Each result is
compared with the oracle: bit-exact for integer programs (directly, or by
the O(m) exactness certificate where the oracle cannot run per result), and
1e-6 max-abs for PageRank against the FP64 oracle's own solve of every
instance."""
import sys
import time

import numpy as np
import pytest

import graphgen
import oracle

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def sr():
    import paper_1806_00762_amd as sr
    sr.lib()
    return sr


@pytest.mark.parametrize("equal_edges", [True, False])
def test_pagerank_s16_four_pages_four_inner(sr, equal_edges):
    """4 equal-edge pages as the workload states (and the equal-byte cut the
    streamed programs use), one page resident at a time. Gate: 1e-6 max-abs
    as stated, and 1e-8 (the mean rank here is 1.5e-5, so 1e-6 alone would
    admit 7% relative error; the runs measure below 1e-9)."""
    g = graphgen.recipes.pagerank_s16()
    ref, _, _ = oracle.pagerank(g, tol=1e-13)
    with sr.Context(0, 0) as ctx:
        G = ctx.load(g)
        G.partition(4, 2, equal_edges=equal_edges)   # one page resident at a time, iterated up to 4 times
        for pvu in ("weak", "off"):
            st = G.run("pagerank", pvu=pvu, max_inner_iters=4, force_stream=True, tol_l1=1e-9)
            x = G.values(np.float32).astype(np.float64)
            err = float(np.max(np.abs(x - ref)))
            rel = float(np.max(np.abs(x - ref) / ref))
            say(f"pagerank s16 equal_edges={equal_edges} {pvu}: max-abs {err:.3e} max-rel {rel:.3e} "
                f"passes {st['passes']} stop {st['stop_reason']} L1 {st['final_l1']:.3e}")
            assert st["stop_reason"] in (1, 2)
            assert err <= 1e-6
            assert err <= 1e-8
            assert G.info()["num_parts"] == 4
        G.close()


def test_sssp_s22_streamed_quarter_budget(sr):
    t = time.time()
    g = graphgen.recipes.sssp_s22()
    ref = oracle.sssp(g, 0)
    say(f"sssp s22 gen+oracle {time.time() - t:.1f}s")
    budget = (4 * (g.n + 1) + 8 * g.m) // 4
    with sr.Context(0, budget) as ctx:
        G = ctx.load(g)
        G.partition(0, 4)
        info = G.info()
        assert info["num_parts"] >= 4 and info["resident"] == 0
        configs = [("weak", {}), ("strong", {}), ("off", {}), ("strong", {"copy_depth": 2}),
                   ("strong", {"copy_depth": 2, "hetero": True})]
        for pvu, kw in configs:
            st = G.run("sssp", source=0, pvu=pvu, max_inner_iters=8, force_stream=True, **kw)
            d = G.values()
            say(f"sssp s22 {pvu} {kw}: passes {st['passes']} h2d {st['h2d_bytes'] / 1e6:.0f} MB "
                f"wall {st['wall_ms']:.0f} ms sparse {st['sparse_stage']} frontier {st['sparse_frontier']}")
            assert np.array_equal(d, ref)
            assert st["h2d_bytes"] >= info["graph_bytes"]
            used, cap = ctx.memory()
            assert used <= cap == budget
        G.close()


def _cc_streamed(sr, g, name):
    t = time.time()
    ref = oracle.cc(g)
    say(f"{name}: union-find {time.time() - t:.1f}s, components {len(np.unique(ref))}")
    gbytes = 4 * (g.n + 1) + 4 * g.m
    # pages stream through slots worth 1/4 of the graph next to the vertex
    # state (and the host stage's in-edge bitmap, one bit per vertex)
    budget = gbytes // 4 + 5 * g.n + g.n // 8 + (1 << 20)
    with sr.Context(0, budget) as ctx:
        t = time.time()
        G = ctx.load(g, symmetric=True)
        G.partition(0, 4)
        say(f"{name}: load+partition {time.time() - t:.1f}s, pages {G.info()['num_parts']}")
        st0 = st = G.run("cc", pvu="strong", max_inner_iters=4, force_stream=True)
        lab = G.values()
        say(f"{name}: passes {st['passes']} wall {st['wall_ms']:.0f} ms h2d {st['h2d_bytes'] / 1e9:.2f} GB")
        assert np.array_equal(lab, ref)
        # with the host stage, as the CC bench legs run: device passes, then
        # the host checks the vertices the next pass would attempt (reading
        # only the values it touches when they fit half the frontier buffer,
        # else the whole array, down and back once per entry)
        st = G.run("cc", pvu="strong", max_inner_iters=8, force_stream=True, copy_depth=2, deterministic=True,
                   hetero=True)
        say(f"{name} host stage: passes {st['passes']} list {st['sparse_frontier']} rounds {st['sparse_rounds']} "
            f"relaxations {st['sparse_relaxations']} copied {st['sparse_copy_bytes']} B in {st['sparse_ms']:.2f} ms")
        assert np.array_equal(G.values(), ref)
        assert st["sparse_stage"] == 1 and st["passes"] <= st0["passes"]
        assert 0 < st["sparse_copy_bytes"] <= 8 * g.n * st["sparse_entries"]
        G.close()


def test_cc_rmat_s24_ef32_streamed(sr):
    t = time.time()
    g = graphgen.recipes.cc_rmat_s24()
    say(f"cc rmat24: generated m={g.m} in {time.time() - t:.1f}s")
    _cc_streamed(sr, g, "cc rmat24")


def test_cc_uniform_twin_s24_streamed(sr):
    t = time.time()
    g = graphgen.recipes.cc_uniform_s24()
    say(f"cc uniform24: generated m={g.m} in {time.time() - t:.1f}s")
    _cc_streamed(sr, g, "cc uniform24")


def test_batched_ppr_256_over_32_graphs(sr):
    """Every one of the 256 instances against its own FP64 oracle solve, held
    to the stated 1e-6 max-abs (the runs measure ~1.7e-7 at worst, on the
    seed vertex of a scale-19/20 graph, whose rank ~0.15-0.3 has an FP32 ulp
    of ~1.5e-8); the oracle solves run in a thread pool (the C oracle
    releases the GIL)."""
    import os
    from concurrent.futures import ThreadPoolExecutor
    graphs = [graphgen.recipes.batched_graph(i) for i in range(32)]
    with sr.Context(0, 0) as ctx:
        Gs = [ctx.load(g) for g in graphs]
        insts = [(gi, int(s)) for gi, g in enumerate(graphs)
                 for s in graphgen.sources_with_outedges(g, 8, seed=2000 + gi)]
        outs, per, bs = sr.batch_run(ctx, [(Gs[gi], "ppr", s) for gi, s in insts])
        say(f"batched ppr: {bs}")
        for G in Gs:
            G.close()
        ctx.close()
    assert all(st["converged"] == 1 for st in per)

    def err_of(k):
        gi, s = insts[k]
        ref, _, _ = oracle.pagerank(graphs[gi], seed=s, tol=1e-13)
        return float(np.max(np.abs(outs[k].view(np.float32).astype(np.float64) - ref)))

    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    t = time.time()
    # largest graphs first, so the pool ends together
    order = sorted(range(len(insts)), key=lambda k: -graphs[insts[k][0]].m)
    with ThreadPoolExecutor(workers) as ex:
        errs = dict(zip(order, ex.map(err_of, order)))
    worst = max(errs.values())
    say(f"batched ppr: {len(errs)} instances vs the FP64 oracle in {time.time() - t:.1f}s "
        f"({workers} threads): worst max-abs {worst:.3e}")
    assert len(errs) == 256
    assert worst <= 1e-6


def test_serving_stream_three_graphs(sr):
    """1,500 Poisson arrivals at 2,000/s over the three resident graphs. Every
    result on the scale-20 graph and a seeded sample of 100 per larger graph
    is checked bit-exact: by the exactness certificate (O(m): d[src] = 0, no
    edge violates d[v] <= d[u] + w, every reached vertex has a tight in-edge,
    unreached ones no reached in-neighbour), and every 50th of them against
    the oracle's own Dijkstra / BFS as well."""
    graphs = [graphgen.recipes.serving_graph(s) for s in (20, 22, 23)]
    nreq = 1500
    arr = graphgen.poisson_arrivals(2000.0, nreq, seed=4000)
    pick = graphgen.bounded_draws(4001, 1, nreq, 0, 2)
    kind = graphgen.bounded_draws(4002, 1, nreq, 0, 1)
    srcs = [graphgen.sources_with_outedges(graphs[gi], nreq, seed=4003 + gi) for gi in range(3)]
    reqs = [(int(pick[i]), "sssp" if kind[i] == 0 else "bfs", int(srcs[int(pick[i])][i])) for i in range(nreq)]
    check = set(i for i in range(nreq) if reqs[i][0] == 0)
    for gi in (1, 2):
        on = [i for i in range(nreq) if reqs[i][0] == gi]
        take = graphgen.bounded_draws(4100 + gi, 1, 100, 0, len(on) - 1)
        check |= set(on[int(t)] for t in take)
    n_checked = {0: 0, 1: 0, 2: 0}
    with sr.Context(0, 0) as ctx:
        Gs = [ctx.load(g, reorder=True) for g in graphs]
        srv = sr.Server(ctx, Gs, slots=64)
        t0 = time.time()
        tickets = []
        for i, (gi, algo, s) in enumerate(reqs):
            while time.time() - t0 < arr[i]:
                time.sleep(0.0001)
            tickets.append(srv.submit(gi, algo, s))
        t_sub = time.time() - t0
        pending = set(range(nreq))
        lat = {}
        bufs = [np.empty(g.n, dtype=np.uint32) for g in graphs]
        direct = 0
        while pending and time.time() - t0 < 300:
            for i in sorted(pending):
                gi, algo, s = reqs[i]
                out = bufs[gi] if i in check else None
                done, l = srv.poll(tickets[i], out)
                if not done:
                    continue
                lat[i] = l
                pending.discard(i)
                if out is None:
                    continue
                cert = oracle.sssp_certificate(graphs[gi], s, out, weights=(algo == "sssp"))
                assert cert == 0, (i, gi, algo, s, cert)
                n_checked[gi] += 1
                if n_checked[gi] % 50 == 1:
                    ref = oracle.sssp(graphs[gi], s) if algo == "sssp" else oracle.bfs(graphs[gi], s)
                    assert np.array_equal(out, ref), (i, gi, algo, s)
                    direct += 1
            time.sleep(0.0005)
        elapsed = time.time() - t0
        assert not pending
        v = np.array(list(lat.values()))
        say(f"serving: submitted over {t_sub:.2f} s, all done after {elapsed:.2f} s; p50 {np.percentile(v, 50):.1f} ms "
            f"p99 {np.percentile(v, 99):.1f} ms; certified {n_checked}, {direct} also vs the oracle; {srv.stats()}")
        assert n_checked[0] == sum(1 for r in reqs if r[0] == 0)
        assert n_checked[1] >= 90 and n_checked[2] >= 90   # 100 seeded draws, a few repeats
        srv.close()
        for G in Gs:
            G.close()
