"""Continuous-batching query server: queries admitted while others run give
exactly the result they give alone (solo sr_run) and the oracle's."""
import time

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


def wait_all(srv, tickets, outs, timeout=60.0):
    lat = {}
    t0 = time.time()
    pending = set(tickets)
    while pending and time.time() - t0 < timeout:
        for t in list(pending):
            done, l = srv.poll(t, outs[t])
            if done:
                lat[t] = l
                pending.discard(t)
        time.sleep(0.0005)
    assert not pending, f"{len(pending)} queries not done"
    return lat


@pytest.mark.parametrize("slots", [8, 16, 32, 64])
def test_server_alone_vs_mix(sr, slots):
    # the scale-16 graph has vertices of in-degree above 2048 (heavy chunks,
    # split over several wavefronts for the wider slot groups)
    graphs = [graphgen.rmat(12, 16, seed=81, weights=(1, 255, 82)),
              graphgen.rmat(14, 8, seed=83, weights=(1, 255, 84)),
              graphgen.rmat(16, 16, seed=85, weights=(1, 255, 86))]
    ctx = sr.Context(0, 0)
    Gs = [ctx.load(g) for g in graphs]
    srv = sr.Server(ctx, Gs, state_budget_bytes=0, slots=slots)
    say(f"case server slots={slots} stats {srv.stats()}")
    reqs = []
    r = np.random.default_rng(slots)
    for i in range(60):
        gi = int(r.integers(0, 3))
        algo = "sssp" if r.random() < 0.5 else "bfs"
        src = int(graphgen.sources_with_outedges(graphs[gi], 1, seed=100 + i)[0])
        reqs.append((gi, algo, src))
    tickets, outs = [], {}
    # first wave, then a second wave submitted while the first is running
    for k, (gi, algo, src) in enumerate(reqs):
        t = srv.submit(gi, algo, src)
        tickets.append(t)
        outs[t] = np.empty(graphs[gi].n, dtype=np.uint32)
        if k == 30:
            time.sleep(0.002)
    lat = wait_all(srv, tickets, outs)
    st = srv.stats()
    say(f"  stats {st}; p50 {np.percentile(list(lat.values()), 50):.2f} ms")
    assert st["completed"] == len(reqs)
    for t, (gi, algo, src) in zip(tickets, reqs):
        ref = oracle.sssp(graphs[gi], src) if algo == "sssp" else oracle.bfs(graphs[gi], src)
        assert np.array_equal(outs[t], ref), (gi, algo, src)
    srv.close()
    # alone: the same queries through sr_run one at a time
    for t, (gi, algo, src) in list(zip(tickets, reqs))[:10]:
        Gs[gi].run(algo, source=src)
        assert np.array_equal(Gs[gi].values(), outs[t])
    for G in Gs:
        G.close()
    ctx.close()


def test_server_rejects_bad_requests(sr):
    g = graphgen.rmat(10, 8, seed=5)  # unweighted: SSSP refused, BFS fine
    ctx = sr.Context(0, 0)
    G = ctx.load(g)
    srv = sr.Server(ctx, [G], slots=8)
    with pytest.raises(sr.SeraphError):
        srv.submit(0, "sssp", 0)
    with pytest.raises(sr.SeraphError):
        srv.submit(1, "bfs", 0)
    with pytest.raises(sr.SeraphError):
        srv.submit(0, "bfs", g.n)
    t = srv.submit(0, "bfs", 0)
    out = np.empty(g.n, dtype=np.uint32)
    lat = wait_all(srv, [t], {t: out})
    assert np.array_equal(out, oracle.bfs(g, 0))
    srv.close()
    G.close()
    ctx.close()


def test_server_wide_distances_completed_exactly(sr):
    """Served slots hold 16-bit values below 32767. On a weighted path
    (weight 250 per hop) the vertices past hop 131 lie at distance 32767 or
    more; queries from its start overflow their slot and are completed on the
    host when they retire, a query from hop 300 does not. A second path has
    weights above the 16-bit range (separate u32 weights, clamped in the
    packed relaxation): every query on it overflows at once. Every result
    stays bit-exact (BFS levels fit), and the stats count the completions;
    queries on a small graph in the same server do not need it."""
    n = 400
    src = list(range(n - 1)) + [0]
    dst = list(range(1, n)) + [n - 1]
    w = [250] * (n - 1) + [255]
    path = graphgen.from_edges(n, src, dst, w)
    small = graphgen.rmat(10, 8, seed=91, weights=(1, 255, 92))
    nh = 40
    heavy = graphgen.from_edges(nh, list(range(nh - 1)), list(range(1, nh)),
                                [(40000, 5, 30000, 70000, 1)[i % 5] for i in range(nh - 1)])
    ctx = sr.Context(0, 0)
    Gs = [ctx.load(path), ctx.load(small, reorder=True), ctx.load(heavy)]
    srv = sr.Server(ctx, Gs, slots=8)
    reqs = [(0, "sssp", 0), (0, "sssp", 3), (1, "sssp", 0), (1, "bfs", 1), (0, "bfs", 0), (0, "sssp", 300),
            (2, "sssp", 0), (2, "sssp", 1), (2, "bfs", 0)]
    tickets, outs = [], {}
    for gi, algo, s in reqs:
        t = srv.submit(gi, algo, s)
        tickets.append(t)
        outs[t] = np.empty(Gs[gi].n, dtype=np.uint32)
    wait_all(srv, tickets, outs)
    st = srv.stats()
    say(f"  wide distances: stats {st}")
    graphs = [path, small, heavy]
    for t, (gi, algo, s) in zip(tickets, reqs):
        ref = oracle.sssp(graphs[gi], s) if algo == "sssp" else oracle.bfs(graphs[gi], s)
        assert np.array_equal(outs[t], ref), (gi, algo, s)
    # sources 0 and 3 reach distances beyond 32766 along the path, 300 does not
    assert int(oracle.sssp(path, 0)[n - 2]) > 32766
    assert int(oracle.sssp(path, 300).max()) == 0xFFFFFFFF  # (vertices before 300 unreached)
    assert int(oracle.sssp(path, 300)[n - 2]) < 32767
    assert st["narrow_fallbacks"] >= 4
    srv.close()
    for G in Gs:
        G.close()
    ctx.close()
