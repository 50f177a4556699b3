"""Subgraph schedules of Section 3.2 / Section 5.4 through the C ABI.

Schedules compared (all on streamed pages, prediction off unless stated):
  baseline  -- two slots, one sweep per page per pass (each page once)
  rsi       -- two slots, a fixed number of sweeps per page (CLIP's loaded
               data re-entry, maximum re-entry times MRT)
  psi_fixed -- S slots, the window of S-1 pages swept a fixed number of times
  psi       -- S slots, adaptive re-entry (until the copy lands / no change)

Every schedule must reach the oracle's exact result; the per-sweep trace
(sr_run_sweeps) must add up to the run's totals; and on the two-page
alternating chain that Section 3.2 uses to show the limit of re-entry, re-entry
gains nothing over the baseline while the pipelined window cuts the passes."""
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


SCHEDULES = {
    "baseline": dict(slots=2, inner=1, fixed=True),
    "rsi": dict(slots=2, inner=3, fixed=True),
    "psi_fixed": dict(slots=4, inner=3, fixed=True),
    "psi": dict(slots=4, inner=8, fixed=False),
}


def run(ctx, g, algo, sched, parts, pvu="off", source=0, symmetrize=False, slots=None):
    s = SCHEDULES[sched]
    G = ctx.load(g, symmetrize=symmetrize)
    try:
        G.partition(parts, slots or s["slots"])
        st = G.run(algo, source=source, pvu=pvu, max_inner_iters=s["inner"], force_stream=True,
                   fixed_inner=s["fixed"], max_passes=5000)
        return G.values(), st, G.sweeps()
    finally:
        G.close()


def zigzag(h):
    """Chain a0 -> b0 -> a1 -> b1 -> ... with a_i = i in the low half of the ids
    and b_i = h + i in the high half, so consecutive hops alternate pages."""
    src, dst = [], []
    for i in range(h):
        src.append(i)
        dst.append(h + i)
        if i + 1 < h:
            src.append(h + i)
            dst.append(i + 1)
    return graphgen.from_edges(2 * h, src, dst, [1] * len(src))


def check_trace(st, tr):
    assert len(tr) == st["sweeps"]
    assert sum(r["edges"] for r in tr) == st["edges_scanned"]
    assert sum(r["attempted"] for r in tr) == st["vertices_attempted"]
    assert sum(r["skipped"] for r in tr) == st["vertices_skipped"]
    passes = [r["pass"] for r in tr]
    assert passes == sorted(passes)
    assert passes[-1] == st["passes"] - 1
    for i in range(8):
        assert sum(r["state_hist"][i] for r in tr) == st["state_hist"][i]


def test_zigzag_reentry_vs_pipelined(sr, ctx):
    g = zigzag(48)
    ref = oracle.bfs(g, 0)
    res = {}
    for sched in ("baseline", "rsi", "psi_fixed"):
        # psi_fixed on two pages: three slots, a window of both pages
        got, st, tr = run(ctx, g, "bfs", sched, parts=2, slots=3 if sched == "psi_fixed" else None)
        say(f"case zigzag {sched}: passes {st['passes']} sweeps {st['sweeps']}")
        assert np.array_equal(got, ref)
        check_trace(st, tr)
        res[sched] = st
    # re-entry of a lone page cannot advance a chain that leaves the page
    # (the page split puts b0 on a's page: one hop of gain at most)
    assert res["rsi"]["passes"] >= res["baseline"]["passes"] - 1
    assert res["rsi"]["sweeps"] > 2 * res["baseline"]["sweeps"]
    # the window of both pages advances >= 4 hops a pass instead of 2
    assert 3 * res["psi_fixed"]["passes"] <= 2 * res["rsi"]["passes"]


@pytest.mark.parametrize("sched", list(SCHEDULES))
def test_schedules_min_programs(sr, ctx, sched):
    g = graphgen.rmat(14, 16, seed=14, weights=(1, 255, 5))
    src = int(np.argmax(np.diff(g.offsets)))
    for algo, ref, sym in (("sssp", oracle.sssp(g, src), False), ("bfs", oracle.bfs(g, src), False),
                           ("cc", oracle.cc(g), True)):
        say(f"case schedule {sched} {algo}")
        got, st, tr = run(ctx, g, algo, sched, parts=6, source=src, symmetrize=sym)
        assert np.array_equal(got, ref), f"{np.sum(got != ref)} mismatches"
        check_trace(st, tr)
        say(f"  passes {st['passes']} sweeps {st['sweeps']} edges {st['edges_scanned']}")


@pytest.mark.parametrize("sched", list(SCHEDULES))
def test_schedules_pagerank(sr, ctx, sched):
    g = graphgen.rmat(14, 16, seed=14)
    ref, _, _ = oracle.pagerank(g, tol=1e-13)
    say(f"case schedule {sched} pagerank")
    got, st, tr = run(ctx, g, "pagerank", sched, parts=5)
    x = got.view(np.float32).astype(np.float64)
    assert np.max(np.abs(x - ref)) <= 1e-6
    check_trace(st, tr)
    last = sum(r["l1"] for r in tr if r["pass"] == st["passes"] - 1)
    assert abs(last - st["final_l1"]) <= 1e-12 + 1e-6 * st["final_l1"]


def test_weak_predictor_trace(sr, ctx):
    """Weak prediction (Section 4.3): vertices enter the dormant states and are
    skipped; a verification sweep (phase 1) runs before the stop."""
    g = graphgen.rmat(14, 16, seed=14, weights=(1, 255, 5))
    got, st, tr = run(ctx, g, "sssp", "psi_fixed", parts=6, pvu="weak")
    assert np.array_equal(got, oracle.sssp(g, 0))
    check_trace(st, tr)
    assert any(r["phase"] == 1 for r in tr)
    assert tr[-1]["phase"] == 1 and tr[-1]["changed"] == 0
    dormant = [sum(r["state_hist"][2:5]) for r in tr]
    assert max(dormant) > 0 and dormant[0] == 0
    assert sum(r["skipped"] for r in tr if r["phase"] == 0) > 0
    assert all(r["skipped"] == 0 for r in tr if r["phase"] == 1)


@pytest.mark.parametrize("depth", [2, 3])
def test_copy_depth(sr, ctx, depth):
    """More copies in flight (a window of num_slots - depth pages) reach the
    same fixed point; depth >= num_slots is refused."""
    g = graphgen.rmat(14, 16, seed=14, weights=(1, 255, 5))
    src = int(np.argmax(np.diff(g.offsets)))
    for algo, ref, sym in (("sssp", oracle.sssp(g, src), False), ("cc", oracle.cc(g), True)):
        G = ctx.load(g, symmetrize=sym)
        try:
            G.partition(7, 4)
            say(f"case copy depth {depth} {algo}")
            for pvu in ("strong", "weak"):
                st = G.run(algo, source=src, pvu=pvu, max_inner_iters=4, force_stream=True, copy_depth=depth)
                assert np.array_equal(G.values(), ref), (algo, pvu)
                assert st["converged"] == 1
        finally:
            G.close()
    G = ctx.load(g)
    try:
        G.partition(7, 4)
        with pytest.raises(sr.SeraphError) as e:
            G.run("sssp", source=src, force_stream=True, copy_depth=4)
        assert e.value.status == sr.SR_EINVAL
    finally:
        G.close()
