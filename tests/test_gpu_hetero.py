"""Heterogeneous execution (Section 3.1): the device runs dense pull passes
and, once a pass changes few vertices, the host continues with push
relaxations from that pass's frontier; with weak prediction the switch first
runs an all-pull verification pass (Section 4.3), and a host frontier that
grows dense again sends the run back to the device. The result must equal
the oracle exactly, whatever the switch point, predictor, schedule or
graph."""
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
_cache = {}


def graph(name):
    if name not in _cache:
        _cache[name] = GRAPHS[name]()
    return _cache[name]


SCHED = {
    "resident": dict(parts=1, slots=4, force=False, depth=0),
    "s3p3": dict(parts=3, slots=3, force=True, depth=1),
    "s4p7d2": dict(parts=7, slots=4, force=True, depth=2),
}


def run(ctx, g, algo, sched, sym=False, source=0, **kw):
    s = SCHED[sched]
    G = ctx.load(g, symmetrize=sym)
    try:
        G.partition(s["parts"], s["slots"])
        st = G.run(algo, source=source, max_inner_iters=4, force_stream=s["force"], copy_depth=s["depth"],
                   hetero=True, max_passes=5000, **kw)
        st["records"] = G.sweeps()
        return G.values(), st
    finally:
        G.close()


@pytest.mark.parametrize("gname", list(GRAPHS))
@pytest.mark.parametrize("sched", list(SCHED))
@pytest.mark.parametrize("switch", [0, 64, 1 << 30])
@pytest.mark.parametrize("det", [False, True])
def test_hetero_exact(sr, ctx, gname, sched, switch, det):
    """det: the deterministic window schedule (the device keeps a sweep
    queued ahead of the host) under the sparse stage's pass-end handovers."""
    g = graph(gname)
    src = int(np.argmax(np.diff(g.offsets)))
    cases = (("sssp", oracle.sssp(g, src), False), ("bfs", oracle.bfs(g, src), False), ("cc", oracle.cc(g), True))
    for algo, ref, sym in cases:
        for pvu in ("strong", "off", "weak"):
            got, st = run(ctx, g, algo, sched, sym=sym, source=src, pvu=pvu, sparse_switch=switch,
                          deterministic=det)
            say(f"case hetero {gname} {sched} switch={switch} {algo} {pvu}: passes {st['passes']} "
                f"sparse {st['sparse_stage']} frontier {st['sparse_frontier']} rounds {st['sparse_rounds']}")
            assert st["converged"] == 1
            assert np.array_equal(got, ref), f"{algo} {pvu}: {np.sum(got != ref)} mismatches"
            if switch == 1 << 30 and pvu == "strong" and sched != "resident":
                # streamed under strong prediction: the vertices the second
                # pass would attempt (at most n) go to the host after the first
                assert st["sparse_stage"] == 1 and st["passes"] == 1
    if switch == 1 << 30:
        # a switch threshold above n hands over once a pass's changes fit it
        # (weak prediction: after the verification pass that follows such a
        # pass, unless that verification pass changed nothing and so ended
        # the run on the device)
        recs = st["records"]
        last = [r for r in recs if r["pass"] == recs[-1]["pass"]]
        ended_on_device = recs[-1]["phase"] == 1 and all(r["changed"] == 0 for r in last)
        assert st["sparse_stage"] == 1 or ended_on_device


def test_hetero_triggers_and_saves_passes(sr, ctx):
    g = graph("rmat14w")
    src = int(np.argmax(np.diff(g.offsets)))
    G = ctx.load(g)
    try:
        G.partition(7, 4)
        base = G.run("sssp", source=src, pvu="strong", force_stream=True)
        ref = G.values()
        het = G.run("sssp", source=src, pvu="strong", force_stream=True, hetero=True, sparse_switch=2048)
        assert np.array_equal(G.values(), ref)
        assert np.array_equal(ref, oracle.sssp(g, src))
        say(f"case hetero passes {het['passes']} vs {base['passes']}, frontier {het['sparse_frontier']}")
        assert het["sparse_stage"] == 1
        assert het["passes"] < base["passes"]
        # (the stage may start from an empty list: then the pass before it
        # left no vertex to attempt)
        assert 0 <= het["sparse_frontier"] <= 2048
    finally:
        G.close()


def test_hetero_refused_cases(sr, ctx):
    g = graph("rmat14w")
    G = ctx.load(g)
    try:
        G.partition(1, 4)
        for algo, pvu in (("pagerank", "weak"), ("pagerank", "off")):
            with pytest.raises(sr.SeraphError) as e:
                G.run(algo, source=0, pvu=pvu, hetero=True)
            assert e.value.status == sr.SR_EINVAL
        with pytest.raises(sr.SeraphError):
            G.run("sssp", source=0, pvu="strong", hetero=True, sparse_switch=-1)
        with pytest.raises(sr.SeraphError):
            G.run("sssp", source=0, pvu="strong", hetero=True, sparse_return=-1)
        with pytest.raises(sr.SeraphError) as e:
            G.run("sssp", source=0, pvu="weak", skip_clean=True, force_stream=True)
        assert e.value.status == sr.SR_EINVAL
        st = G.run("sssp", source=0, hetero=True)  # default prediction becomes strong
        assert np.array_equal(G.values(), oracle.sssp(g, 0))
    finally:
        G.close()


def test_hetero_tiny_graphs(sr, ctx):
    cases = [
        graphgen.from_edges(1, [], [], []),
        graphgen.from_edges(2, [0], [1], [5]),
        graphgen.from_edges(5, [0, 1, 2, 3], [1, 2, 3, 4], [1, 2, 3, 4]),
        graphgen.from_edges(4, [1, 2], [2, 3], [7, 7]),
    ]
    for g in cases:
        for sched in ("resident", "s3p3"):
            got, _ = run(ctx, g, "sssp", sched, pvu="strong", sparse_switch=1 << 30)
            assert np.array_equal(got, oracle.sssp(g, 0))
            got, _ = run(ctx, g, "cc", sched, sym=True, pvu="strong", sparse_switch=1 << 30)
            assert np.array_equal(got, oracle.cc(g))


def test_hetero_weak_switch_after_verification(sr, ctx):
    """Weak prediction (the paper's SSSP default): the switch runs one
    verification pass with prediction off and hands its frontier to the
    host, which finishes exactly."""
    g = graph("rmat14w")
    src = int(np.argmax(np.diff(g.offsets)))
    ref = oracle.sssp(g, src)
    G = ctx.load(g)
    try:
        G.partition(7, 4)
        for sched_kw in (dict(force_stream=True, copy_depth=2), dict(force_stream=False)):
            st = G.run("sssp", source=src, pvu="weak", hetero=True, sparse_switch=2048, **sched_kw)
            tr = G.sweeps()
            say(f"case weak hetero {sched_kw}: passes {st['passes']} verify {st['verify_passes']} "
                f"entries {st['sparse_entries']} frontier {st['sparse_frontier']}")
            assert np.array_equal(G.values(), ref)
            assert st["sparse_stage"] == 1 and st["sparse_entries"] >= 1
            # the last device pass was a verification pass
            assert tr[-1]["phase"] == 1
            assert st["verify_passes"] >= 1
    finally:
        G.close()


def chain_fan(n_leaves=5000, chain=300, pad=700, seed=31):
    """A chain that runs against the sweep order (from the highest id down)
    and then fans out to every leaf: device passes change a few chain
    vertices each, the host walks the chain one vertex per round, and the
    fan makes its frontier dense again."""
    n = n_leaves + pad + chain
    top = n - 1
    src = list(range(top, top - chain + 1, -1))
    dst = list(range(top - 1, top - chain, -1))
    hub = top - chain + 1
    src += [hub] * n_leaves
    dst += list(range(n_leaves))
    # leaves point back into the chain's first part, so the return also has work to do
    rng = np.random.default_rng(seed)
    extra_s = rng.integers(0, n_leaves, 2000)
    extra_d = rng.integers(0, n_leaves, 2000)
    src += extra_s.tolist()
    dst += extra_d.tolist()
    w = rng.integers(1, 10, len(src)).tolist()
    return graphgen.from_edges(n, src, dst, w), top


@pytest.mark.parametrize("sched", ["resident", "s3p3", "s4p7d2"])
def test_hetero_two_way_switch(sr, ctx, sched):
    """The host stage gives the run back to the device when its frontier
    passes sparse_return, and takes it again later: SSSP and BFS bit-exact
    with every predictor, with at least one return."""
    g, src = chain_fan()
    for algo, ref in (("sssp", oracle.sssp(g, src)), ("bfs", oracle.bfs(g, src))):
        for pvu in ("strong", "off", "weak"):
            got, st = run(ctx, g, algo, sched, source=src, pvu=pvu, sparse_switch=64, sparse_return=256)
            say(f"case two-way {sched} {algo} {pvu}: passes {st['passes']} entries {st['sparse_entries']} "
                f"returns {st['sparse_returns']} rounds {st['sparse_rounds']} finished {st['sparse_stage']}")
            assert np.array_equal(got, ref), f"{algo} {pvu}: {np.sum(got != ref)} mismatches"
            assert st["converged"] == 1
            assert st["sparse_returns"] >= 1
            assert st["sparse_entries"] >= st["sparse_returns"]


OPEN_GRAPHS = {
    "rmat16_sym": (lambda: graphgen.rmat(16, 16, seed=61, symmetrize=True), ("cc", "bfs")),
    "uniform16_sym": (lambda: graphgen.uniform(16, 1 << 20, seed=62, symmetrize=True), ("cc", "bfs")),
    "rmat16w": (lambda: graphgen.rmat(16, 8, seed=63, weights=(1, 255, 64)), ("sssp", "bfs")),
}


@pytest.mark.parametrize("gname", list(OPEN_GRAPHS))
@pytest.mark.parametrize("sched", ["s3p3", "s4p7d2"])
@pytest.mark.parametrize("reorder", [False, True])
def test_hetero_open_list(sr, ctx, gname, sched, reorder):
    """Streamed runs under strong prediction enter the host stage from the
    list of vertices the next pass would attempt (an in-edge and a value
    above the Table I threshold) once it is short, even when the pass before
    changed far more vertices: the host pulls them and pushes from those that
    changed. Bit-exact against the oracle, with no more device passes than
    without the host stage; CC on the R-MAT graph ends after one pass."""
    g = _open_graph(gname)
    s = SCHED[sched]
    src = int(np.argmax(np.diff(g.offsets)))
    for algo in OPEN_GRAPHS[gname][1]:
        ref = oracle.cc(g) if algo == "cc" else (oracle.sssp(g, src) if algo == "sssp" else oracle.bfs(g, src))
        G = ctx.load(g, reorder=reorder, symmetric=algo == "cc")
        try:
            G.partition(s["parts"], s["slots"])
            kw = dict(source=src, pvu="strong", force_stream=True, copy_depth=s["depth"], max_inner_iters=8,
                      deterministic=True)
            base = G.run(algo, **kw)
            assert np.array_equal(G.values(), ref)
            het = G.run(algo, hetero=True, sparse_switch=1024, **kw)
            say(f"case open {gname} {sched} reorder={reorder} {algo}: passes {het['passes']} (without "
                f"{base['passes']}) entries {het['sparse_entries']} list {het['sparse_frontier']} rounds "
                f"{het['sparse_rounds']} finished {het['sparse_stage']}")
            assert np.array_equal(G.values(), ref), f"{algo}: {np.sum(G.values() != ref)} mismatches"
            assert het["converged"] == 1
            assert het["passes"] <= base["passes"]
            if algo == "cc" and gname == "rmat16_sym":
                assert het["sparse_stage"] == 1 and het["passes"] == 1
        finally:
            G.close()


_open_cache = {}


def _open_graph(name):
    if name not in _open_cache:
        _open_cache[name] = OPEN_GRAPHS[name][0]()
    return _open_cache[name]


def layered(pad=20000, seed=71):
    """Leaves C (ids 0-899) below B (900-1199) below A (1200-1799) below the
    source 1800, then isolated padding: SSSP/BFS/CC need three layers of
    relaxations, and a push from any pass's changed set stays within the
    1,801 connected vertices."""
    rng = np.random.default_rng(seed)
    nc, nb, na = 900, 300, 600
    src_id = nc + nb + na
    s = [src_id] * na + list(range(nc + nb, src_id)) + [nc + j // 3 for j in range(nc)]
    d = list(range(nc + nb, src_id)) + [nc + i % nb for i in range(na)] + list(range(nc))
    w = rng.integers(1, 10, len(s)).tolist()
    return graphgen.from_edges(src_id + 1 + pad, s, d, w), src_id


@pytest.mark.parametrize("sched", ["resident", "s3p3"])
def test_hetero_short_push(sr, ctx, sched):
    """A host push that stays small fetches the values it reads and writes
    back only the lowered ones: bit-exact, finished on the host, with fewer
    value bytes moved than one copy of the value array (the whole-array path
    moves two)."""
    g, src = layered()
    for algo, sym in (("sssp", False), ("bfs", False), ("cc", True)):
        ref = oracle.cc(g) if algo == "cc" else (oracle.sssp(g, src) if algo == "sssp" else oracle.bfs(g, src))
        for pvu in ("strong", "off", "weak"):
            got, st = run(ctx, g, algo, sched, sym=sym, source=src, pvu=pvu, sparse_switch=g.n)
            say(f"case short push {sched} {algo} {pvu}: passes {st['passes']} entries {st['sparse_entries']} "
                f"rounds {st['sparse_rounds']} relaxations {st['sparse_relaxations']} "
                f"copied {st['sparse_copy_bytes']} B finished {st['sparse_stage']}")
            assert np.array_equal(got, ref), f"{algo} {pvu}: {np.sum(got != ref)} mismatches"
            assert st["converged"] == 1
            if pvu == "weak":
                # entered only after a verification pass, from a frontier that
                # may need more round trips than the short path allows: then
                # it falls back to copying the array both ways, after at most
                # half the frontier buffer's worth of fetched values
                assert st["sparse_copy_bytes"] <= 8 * g.n * max(1, st["sparse_entries"]) + 4 * g.n
                continue
            assert st["sparse_stage"] == 1
            assert 0 < st["sparse_copy_bytes"] < 4 * g.n

