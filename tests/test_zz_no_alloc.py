"""The allocation-free solve (sr_run_noalloc) against sr_run on the same
resident graphs: two calls in a row, the second on a smaller graph, for
SSSP (weak and strong prediction), BFS and CC. Values go to torch-allocated
device buffers; results must be bit-identical to sr_run's and to the
oracle's, and the library's device-memory account must not move."""
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
def torch():
    import torch
    torch.cuda.init()
    return torch


def _solve_pair(sr, torch, ctx, G, g, algo, pvu, source, ref):
    """sr_run, then sr_run_noalloc into torch buffers, on one resident graph."""
    st = G.run(algo, source=source, pvu=pvu)
    assert st["status"] == 0
    want = G.values()
    assert np.array_equal(want, ref), (algo, pvu, "sr_run vs oracle")
    vals = torch.full((g.n,), -7, dtype=torch.int32, device="cuda:0")
    stat = torch.full((g.n,), 0xAB, dtype=torch.uint8, device="cuda:0")
    torch.cuda.synchronize()
    used0, _ = ctx.memory()
    st2 = G.run_noalloc(algo, vals.data_ptr(), stat.data_ptr() if pvu == "weak" else 0,
                        source=source, pvu=pvu)
    used1, _ = ctx.memory()
    got = vals.cpu().numpy().view(np.uint32)
    say(f"noalloc {algo} {pvu} n={g.n}: passes {st2['passes']} (sr_run {st['passes']}), "
        f"edges {st2['edges_scanned']}, stop {st2['stop_reason']}")
    assert used1 == used0
    assert st2["stop_reason"] == 1
    assert np.array_equal(got, want), (algo, pvu, int(np.sum(got != want)))
    return st2


@pytest.mark.parametrize("algo,pvu", [("sssp", "weak"), ("sssp", "strong"), ("bfs", "strong"),
                                      ("cc", "strong"), ("sssp", "off")])
def test_noalloc_matches_sr_run_two_calls(sr, torch, algo, pvu):
    big = graphgen.rmat(14, 16, seed=41, weights=(1, 255, 141))
    small = graphgen.rmat(10, 8, seed=42, weights=(1, 255, 142))
    sym = algo == "cc"
    with sr.Context(0, 0) as ctx:
        for g in (big, small):   # the second call has the smaller input
            G = ctx.load(g, symmetrize=sym)
            if algo == "sssp":
                ref = oracle.sssp(g, 0)
            elif algo == "bfs":
                ref = oracle.bfs(g, 0)
            else:
                ref = oracle.cc(g)
            _solve_pair(sr, torch, ctx, G, g, algo, pvu, 0, ref)
            G.close()


def test_noalloc_refusals(sr, torch):
    """Argument checks: a streamed (not resident) graph, a reordered graph,
    PageRank, weak prediction without a state buffer, a refused flag."""
    g = graphgen.rmat(10, 8, seed=43, weights=(1, 255, 143))
    vals = torch.zeros(g.n, dtype=torch.int32, device="cuda:0")
    with sr.Context(0, 0) as ctx:
        G = ctx.load(g)
        with pytest.raises(sr.SeraphError) as e:
            G.run_noalloc("sssp", vals.data_ptr(), source=0, pvu="strong")
        assert e.value.status == sr.SR_ESTATE
        G.run("sssp", source=0, pvu="strong", force_stream=True)
        with pytest.raises(sr.SeraphError) as e:
            G.run_noalloc("sssp", vals.data_ptr(), source=0, pvu="strong")
        assert e.value.status == sr.SR_ESTATE
        G.run("sssp", source=0, pvu="strong")
        for kw in ({"algo": "pagerank"}, {"algo": "sssp", "pvu": "weak"},
                   {"algo": "sssp", "pvu": "strong", "force_stream": True}):
            with pytest.raises(sr.SeraphError) as e:
                G.run_noalloc(kw.pop("algo"), vals.data_ptr(), source=0, **kw)
            assert e.value.status == sr.SR_EINVAL
        G.close()
        G = ctx.load(g, reorder=True)
        G.run("sssp", source=0, pvu="strong")
        with pytest.raises(sr.SeraphError) as e:
            G.run_noalloc("sssp", vals.data_ptr(), source=0, pvu="strong")
        assert e.value.status == sr.SR_EINVAL
        G.close()
