"""Pins for the SSSP and BFS oracle: brute force, exhaustive enumeration,
certificates and their rejection of mutated answers."""
import itertools

import numpy as np
import pytest

import graphgen
import oracle

INF = oracle.INF


def floyd_warshall(n, src, dst, w):
    d = np.full((n, n), np.inf)
    np.fill_diagonal(d, 0.0)
    for u, v, ww in zip(src, dst, w):
        d[u, v] = min(d[u, v], ww)
    for k in range(n):
        d = np.minimum(d, d[:, k:k + 1] + d[k:k + 1, :])
    return d


@pytest.mark.parametrize("trial", range(60))
def test_dijkstra_matches_floyd_warshall(trial):
    r = np.random.default_rng(1000 + trial)
    n = int(r.integers(1, 9))
    m = int(r.integers(0, n * n + 1))
    src = r.integers(0, n, m); dst = r.integers(0, n, m); w = r.integers(1, 6, m)
    g = graphgen.from_edges(n, src, dst, w)
    es = np.repeat(np.arange(n), np.diff(g.offsets))
    fw = floyd_warshall(n, es, g.col, g.weights.astype(float))
    for s in range(n):
        d = oracle.sssp(g, s)
        exp = np.where(np.isinf(fw[s]), INF, fw[s]).astype(np.uint64)
        assert np.array_equal(d.astype(np.uint64), exp)
        assert oracle.sssp_certificate(g, s, d) == 0


def test_bellman_ford_equals_dijkstra_rmat():
    g = graphgen.rmat(13, 16, seed=21, weights=(1, 255, 5))
    for s in (0, 5, 77):
        d = oracle.sssp(g, s)
        bf, rounds = oracle.sssp_bellman_ford(g, s)
        assert np.array_equal(d, bf)
        assert oracle.sssp_certificate(g, s, d) == 0


def test_triangle_inequality_every_edge():
    g = graphgen.rmat(14, 16, seed=22, weights=(1, 255, 122))
    d = oracle.sssp(g, 0).astype(np.uint64)
    es = np.repeat(np.arange(g.n), np.diff(g.offsets))
    fin = d[es] != INF
    assert np.all(d[g.col[fin]] <= d[es[fin]] + g.weights[fin])
    assert np.any(d != INF) and d[0] == 0


def test_certificate_rejects_mutations():
    g = graphgen.rmat(10, 8, seed=3, weights=(1, 255, 4))
    d = oracle.sssp(g, 0)
    assert oracle.sssp_certificate(g, 0, d) == 0
    reach = np.nonzero((d != INF) & (np.arange(g.n) != 0))[0]
    r = np.random.default_rng(0)
    for v in r.choice(reach, size=min(20, reach.size), replace=False):
        for delta in (-1, 1):
            bad = d.copy(); bad[v] = np.uint32(int(bad[v]) + delta)
            assert oracle.sssp_certificate(g, 0, bad) != 0
    unreached = np.nonzero(d == INF)[0]
    if unreached.size:
        bad = d.copy(); bad[unreached[0]] = 5
        assert oracle.sssp_certificate(g, 0, bad) != 0
    reached = reach[0]
    bad = d.copy(); bad[reached] = INF
    assert oracle.sssp_certificate(g, 0, bad) != 0


def bfs_by_matrix_powers(n, adj, s):
    """Level of v = smallest k with (A^k)[s, v] > 0 (boolean powers)."""
    lvl = np.full(n, INF, dtype=np.uint64)
    frontier = np.zeros(n, dtype=bool); frontier[s] = True
    reach = frontier.copy(); lvl[s] = 0
    for k in range(1, n):
        frontier = (adj[frontier].any(axis=0)) & ~reach
        if not frontier.any():
            break
        lvl[frontier] = k
        reach |= frontier
    return lvl


def test_bfs_exhaustive_directed_n4():
    """All 2^12 directed graphs on 4 vertices, every source."""
    n = 4
    pairs = [(u, v) for u in range(n) for v in range(n) if u != v]
    for mask in range(1 << len(pairs)):
        es = [pairs[i] for i in range(len(pairs)) if mask >> i & 1]
        adj = np.zeros((n, n), dtype=bool)
        for u, v in es:
            adj[u, v] = True
        g = graphgen.from_edges(n, [u for u, _ in es], [v for _, v in es])
        for s in range(n):
            got = oracle.bfs(g, s).astype(np.uint64)
            assert np.array_equal(got, bfs_by_matrix_powers(n, adj, s)), (mask, s)


def test_bfs_equals_unit_weight_sssp():
    g = graphgen.rmat(13, 16, seed=8, weights=(1, 255, 9))
    for s in (0, 3):
        b = oracle.bfs(g, s)
        assert np.array_equal(b, oracle.sssp(g, s, weights=False))
        assert oracle.sssp_certificate(g, s, b, weights=False) == 0
