"""Pins for the connected-components oracle and for the Table I strong
thresholds: exhaustive small graphs, invariants, the Section 4.1 example."""
import itertools
import json
import os

import numpy as np
import pytest

import graphgen
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def closure_labels(n, adj):
    """Label = smallest vertex reachable in the undirected graph (Warshall closure)."""
    r = adj | adj.T | np.eye(n, dtype=bool)
    for k in range(n):
        r = r | (r[:, k:k + 1] & r[k:k + 1, :])
    return np.array([np.nonzero(r[v])[0].min() for v in range(n)], dtype=np.uint32)


def test_cc_exhaustive_undirected_n5():
    """All 2^10 undirected graphs on 5 vertices."""
    n = 5
    pairs = list(itertools.combinations(range(n), 2))
    for mask in range(1 << len(pairs)):
        es = [pairs[i] for i in range(len(pairs)) if mask >> i & 1]
        adj = np.zeros((n, n), dtype=bool)
        for u, v in es:
            adj[u, v] = True
        g = graphgen.from_edges(n, [u for u, _ in es], [v for _, v in es], symmetrize=True)
        lab = oracle.cc(g)
        assert np.array_equal(lab, closure_labels(n, adj)), mask
        assert oracle.cc_check(g, lab) == 0


def test_cc_directed_input_taken_as_undirected():
    # one direction only: the oracle still joins both endpoints
    g = graphgen.from_edges(4, [3, 2], [1, 0])
    assert oracle.cc(g).tolist() == [0, 1, 0, 1]


def test_cc_invariants_rmat_and_labelprop_fixed_point():
    g = graphgen.rmat(13, 8, seed=6, symmetrize=True)
    lab = oracle.cc(g)
    assert oracle.cc_check(g, lab) == 0
    lp, _, _ = oracle.cc_labelprop_sync(g, 200)
    assert np.array_equal(lp, lab)
    # number of labels = number of components from scipy
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import connected_components
    a = csr_matrix((np.ones(g.m), g.col, g.offsets), shape=(g.n, g.n))
    ncomp, _ = connected_components(a, directed=False)
    assert len(np.unique(lab)) == ncomp


def test_cc_check_rejects_mutations():
    g = graphgen.rmat(10, 8, seed=1, symmetrize=True)
    lab = oracle.cc(g)
    bad = lab.copy(); v = int(np.nonzero(lab != np.arange(g.n))[0][0]); bad[v] = v
    assert oracle.cc_check(g, bad) != 0
    bad = lab.copy(); bad[0] = 1
    assert oracle.cc_check(g, bad) != 0


def test_section_4_1_worked_example():
    fx = json.load(open(os.path.join(GOLDEN, "cc_example_sec4_1.json")))
    e = np.array(fx["undirected_edges"])
    g = graphgen.from_edges(fx["n"], e[:, 0], e[:, 1], symmetrize=True)
    _, hist, _ = oracle.cc_labelprop_sync(g, fx["iterations"])
    for v, expect in fx["expect_labels_after_iteration"].items():
        assert hist[:, int(v)].tolist() == expect, v


def test_strong_cc_threshold_reading():
    """Table I defines s via component-size histograms; the engine uses the
    minimum new label among vertices that changed. Both agree on every pair
    of consecutive synchronous iterations of random graphs."""
    r = np.random.default_rng(5)
    for trial in range(40):
        n = int(r.integers(2, 40)); m = int(r.integers(1, 3 * n))
        g = graphgen.from_edges(n, r.integers(0, n, m), r.integers(0, n, m), symmetrize=True)
        _, hist, _ = oracle.cc_labelprop_sync(g, n + 1)
        seq = [np.arange(n, dtype=np.uint32)] + list(hist)
        for k in range(1, len(seq)):
            prev, cur = seq[k - 1], seq[k]
            changed = cur != prev
            alt = int(cur[changed].min()) if changed.any() else oracle.INF
            assert oracle.strong_threshold_cc(prev, cur) == alt
            assert oracle.strong_threshold_sssp(prev, cur) == alt


def test_strong_thresholds_sound_synchronous():
    """Table I soundness on synchronous runs: a vertex meeting the condition
    before iteration k never changes afterwards (BFS: value <= k-1 after k-1
    iterations; SSSP: value <= l; CC: label <= s)."""
    r = np.random.default_rng(9)
    for trial in range(25):
        n = int(r.integers(2, 30)); m = int(r.integers(1, 4 * n))
        s_, d_ = r.integers(0, n, m), r.integers(0, n, m)
        gw = graphgen.from_edges(n, s_, d_, r.integers(1, 9, m))
        # synchronous SSSP trajectory (numpy, from the definition)
        es = np.repeat(np.arange(n), np.diff(gw.offsets))
        cur = np.full(n, oracle.INF, dtype=np.uint64); cur[0] = 0
        traj = [cur.copy()]
        for _ in range(n + 1):
            nxt = cur.copy()
            fin = cur[es] != oracle.INF
            np.minimum.at(nxt, gw.col[fin], cur[es[fin]] + gw.weights[fin])
            traj.append(nxt); cur = nxt
        final = traj[-1]
        assert np.array_equal(final.astype(np.uint32), oracle.sssp(gw, 0))
        for k in range(2, len(traj)):
            l = oracle.strong_threshold_sssp(traj[k - 2].astype(np.uint32), traj[k - 1].astype(np.uint32))
            conv = traj[k - 1] <= l
            assert np.array_equal(traj[k - 1][conv], final[conv])
        # BFS levels
        cur = np.full(n, oracle.INF, dtype=np.uint64); cur[0] = 0
        for k in range(1, n + 1):
            nxt = cur.copy()
            fin = cur[es] != oracle.INF
            np.minimum.at(nxt, gw.col[fin], cur[es[fin]] + 1)
            cur = nxt
            t = oracle.strong_threshold_bfs(k)
            lv = oracle.bfs(gw, 0).astype(np.uint64)
            conv = cur <= t
            assert np.array_equal(cur[conv], lv[conv])


def test_labelprop_treats_arcs_as_undirected():
    # one-directional input: propagation must still cross every arc both ways
    g = graphgen.rmat(11, 4, seed=13)
    lp, _, _ = oracle.cc_labelprop_sync(g, 400)
    assert np.array_equal(lp, oracle.cc(g))
    chain = graphgen.from_edges(5, [4, 3, 2, 1], [3, 2, 1, 0])
    lp, _, _ = oracle.cc_labelprop_sync(chain, 5)
    assert lp.tolist() == [0, 0, 0, 0, 0]


def test_parallel_labelprop_equals_closure_and_union_find():
    """The multi-core CPU baseline (OpenMP synchronous label propagation) is
    pinned to the Warshall closure on every undirected graph on 5 vertices,
    to union-find on R-MAT / uniform graphs with isolated vertices, and gives
    the same labels and iteration count whatever the thread count; on a path
    0-1-...-k its iteration count is the diameter bound k + 1 (k rounds move
    label 0 to the far end, one more sees no change)."""
    n = 5
    pairs = list(itertools.combinations(range(n), 2))
    for mask in range(0, 1 << len(pairs), 7):
        es = [pairs[i] for i in range(len(pairs)) if mask >> i & 1]
        adj = np.zeros((n, n), dtype=bool)
        for u, v in es:
            adj[u, v] = True
        g = graphgen.from_edges(n, [u for u, _ in es], [v for _, v in es], symmetrize=True)
        lab, _, _ = oracle.cc_labelprop_parallel(g, threads=2)
        assert np.array_equal(lab, closure_labels(n, adj)), mask
    for g in (graphgen.rmat(13, 8, seed=6, symmetrize=True),
              graphgen.uniform(12, 3000, seed=9, symmetrize=True)):
        ref = oracle.cc(g)
        runs = [oracle.cc_labelprop_parallel(g, threads=t) for t in (1, 3, 0)]
        for lab, it, used in runs:
            assert np.array_equal(lab, ref)
            assert it == runs[0][1]
        assert runs[0][2] == 1 and runs[1][2] == 3
    k = 9
    path = graphgen.from_edges(k + 1, list(range(k)), list(range(1, k + 1)), symmetrize=True)
    lab, it, _ = oracle.cc_labelprop_parallel(path, threads=2)
    assert lab.tolist() == [0] * (k + 1)
    assert it == k + 1
