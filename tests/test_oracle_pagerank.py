"""Pins for the PageRank / personalized PageRank oracle: closed forms, the
dense linear solve, invariants and the residual error bound."""
import numpy as np
import pytest

import graphgen
import oracle

D = 0.85


def dense_solve(g, d=D, seed=-1):
    """x = (1-d) t + d (P^T x + (sum of dangling x) t) as one linear system."""
    n = g.n
    t = np.full(n, 1.0 / n) if seed < 0 else np.eye(n)[seed]
    M = np.zeros((n, n))
    deg = np.diff(g.offsets)
    for u in range(n):
        if deg[u] == 0:
            M[:, u] += t            # dangling column follows the teleport vector
        else:
            for v in g.col[g.offsets[u]:g.offsets[u + 1]]:
                M[v, u] += 1.0 / deg[u]
    return np.linalg.solve(np.eye(n) - d * M, (1 - d) * t)


def test_directed_cycle_uniform():
    n = 37
    g = graphgen.from_edges(n, np.arange(n), (np.arange(n) + 1) % n)
    x, _, _ = oracle.pagerank(g)
    assert np.max(np.abs(x - 1.0 / n)) < 1e-14


def test_undirected_star_closed_form():
    n = 20                                    # leaves; centre 0; N = n+1
    g = graphgen.from_edges(n + 1, np.zeros(n, int), np.arange(1, n + 1), symmetrize=True)
    x, _, _ = oracle.pagerank(g)
    N = n + 1
    xc = (1 + D * n) / (N * (1 + D))
    xl = (n + D) / (n * N * (1 + D))
    assert abs(x[0] - xc) < 1e-13
    assert np.max(np.abs(x[1:] - xl)) < 1e-13


def test_complete_graph_uniform():
    n = 9
    u, v = np.meshgrid(np.arange(n), np.arange(n))
    g = graphgen.from_edges(n, u.ravel(), v.ravel())
    x, _, _ = oracle.pagerank(g)
    assert np.max(np.abs(x - 1.0 / n)) < 1e-14


@pytest.mark.parametrize("trial", range(12))
def test_dense_solve_random_with_dangling(trial):
    r = np.random.default_rng(trial)
    n = int(r.integers(2, 200)); m = int(r.integers(1, 5 * n))
    g = graphgen.from_edges(n, r.integers(0, n, m), r.integers(0, n, m))
    assert np.any(np.diff(g.offsets) == 0) or trial > 6
    x, _, _ = oracle.pagerank(g)
    assert np.max(np.abs(x - dense_solve(g))) < 1e-11
    s = int(r.integers(0, n))
    xp, _, _ = oracle.pagerank(g, seed=s)
    assert np.max(np.abs(xp - dense_solve(g, seed=s))) < 1e-11


def test_ppr_cycle_closed_form():
    n, s = 23, 5
    g = graphgen.from_edges(n, np.arange(n), (np.arange(n) + 1) % n)
    x, _, _ = oracle.pagerank(g, seed=s)
    j = (np.arange(n) - s) % n
    exp = (1 - D) * D ** j / (1 - D ** n)
    assert np.max(np.abs(x - exp)) < 1e-13


def test_invariants_rmat16():
    g = graphgen.recipes.pagerank_s16()
    x, it, l1 = oracle.pagerank(g, tol=1e-9)
    assert l1 < 1e-9 and it < 100
    assert abs(x.sum() - 1.0) < 1e-12
    assert x.min() >= (1 - D) / g.n - 1e-18
    xt, _, _ = oracle.pagerank(g, tol=1e-13)
    # geometric convergence: the 1e-9 stop is within l1*d/(1-d) of the tight run
    assert np.abs(x - xt).sum() <= l1 * D / (1 - D) + 1e-12


def test_residual_bound_certifies_error():
    g = graphgen.rmat(12, 16, seed=3)
    xs, _, _ = oracle.pagerank(g, tol=1e-15)
    r = np.random.default_rng(1)
    for scale in (1e-3, 1e-6, 1e-9):
        x = xs * (1 + scale * r.standard_normal(g.n))
        res = oracle.pagerank_residual(g, x)
        assert np.abs(x - xs).sum() <= res / (1 - D) * (1 + 1e-9) + 1e-15
    assert oracle.pagerank_residual(g, xs) < 1e-13


def test_damping_and_orientation_matter():
    """A dropped damping factor or transposed operand would fail the star form;
    check the directed star too (leaves -> centre only: leaves dangle? no, centre dangles)."""
    n = 6
    g = graphgen.from_edges(n + 1, np.arange(1, n + 1), np.zeros(n, int))  # leaves -> centre
    x, _, _ = oracle.pagerank(g)
    assert np.max(np.abs(x - dense_solve(g))) < 1e-12
    assert x[0] > x[1]


def test_partial_sums_first_terms():
    """k = 0 gives zero and k = 1 the teleport term (1 - d) t."""
    g = graphgen.rmat(9, 8, seed=4)
    assert np.all(oracle.pagerank_partial(g, 0) == 0.0)
    assert np.max(np.abs(oracle.pagerank_partial(g, 1) - (1 - D) / g.n)) < 1e-18
    x1 = oracle.pagerank_partial(g, 1, seed=7)
    assert x1[7] == pytest.approx(1 - D) and np.count_nonzero(x1) == 1


@pytest.mark.parametrize("trial", range(6))
def test_partial_sums_mass_and_limit(trial):
    """sum x_k = 1 - d^k (each term carries d times the mass of the one before,
    dangling mass included), the sums grow monotonically, and many terms reach
    the dense solve."""
    r = np.random.default_rng(100 + trial)
    n = int(r.integers(3, 150)); m = int(r.integers(1, 4 * n))
    g = graphgen.from_edges(n, r.integers(0, n, m), r.integers(0, n, m))
    s = int(r.integers(0, n)) if trial % 2 else -1
    prev = np.zeros(n)
    for k in (1, 2, 3, 7, 20):
        x = oracle.pagerank_partial(g, k, seed=s)
        assert abs(x.sum() - (1 - D ** k)) < 1e-13
        assert np.all(x >= prev - 1e-18)
        prev = x
    x = oracle.pagerank_partial(g, 400, seed=s)
    assert np.max(np.abs(x - dense_solve(g, seed=s))) < 1e-12


def test_partial_sums_cycle_closed_form():
    """On a directed N-cycle with PPR seed s the mass moves one step per term:
    x_k[s + j] = (1 - d) d^j for j < k <= N, and 0 beyond."""
    n, s, k = 29, 4, 11
    g = graphgen.from_edges(n, np.arange(n), (np.arange(n) + 1) % n)
    x = oracle.pagerank_partial(g, k, seed=s)
    j = (np.arange(n) - s) % n
    exp = np.where(j < k, (1 - D) * D ** j, 0.0)
    assert np.max(np.abs(x - exp)) < 1e-15
