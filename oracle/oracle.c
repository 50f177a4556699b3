/*
 * oracle.c -- plain, slow, obviously correct CPU reference for the vertex
 * programs of Seraph ("Scaling Up Large-Scale Graph Processing for
 * GPU-Accelerated Heterogeneous Systems", Li, arXiv 1806.00762).
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may call this code;
 * only the tests, the smoke check and the benchmark's CPU-baseline leg use it.
 * It shares no code with the GPU library (no headers, no helpers).
 *
 * The paper's method (pipelined multi-pass subgraph iteration, Section 3;
 * predictive vertex updating, Section 4) reaches exactly the plain result
 * of each program, so this file computes the plain definitions and never
 * simulates a schedule:
 *   BFS  (Section 5.1): hop distance from a source       -> queue BFS
 *   SSSP (Section 5.1): weighted distance, weights >= 0  -> Dijkstra; Bellman-Ford cross-check
 *   CC   (Sections 4.1 and 5.1): smallest vertex id in each undirected
 *        component, the fixed point of min-label propagation -> union-find
 *   PageRank / personalized PageRank (named in Section 4.3, not defined by
 *        the paper): x = (1-d) t + d (P^T x + D t), D = dangling mass, t the
 *        teleport vector (uniform, or e_s for personalized); FP64 Jacobi
 *        power iteration.
 * Plus the predictive-vertex-updating reference semantics (Table I strong
 * thresholds, Fig. 6 weak state machine) and result certificates.
 *
 * Graphs are out-edge CSR: row u holds the heads col[off[u] .. off[u+1]-1]
 * with optional uint32 weights w[]. Unreached vertices hold UINT32_MAX.
 * Every function returns 0 on success and a negative code on bad input.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_INF 0xFFFFFFFFu

/* ------------------------------------------------------------------------ */
/* SSSP: Dijkstra with an indexed binary min-heap over 64-bit tentative      */
/* distances (no overflow whatever the weights).                             */

typedef struct {
  int32_t *heap;  /* heap of vertex ids */
  int32_t *pos;   /* pos[v] = index in heap, -1 if absent */
  uint64_t *key;  /* tentative distance */
  int32_t size;
} ixheap;

static void hswap(ixheap *h, int32_t i, int32_t j) {
  int32_t a = h->heap[i], b = h->heap[j];
  h->heap[i] = b; h->heap[j] = a;
  h->pos[b] = i; h->pos[a] = j;
}

static void hup(ixheap *h, int32_t i) {
  while (i > 0) {
    int32_t p = (i - 1) / 2;
    if (h->key[h->heap[p]] <= h->key[h->heap[i]]) break;
    hswap(h, i, p);
    i = p;
  }
}

static void hdown(ixheap *h, int32_t i) {
  for (;;) {
    int32_t l = 2 * i + 1, r = l + 1, s = i;
    if (l < h->size && h->key[h->heap[l]] < h->key[h->heap[s]]) s = l;
    if (r < h->size && h->key[h->heap[r]] < h->key[h->heap[s]]) s = r;
    if (s == i) break;
    hswap(h, i, s);
    i = s;
  }
}

int or_sssp_dijkstra(int32_t n, const int64_t *off, const int32_t *col, const uint32_t *w,
                     int32_t src, uint32_t *dist) {
  if (n <= 0 || src < 0 || src >= n) return -1;
  ixheap h;
  h.heap = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  h.pos = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  h.key = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
  char *done = (char *)calloc((size_t)n, 1);
  if (!h.heap || !h.pos || !h.key || !done) {
    free(h.heap); free(h.pos); free(h.key); free(done);
    return -2;
  }
  for (int32_t v = 0; v < n; ++v) { h.pos[v] = -1; h.key[v] = UINT64_MAX; }
  h.size = 0;
  h.key[src] = 0;
  h.heap[0] = src; h.pos[src] = 0; h.size = 1;
  while (h.size > 0) {
    int32_t u = h.heap[0];
    hswap(&h, 0, h.size - 1);
    h.size--;
    h.pos[u] = -1;
    if (h.size > 0) hdown(&h, 0);
    done[u] = 1;
    for (int64_t e = off[u]; e < off[u + 1]; ++e) {
      int32_t v = col[e];
      if (done[v]) continue;
      uint64_t cand = h.key[u] + (uint64_t)(w ? w[e] : 1u);
      if (cand < h.key[v]) {
        h.key[v] = cand;
        if (h.pos[v] < 0) { h.heap[h.size] = v; h.pos[v] = h.size; h.size++; }
        hup(&h, h.pos[v]);
      }
    }
  }
  int rc = 0;
  for (int32_t v = 0; v < n; ++v) {
    if (h.key[v] == UINT64_MAX) dist[v] = OR_INF;
    else if (h.key[v] >= (uint64_t)OR_INF) { dist[v] = OR_INF; rc = -3; } /* not representable */
    else dist[v] = (uint32_t)h.key[v];
  }
  free(h.heap); free(h.pos); free(h.key); free(done);
  return rc;
}

/* Synchronous Bellman-Ford: every round relaxes every edge from the previous
 * round's distances; stops on a round without change. *rounds_out receives the
 * number of rounds that changed something. */
int or_sssp_bellman_ford(int32_t n, const int64_t *off, const int32_t *col, const uint32_t *w,
                         int32_t src, uint32_t *dist, int32_t *rounds_out) {
  if (n <= 0 || src < 0 || src >= n) return -1;
  uint64_t *cur = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
  uint64_t *nxt = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
  if (!cur || !nxt) { free(cur); free(nxt); return -2; }
  for (int32_t v = 0; v < n; ++v) cur[v] = UINT64_MAX;
  cur[src] = 0;
  int32_t rounds = 0;
  for (;;) {
    memcpy(nxt, cur, sizeof(uint64_t) * (size_t)n);
    int changed = 0;
    for (int32_t u = 0; u < n; ++u) {
      if (cur[u] == UINT64_MAX) continue;
      for (int64_t e = off[u]; e < off[u + 1]; ++e) {
        uint64_t cand = cur[u] + (uint64_t)(w ? w[e] : 1u);
        if (cand < nxt[col[e]]) { nxt[col[e]] = cand; changed = 1; }
      }
    }
    uint64_t *t = cur; cur = nxt; nxt = t;
    if (!changed) break;
    rounds++;
    if (rounds > n) break; /* impossible with non-negative weights */
  }
  for (int32_t v = 0; v < n; ++v) dist[v] = cur[v] >= (uint64_t)OR_INF ? OR_INF : (uint32_t)cur[v];
  if (rounds_out) *rounds_out = rounds;
  free(cur); free(nxt);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* BFS: FIFO queue, level = hop count from src.                              */

int or_bfs(int32_t n, const int64_t *off, const int32_t *col, int32_t src, uint32_t *level) {
  if (n <= 0 || src < 0 || src >= n) return -1;
  int32_t *q = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  if (!q) return -2;
  for (int32_t v = 0; v < n; ++v) level[v] = OR_INF;
  int32_t head = 0, tail = 0;
  level[src] = 0;
  q[tail++] = src;
  while (head < tail) {
    int32_t u = q[head++];
    for (int64_t e = off[u]; e < off[u + 1]; ++e) {
      int32_t v = col[e];
      if (level[v] == OR_INF) { level[v] = level[u] + 1; q[tail++] = v; }
    }
  }
  free(q);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* CC: union-find over the arcs taken as undirected edges. The root of every */
/* set is its smallest vertex id (union links the larger root under the      */
/* smaller), so the label of v is find(v).                                   */

static int32_t uf_find(int32_t *parent, int32_t x) {
  while (parent[x] != x) {
    parent[x] = parent[parent[x]]; /* path halving */
    x = parent[x];
  }
  return x;
}

int or_cc_union_find(int32_t n, const int64_t *off, const int32_t *col, uint32_t *label) {
  if (n <= 0) return -1;
  int32_t *parent = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  if (!parent) return -2;
  for (int32_t v = 0; v < n; ++v) parent[v] = v;
  for (int32_t u = 0; u < n; ++u) {
    for (int64_t e = off[u]; e < off[u + 1]; ++e) {
      int32_t a = uf_find(parent, u), b = uf_find(parent, col[e]);
      if (a == b) continue;
      if (a < b) parent[b] = a; else parent[a] = b;
    }
  }
  for (int32_t v = 0; v < n; ++v) label[v] = (uint32_t)uf_find(parent, v);
  free(parent);
  return 0;
}

/* Synchronous min-label propagation (the connected-components example of
 * Section 4.1): label_0 = id; in iteration i every vertex takes the minimum
 * of its own and its neighbours' labels from iteration i-1. Arcs are taken as
 * undirected. Runs `iters` iterations; hist (iters x n, may be NULL) receives
 * the labels after each one. Returns the number of iterations that changed a
 * label through *changed_iters. */
int or_cc_labelprop_sync(int32_t n, const int64_t *off, const int32_t *col, int32_t iters,
                         uint32_t *label, uint32_t *hist, int32_t *changed_iters) {
  if (n <= 0 || iters < 0) return -1;
  uint32_t *old = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n);
  if (!old) return -2;
  for (int32_t v = 0; v < n; ++v) label[v] = (uint32_t)v;
  int32_t nch = 0;
  for (int32_t it = 0; it < iters; ++it) {
    memcpy(old, label, sizeof(uint32_t) * (size_t)n);
    int changed = 0;
    for (int32_t u = 0; u < n; ++u) {
      for (int64_t e = off[u]; e < off[u + 1]; ++e) {
        int32_t v = col[e];
        if (old[u] < label[v]) { label[v] = old[u]; changed = 1; }
        if (old[v] < label[u]) { label[u] = old[v]; changed = 1; }
      }
    }
    if (changed) nch++;
    if (hist) memcpy(hist + (size_t)it * (size_t)n, label, sizeof(uint32_t) * (size_t)n);
  }
  if (changed_iters) *changed_iters = nch;
  free(old);
  return 0;
}

/* Synchronous min-label propagation to the fixed point, every iteration
 * split over `threads` OpenMP threads (0 = all): label_0 = id; in each
 * iteration every vertex takes the minimum of its own label and its
 * neighbours' labels from the previous iteration (two arrays, so the result
 * and the iteration count do not depend on the thread count). The input
 * must be symmetric (row v lists v's neighbours), so each vertex pulls from
 * its own row. The fixed point gives every vertex the smallest id of its
 * component (Section 4.1's example run to the end). Returns the iterations
 * run, the last one changing nothing, in *iters, and the threads used in
 * *threads_used. */
int or_cc_labelprop_parallel(int32_t n, const int64_t *off, const int32_t *col, int32_t threads,
                             uint32_t *label, int32_t *iters, int32_t *threads_used) {
  if (n <= 0 || threads < 0) return -1;
  uint32_t *old = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n);
  if (!old) return -2;
  int T = threads > 0 ? threads : omp_get_max_threads();
  for (int32_t v = 0; v < n; ++v) label[v] = (uint32_t)v;
  int32_t it = 0;
  int changed = 1;
  while (changed) {
    memcpy(old, label, sizeof(uint32_t) * (size_t)n);
    changed = 0;
#pragma omp parallel for num_threads(T) schedule(dynamic, 4096) reduction(| : changed)
    for (int32_t v = 0; v < n; ++v) {
      uint32_t x = old[v];
      for (int64_t e = off[v]; e < off[v + 1]; ++e)
        if (old[col[e]] < x) x = old[col[e]];
      if (x < old[v]) { label[v] = x; changed = 1; }
    }
    it++;
  }
  if (iters) *iters = it;
  if (threads_used) *threads_used = T;
  free(old);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* PageRank. t = uniform 1/n (seed < 0) or e_seed (personalized). One Jacobi  */
/* step: D = sum of x over vertices without out-edges; y[v] = sum over arcs   */
/* u->v of x[u]/outdeg(u); x'[v] = (1-d) t[v] + d (y[v] + D t[v]).            */

static double tele(int32_t n, int32_t seed, int32_t v) {
  if (seed < 0) return 1.0 / (double)n;
  return v == seed ? 1.0 : 0.0;
}

static void pr_step(int32_t n, const int64_t *off, const int32_t *col, double d, int32_t seed,
                    const double *x, double *y) {
  double dangling = 0.0;
  for (int32_t u = 0; u < n; ++u)
    if (off[u + 1] == off[u]) dangling += x[u];
  for (int32_t v = 0; v < n; ++v) y[v] = 0.0;
  for (int32_t u = 0; u < n; ++u) {
    int64_t deg = off[u + 1] - off[u];
    if (deg == 0) continue;
    double share = x[u] / (double)deg;
    for (int64_t e = off[u]; e < off[u + 1]; ++e) y[col[e]] += share;
  }
  for (int32_t v = 0; v < n; ++v) {
    double t = tele(n, seed, v);
    y[v] = (1.0 - d) * t + d * (y[v] + dangling * t);
  }
}

/* Power iteration from x0 = t until the L1 change of one step is below tol or
 * max_iter steps ran. Returns the step count in *iters and the last L1 change
 * in *l1_last. */
int or_pagerank(int32_t n, const int64_t *off, const int32_t *col, double d, int32_t seed,
                double tol, int32_t max_iter, double *x, int32_t *iters, double *l1_last) {
  if (n <= 0 || !(d >= 0.0 && d < 1.0) || seed >= n) return -1;
  double *y = (double *)malloc(sizeof(double) * (size_t)n);
  if (!y) return -2;
  for (int32_t v = 0; v < n; ++v) x[v] = tele(n, seed, v);
  int32_t it = 0;
  double l1 = INFINITY;
  while (it < max_iter) {
    pr_step(n, off, col, d, seed, x, y);
    l1 = 0.0;
    for (int32_t v = 0; v < n; ++v) l1 += fabs(y[v] - x[v]);
    memcpy(x, y, sizeof(double) * (size_t)n);
    it++;
    if (l1 < tol) break;
  }
  if (iters) *iters = it;
  if (l1_last) *l1_last = l1;
  free(y);
  return 0;
}

/* The first k terms of PageRank's Neumann series: k steps of the same map
 * from x0 = 0, so x_k = sum_{j<k} A^j (1 - d) t with A y = d (P^T y + D(y) t).
 * This is the state that propagating rank mass as residuals (the data-driven
 * PageRank-delta of Section 4.3, no vertex held back) reaches after k
 * synchronous passes; the sum of x_k is 1 - d^k. */
int or_pagerank_partial(int32_t n, const int64_t *off, const int32_t *col, double d, int32_t seed,
                        int32_t k, double *x) {
  if (n <= 0 || !(d >= 0.0 && d < 1.0) || seed >= n || k < 0) return -1;
  double *y = (double *)malloc(sizeof(double) * (size_t)n);
  if (!y) return -2;
  for (int32_t v = 0; v < n; ++v) x[v] = 0.0;
  for (int32_t it = 0; it < k; ++it) {
    pr_step(n, off, col, d, seed, x, y);
    memcpy(x, y, sizeof(double) * (size_t)n);
  }
  free(y);
  return 0;
}

/* ||T(x) - x||_1 for a given x (FP64). For the d-contraction T this bounds
 * the distance to the fixed point: ||x - x*||_1 <= ||T(x) - x||_1 / (1 - d). */
int or_pagerank_residual(int32_t n, const int64_t *off, const int32_t *col, double d,
                         int32_t seed, const double *x, double *residual) {
  if (n <= 0 || seed >= n) return -1;
  double *y = (double *)malloc(sizeof(double) * (size_t)n);
  if (!y) return -2;
  pr_step(n, off, col, d, seed, x, y);
  double r = 0.0;
  for (int32_t v = 0; v < n; ++v) r += fabs(y[v] - x[v]);
  *residual = r;
  free(y);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Certificates.                                                             */

/* SSSP/BFS distances (w == NULL means unit weights). With weights >= 1 the
 * checks below hold iff dist is exact:
 *   dist[src] == 0;
 *   every arc u->v with finite dist[u] has dist[v] <= dist[u] + w;
 *   every finite dist[v], v != src, has a tight in-arc: dist[u] + w == dist[v].
 * Returns 0 if all hold, otherwise a negative code; *bad receives a witness. */
int or_sssp_certificate(int32_t n, const int64_t *off, const int32_t *col, const uint32_t *w,
                        int32_t src, const uint32_t *dist, int64_t *bad) {
  if (n <= 0 || src < 0 || src >= n) return -1;
  if (dist[src] != 0) { if (bad) *bad = src; return -10; }
  char *tight = (char *)calloc((size_t)n, 1);
  if (!tight) return -2;
  for (int32_t u = 0; u < n; ++u) {
    if (dist[u] == OR_INF) continue;
    for (int64_t e = off[u]; e < off[u + 1]; ++e) {
      if (w && w[e] == 0) { free(tight); if (bad) *bad = e; return -13; }
      uint64_t cand = (uint64_t)dist[u] + (uint64_t)(w ? w[e] : 1u);
      uint32_t dv = dist[col[e]];
      if ((uint64_t)dv > cand) { free(tight); if (bad) *bad = e; return -11; }
      if ((uint64_t)dv == cand) tight[col[e]] = 1;
    }
  }
  for (int32_t v = 0; v < n; ++v) {
    if (v == src || dist[v] == OR_INF) continue;
    if (!tight[v]) { free(tight); if (bad) *bad = v; return -12; }
  }
  free(tight);
  return 0;
}

/* CC labels on a graph taken as undirected: label[u] == label[v] on every
 * arc; label[v] <= v; label[label[v]] == label[v]. */
int or_cc_check(int32_t n, const int64_t *off, const int32_t *col, const uint32_t *label,
                int64_t *bad) {
  if (n <= 0) return -1;
  for (int32_t v = 0; v < n; ++v) {
    if (label[v] > (uint32_t)v) { if (bad) *bad = v; return -20; }
    if (label[label[v]] != label[v]) { if (bad) *bad = v; return -21; }
  }
  for (int32_t u = 0; u < n; ++u)
    for (int64_t e = off[u]; e < off[u + 1]; ++e)
      if (label[u] != label[col[e]]) { if (bad) *bad = e; return -22; }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Predictive vertex updating: reference semantics (Section 4).              */

/* Strong threshold for BFS (Table I): after k completed iterations, a vertex
 * whose level is <= k is converged. */
uint32_t or_strong_threshold_bfs(int32_t k) { return k < 0 ? 0u : (uint32_t)k; }

/* Strong threshold for SSSP (Table I): l = min{ value^(k-1)[v] :
 * value^(k-1)[v] != value^(k-2)[v] }; UINT32_MAX if nothing changed. */
uint32_t or_strong_threshold_sssp(int32_t n, const uint32_t *prev, const uint32_t *cur) {
  uint32_t l = OR_INF;
  for (int32_t v = 0; v < n; ++v)
    if (cur[v] != prev[v] && cur[v] < l) l = cur[v];
  return l;
}

/* Strong threshold for CC as Table I states it: with ccsize[v] = number of
 * vertices labelled v, s = min{ v : ccsize^(k-1)[v] != ccsize^(k-2)[v] };
 * UINT32_MAX if no component size changed. */
uint32_t or_strong_threshold_cc(int32_t n, const uint32_t *prev, const uint32_t *cur) {
  int64_t *a = (int64_t *)calloc((size_t)n, sizeof(int64_t));
  int64_t *b = (int64_t *)calloc((size_t)n, sizeof(int64_t));
  uint32_t s = OR_INF;
  if (a && b) {
    for (int32_t v = 0; v < n; ++v) { a[prev[v]]++; b[cur[v]]++; }
    for (int32_t v = 0; v < n; ++v)
      if (a[v] != b[v]) { s = (uint32_t)v; break; }
  }
  free(a); free(b);
  return s;
}

/* Weak predictor (Fig. 6 and the text around it). A diagram has num_states
 * states; bit i of attempt_mask marks state i as one that attempts an update.
 * An attempting state moves to on_success[i] when the attempt changed the
 * value and to on_fail[i] otherwise; a dormant state always moves to
 * on_fail[i]. Returns the next state, or -1 for an invalid state. */
int32_t or_weak_next(int32_t state, int32_t changed, int32_t num_states, uint32_t attempt_mask,
                     const uint8_t *on_success, const uint8_t *on_fail) {
  if (state < 0 || state >= num_states) return -1;
  int attempts = (attempt_mask >> state) & 1u;
  if (attempts && changed) return on_success[state];
  return on_fail[state];
}

/* The default six-state diagram as the text describes it: states 0, 1, 5
 * attempt, 2, 3, 4 are dormant; start in 0; a success returns to 0; 0 fails
 * to 5 (dormancy candidate); 5 fails to 3 (dormant); 3 sleeps to 2, 2 to 1;
 * 1 attempts again and fails to 4 (punishment), which sleeps to 3. */
void or_weak_default_diagram(int32_t *num_states, int32_t *initial, uint32_t *attempt_mask,
                             uint8_t *on_success, uint8_t *on_fail) {
  *num_states = 6;
  *initial = 0;
  *attempt_mask = (1u << 0) | (1u << 1) | (1u << 5);
  static const uint8_t succ[8] = {0, 0, 1, 2, 3, 0, 0, 0};
  static const uint8_t fail[8] = {5, 4, 1, 2, 3, 3, 0, 0};
  memcpy(on_success, succ, 8);
  memcpy(on_fail, fail, 8);
}
