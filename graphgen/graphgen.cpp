// graphgen.cpp -- seeded synthetic graph inputs (R-MAT and uniform edge lists,
// uint32 weights), cleaned into a sorted out-edge CSR.
//
// This module is input generation only. It holds none of the graph
// algorithms: both the CPU oracle and the GPU library consume the CSR it
// produces, so it is the one piece of code the two sides share.
//
// Random numbers: SplitMix64 (Steele, Lea and Flood, "Fast splittable
// pseudorandom number generators", OOPSLA 2014) used as a counter-based
// generator: draw k of a stream keyed by `key` is mix64(key + (k+1)*GAMMA),
// which is exactly the k-th output of a SplitMix64 sequence seeded with `key`.
// Each (edge, level) pair owns its own counter, so generation is parallel and
// the output does not depend on the thread count.
//
// R-MAT (Chakrabarti, Zhan and Faloutsos, SDM 2004): every edge picks one of
// four quadrants per level, most significant bit first, with probabilities
// a, b, c, d = 1-a-b-c; quadrant a = (src bit 0, dst bit 0), b = (0, 1),
// c = (1, 0), d = (1, 1). No noise and no vertex permutation.
//
// Bounded integer draws (weights) use Lemire's multiply-shift with rejection
// ("Fast random integer generation in an interval", ACM TOMACS 2019).
//
// Cleaning: drop self-loops; optionally symmetrize (add the reverse of every
// edge with the same weight); remove duplicate (src, dst) pairs keeping the
// smallest weight; rows sorted by destination.

#include <algorithm>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <vector>
#include <omp.h>

namespace {

constexpr uint64_t GAMMA = 0x9E3779B97F4A7C15ull;

inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// k-th draw (k >= 0) of the SplitMix64 stream seeded with `key`.
inline uint64_t draw(uint64_t key, uint64_t k) { return mix64(key + (k + 1) * GAMMA); }

// Stream keys: distinct seeds for the edge and weight streams of one graph.
inline uint64_t stream_key(uint64_t seed, uint64_t stream) {
  return mix64(seed ^ mix64(stream + 0x632BE59BD9B4E019ull));
}

// uniform double in [0, 1) with 53 random bits
inline double unit(uint64_t r) { return (double)(r >> 11) * 0x1.0p-53; }

// Lemire bounded draw in [0, range), range >= 1; redraws use sub-counters
// k*16 + j of the same stream.
inline uint32_t bounded(uint64_t key, uint64_t k, uint32_t range) {
  for (uint32_t j = 0; j < 16; ++j) {
    uint32_t x = (uint32_t)(draw(key, k * 16 + j) >> 32);
    uint64_t m = (uint64_t)x * (uint64_t)range;
    uint32_t l = (uint32_t)m;
    if (l >= range) return (uint32_t)(m >> 32);
    uint32_t t = (uint32_t)(-range) % range;
    if (l >= t) return (uint32_t)(m >> 32);
  }
  // 16 consecutive rejections have probability below 2^-400 for any range.
  return (uint32_t)(((uint64_t)(uint32_t)(draw(key, k * 16) >> 32) * range) >> 32);
}

enum Kind { RMAT = 0, UNIFORM = 1 };

struct Spec {
  int kind;
  int scale;          // n = 2^scale
  int64_t nedges;     // generated edges before cleaning
  double a, b, c;     // R-MAT quadrant probabilities
  uint64_t seed;      // edge stream seed
  int weighted;
  uint64_t wseed;     // weight stream seed
  uint32_t wmin, wmax;
  int symmetrize;
};

inline void edge_at(const Spec &s, uint64_t ekey, int64_t e, uint32_t &src, uint32_t &dst) {
  if (s.kind == RMAT) {
    const double ab = s.a + s.b, abc = s.a + s.b + s.c;
    uint32_t u = 0, v = 0;
    for (int lvl = 0; lvl < s.scale; ++lvl) {
      double r = unit(draw(ekey, (uint64_t)e * 64 + lvl));
      uint32_t sb, db;
      if (r < s.a) { sb = 0; db = 0; }
      else if (r < ab) { sb = 0; db = 1; }
      else if (r < abc) { sb = 1; db = 0; }
      else { sb = 1; db = 1; }
      u = (u << 1) | sb;
      v = (v << 1) | db;
    }
    src = u; dst = v;
  } else {
    src = (uint32_t)(draw(ekey, (uint64_t)e * 2) >> (64 - s.scale));
    dst = (uint32_t)(draw(ekey, (uint64_t)e * 2 + 1) >> (64 - s.scale));
  }
}

inline uint32_t weight_at(const Spec &s, uint64_t wkey, int64_t e) {
  return s.wmin + bounded(wkey, (uint64_t)e, s.wmax - s.wmin + 1);
}

}  // namespace

struct gg_graph {
  int32_t n;
  int64_t m;
  int64_t *offsets;   // n+1
  int32_t *col;       // m
  uint32_t *w;        // m or null
};

extern "C" {

// Generate and clean a graph. Returns 0 on success, negative on bad arguments
// or allocation failure. The result is owned by the handle; copy it out with
// gg_copy and release it with gg_free.
int gg_generate(int kind, int scale, int64_t nedges, double a, double b, double c,
                uint64_t seed, int weighted, uint64_t wseed, uint32_t wmin, uint32_t wmax,
                int symmetrize, int nthreads, gg_graph **out) {
  if (!out || scale < 1 || scale > 30 || nedges < 0) return -1;
  if (kind != RMAT && kind != UNIFORM) return -1;
  if (kind == RMAT && (a < 0 || b < 0 || c < 0 || a + b + c > 1.0)) return -1;
  if (weighted && (wmin > wmax)) return -1;
  Spec s{kind, scale, nedges, a, b, c, seed, weighted, wseed, wmin, wmax, symmetrize};
  const int32_t n = (int32_t)(1u << scale);
  const uint64_t ekey = stream_key(seed, 1), wkey = stream_key(wseed, 2);
  int T = nthreads > 0 ? nthreads : omp_get_max_threads();
  if (T > 64) T = 64;

  // Phase A: per-thread out-degree histograms (arcs after self-loop removal
  // and optional symmetrization, before dedup).
  std::vector<int32_t *> hist(T, nullptr);
  for (int t = 0; t < T; ++t) {
    hist[t] = (int32_t *)calloc((size_t)n, sizeof(int32_t));
    if (!hist[t]) { for (auto p : hist) free(p); return -2; }
  }
  auto erange = [&](int t, int64_t &lo, int64_t &hi) {
    lo = nedges * t / T; hi = nedges * (t + 1) / T;
  };
#pragma omp parallel num_threads(T)
  {
    int t = omp_get_thread_num();
    int64_t lo, hi; erange(t, lo, hi);
    int32_t *h = hist[t];
    for (int64_t e = lo; e < hi; ++e) {
      uint32_t u, v; edge_at(s, ekey, e, u, v);
      if (u == v) continue;
      h[u]++;
      if (symmetrize) h[v]++;
    }
  }
  // Row starts and per-thread write cursors (hist[t][v] becomes the cursor).
  int64_t *rowstart = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
  if (!rowstart) { for (auto p : hist) free(p); return -2; }
  {
    // per-vertex totals, then a sequential prefix over vertices
    std::vector<int64_t> tot((size_t)n);
#pragma omp parallel for num_threads(T) schedule(static)
    for (int64_t v = 0; v < n; ++v) {
      int64_t sum = 0;
      for (int t = 0; t < T; ++t) sum += hist[t][v];
      tot[v] = sum;
    }
    int64_t acc = 0;
    for (int64_t v = 0; v < n; ++v) { rowstart[v] = acc; acc += tot[v]; }
    rowstart[n] = acc;
#pragma omp parallel for num_threads(T) schedule(static)
    for (int64_t v = 0; v < n; ++v) {
      int64_t cur = rowstart[v];
      for (int t = 0; t < T; ++t) { int64_t c0 = hist[t][v]; hist[t][v] = (int32_t)(cur - rowstart[v]); cur += c0; }
    }
  }
  const int64_t arcs = rowstart[n];
  // packed (dst << 32 | weight): sorting a row sorts by (dst, weight)
  uint64_t *keys = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(arcs > 0 ? arcs : 1));
  if (!keys) { free(rowstart); for (auto p : hist) free(p); return -2; }
#pragma omp parallel num_threads(T)
  {
    int t = omp_get_thread_num();
    int64_t lo, hi; erange(t, lo, hi);
    int32_t *cur = hist[t];
    for (int64_t e = lo; e < hi; ++e) {
      uint32_t u, v; edge_at(s, ekey, e, u, v);
      if (u == v) continue;
      uint32_t w = weighted ? weight_at(s, wkey, e) : 0u;
      keys[rowstart[u] + cur[u]++] = ((uint64_t)v << 32) | w;
      if (symmetrize) keys[rowstart[v] + cur[v]++] = ((uint64_t)u << 32) | w;
    }
  }
  for (auto p : hist) free(p);
  // Sort each row and drop repeated destinations (the first, smallest weight, stays).
  std::vector<int64_t> uniq((size_t)n + 1, 0);
#pragma omp parallel for num_threads(T) schedule(dynamic, 1024)
  for (int64_t v = 0; v < n; ++v) {
    uint64_t *r = keys + rowstart[v];
    int64_t len = rowstart[v + 1] - rowstart[v];
    std::sort(r, r + len);
    int64_t k = 0;
    for (int64_t i = 0; i < len; ++i)
      if (k == 0 || (r[i] >> 32) != (r[k - 1] >> 32)) r[k++] = r[i];
    uniq[v] = k;
  }
  gg_graph *g = (gg_graph *)calloc(1, sizeof(gg_graph));
  if (!g) { free(keys); free(rowstart); return -2; }
  g->n = n;
  g->offsets = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
  int64_t acc = 0;
  for (int64_t v = 0; v < n; ++v) { g->offsets[v] = acc; acc += uniq[v]; }
  g->offsets[n] = acc;
  g->m = acc;
  g->col = (int32_t *)malloc(sizeof(int32_t) * (size_t)(acc > 0 ? acc : 1));
  g->w = weighted ? (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(acc > 0 ? acc : 1)) : nullptr;
  if (!g->offsets || !g->col || (weighted && !g->w)) {
    free(g->offsets); free(g->col); free(g->w); free(g); free(keys); free(rowstart); return -2;
  }
#pragma omp parallel for num_threads(T) schedule(dynamic, 1024)
  for (int64_t v = 0; v < n; ++v) {
    const uint64_t *r = keys + rowstart[v];
    int64_t o = g->offsets[v];
    for (int64_t i = 0; i < uniq[v]; ++i) {
      g->col[o + i] = (int32_t)(r[i] >> 32);
      if (weighted) g->w[o + i] = (uint32_t)(r[i] & 0xFFFFFFFFu);
    }
  }
  free(keys); free(rowstart);
  *out = g;
  return 0;
}

void gg_info(const gg_graph *g, int32_t *n, int64_t *m, int32_t *weighted) {
  *n = g->n; *m = g->m; *weighted = g->w != nullptr;
}

void gg_copy(const gg_graph *g, int64_t *offsets, int32_t *col, uint32_t *w) {
  memcpy(offsets, g->offsets, sizeof(int64_t) * ((size_t)g->n + 1));
  memcpy(col, g->col, sizeof(int32_t) * (size_t)g->m);
  if (w && g->w) memcpy(w, g->w, sizeof(uint32_t) * (size_t)g->m);
}

void gg_free(gg_graph *g) {
  if (!g) return;
  free(g->offsets); free(g->col); free(g->w); free(g);
}

// Raw SplitMix64 draw, exported so tests can check the generator against
// the published reference sequence.
uint64_t gg_splitmix64_draw(uint64_t key, uint64_t k) { return draw(key, k); }

// Bounded draws for callers that need seeded integers in [lo, hi] from the
// same generator (e.g. query sources, personalized-PageRank seeds).
void gg_bounded_draws(uint64_t seed, uint64_t stream, int64_t count, uint32_t lo, uint32_t hi,
                      uint32_t *out) {
  const uint64_t key = stream_key(seed, stream);
  const uint32_t range = hi - lo + 1;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < count; ++i) out[i] = lo + bounded(key, (uint64_t)i, range);
}

}  // extern "C"
