// sparse.cpp -- the sparse stage of the heterogeneous execution model
// (Section 3.1): once few vertices change per pass, the host finishes the
// run by pushing relaxations along out-edges from the compressed frontier
// (the vertices the last device pass changed), instead of streaming every
// page through the GPU again.
#include <algorithm>
#include <cstring>
#include <thread>
#include <unordered_map>

#include "engine.hpp"

namespace sr {

// Out-edge CSR of the graph, rebuilt once from the in-edge CSR by a
// counting sort on the source and kept with the graph.
void build_out_csr(sr_graph *g) {
  if (g->out_built) return;
  const int32_t n = g->n;
  const int64_t m = g->m;
  std::vector<int64_t> off((size_t)n + 1, 0);
  for (int64_t e = 0; e < m; ++e) off[(size_t)g->in_src[e] + 1]++;
  for (int32_t v = 0; v < n; ++v) off[v + 1] += off[v];
  g->out_dst.assign((size_t)m, 0);
  if (g->weighted) g->out_w.assign((size_t)m, 0);
  std::vector<int64_t> cur(off.begin(), off.end() - 1);
  for (int32_t v = 0; v < n; ++v)
    for (int64_t e = g->in_off[v]; e < g->in_off[v + 1]; ++e) {
      const int64_t k = cur[g->in_src[e]]++;
      g->out_dst[k] = v;
      if (g->weighted) g->out_w[k] = g->in_w[e];
    }
  g->out_off = std::move(off);
  g->out_built = true;
}

// Candidate value of v through the edge u -> v (weight w), with the device
// sweep's arithmetic: CC passes the label, BFS adds one level, SSSP adds the
// weight; INF stays INF and sums saturate at INF.
static inline uint32_t relax_value(int algo, uint32_t xu, uint32_t w) {
  if (algo == A_CC) return xu;
  if (xu == INF) return INF;
  const uint64_t c = (uint64_t)xu + (algo == A_SSSP ? (uint64_t)w : 1ull);
  return c >= (uint64_t)INF ? INF : (uint32_t)c;
}

// Push from the frontier until no value decreases: rounds of label
// correction, each round's list split over host threads, atomic minimum on
// the values and an in-list flag per vertex. Monotone min relaxations reach
// the same least fixed point in any order, so the result is exact.
// When a round's list grows beyond `limit` entries (limit > 0) the stage
// stops before that round: the list goes to `rest` (every vertex whose
// out-edges are not yet relaxed since its last decrease) and the run goes
// back to the device (the density switch taken the other way, Section 3.1).
int64_t sparse_push(sr_graph *g, int algo, uint32_t *val, const uint32_t *front, int64_t nf,
                    int32_t *rounds_out, int64_t limit, std::vector<uint32_t> *rest) {
  const int32_t n = g->n;
  // flags are set when a vertex enters the next round and cleared when that
  // round starts, so the array is all zero again on return
  std::vector<uint8_t> &inq = g->push_inq;
  if ((int64_t)inq.size() != (int64_t)n) inq.assign((size_t)n, 0);
  std::vector<int32_t> cur;
  cur.reserve((size_t)nf);
  for (int64_t i = 0; i < nf; ++i) {
    const uint32_t v = front[i];
    if (v < (uint32_t)n && !inq[v]) { inq[v] = 1; cur.push_back((int32_t)v); }
  }
  const int T = host_threads();
  int64_t relaxed = 0;
  int32_t rounds = 0;
  std::vector<std::vector<int32_t>> next(T);
  std::vector<int64_t> cnt(T);
  if (rest) rest->clear();
  while (!cur.empty()) {
    if (limit > 0 && (int64_t)cur.size() > limit && rest) {
      // dense again: hand the unrelaxed list back and clear its flags
      rest->reserve(cur.size());
      for (int32_t u : cur) { inq[u] = 0; rest->push_back((uint32_t)u); }
      break;
    }
    ++rounds;
    for (int32_t u : cur) inq[u] = 0;  // a later decrease puts u back
    auto work = [&](int t, size_t lo, size_t hi) {
      auto &nx = next[t];
      int64_t c = 0;
      for (size_t i = lo; i < hi; ++i) {
        const int32_t u = cur[i];
        const uint32_t xu = __atomic_load_n(&val[u], __ATOMIC_RELAXED);
        if (xu == INF && algo != A_CC) continue;
        for (int64_t e = g->out_off[u]; e < g->out_off[u + 1]; ++e) {
          const int32_t v = g->out_dst[e];
          const uint32_t nd = relax_value(algo, xu, g->weighted ? g->out_w[e] : 1u);
          ++c;
          uint32_t old = __atomic_load_n(&val[v], __ATOMIC_RELAXED);
          bool lowered = false;
          while (nd < old) {
            if (__atomic_compare_exchange_n(&val[v], &old, nd, true, __ATOMIC_RELAXED, __ATOMIC_RELAXED)) {
              lowered = true;
              break;
            }
          }
          if (lowered && __atomic_exchange_n(&inq[v], (uint8_t)1, __ATOMIC_RELAXED) == 0) nx.push_back(v);
        }
      }
      cnt[t] = c;
    };
    const int use = (int)std::min<size_t>((size_t)T, std::max<size_t>(1, cur.size() / 256));
    for (int t = 0; t < T; ++t) { next[t].clear(); cnt[t] = 0; }
    if (use <= 1) {
      work(0, 0, cur.size());
    } else {
      std::vector<std::thread> th;
      for (int t = 0; t < use; ++t)
        th.emplace_back(work, t, cur.size() * t / use, cur.size() * (t + 1) / use);
      for (auto &x : th) x.join();
    }
    cur.clear();
    for (int t = 0; t < T; ++t) {
      relaxed += cnt[t];
      cur.insert(cur.end(), next[t].begin(), next[t].end());
    }
  }
  if (rounds_out) *rounds_out = rounds;
  return relaxed;
}

// The same push over a partial copy of the values: rounds relax in list
// order with immediate updates (monotone min relaxations reach the same
// least fixed point in any order), each preceded by one fetch of the values
// the round will read (its list's and their out-neighbours') that the host
// does not hold yet.
bool sparse_push_partial(sr_graph *g, int algo, std::unordered_map<uint32_t, uint32_t> &known,
                         const std::vector<uint32_t> &front, int64_t limit, size_t cap,
                         const std::function<bool(const std::vector<uint32_t> &, std::vector<uint32_t> &)> &fetch,
                         std::vector<uint32_t> *lowered, int32_t *rounds_out, int64_t *relaxed_out) {
  const uint32_t n = (uint32_t)g->n;
  std::vector<uint32_t> cur, next, need, got;
  std::unordered_map<uint32_t, uint8_t> inq;  // 1: in the next round's list
  std::unordered_map<uint32_t, uint8_t> low;  // vertices lowered so far
  for (uint32_t v : front)
    if (v < n && !inq[v]) { inq[v] = 1; cur.push_back(v); }
  int32_t rounds = 0;
  int64_t relaxed = 0;
  lowered->clear();
  while (!cur.empty()) {
    if (limit > 0 && (int64_t)cur.size() > limit) return false;
    // a round whose values the host cannot hold (more than cap in all)
    // gives up as soon as it has collected cap of them
    need.clear();
    for (uint32_t u : cur)
      if (!known.count(u)) {
        known[u] = INF;
        need.push_back(u);
        if (known.size() > cap) return false;
      }
    for (uint32_t u : cur)
      for (int64_t e = g->out_off[u]; e < g->out_off[u + 1]; ++e) {
        const uint32_t v = (uint32_t)g->out_dst[e];
        if (!known.count(v)) {
          known[v] = INF;  // placeholder until the fetch fills it
          need.push_back(v);
          if (known.size() > cap) return false;
        }
      }
    if (!need.empty()) {
      got.assign(need.size(), INF);
      if (!fetch(need, got)) return false;
      for (size_t i = 0; i < need.size(); ++i) known[need[i]] = got[i];
    }
    ++rounds;
    next.clear();
    for (uint32_t u : cur) inq[u] = 0;
    for (uint32_t u : cur) {
      const uint32_t xu = known[u];
      if (xu == INF && algo != A_CC) continue;
      for (int64_t e = g->out_off[u]; e < g->out_off[u + 1]; ++e) {
        const uint32_t v = (uint32_t)g->out_dst[e];
        const uint32_t nd = relax_value(algo, xu, g->weighted ? g->out_w[e] : 1u);
        ++relaxed;
        uint32_t &xv = known[v];
        if (nd < xv) {
          xv = nd;
          low[v] = 1;
          if (!inq[v]) { inq[v] = 1; next.push_back(v); }
        }
      }
    }
    cur.swap(next);
  }
  lowered->reserve(low.size());
  for (auto &kv : low) lowered->push_back(kv.first);
  *rounds_out = rounds;
  *relaxed_out = relaxed;
  return true;
}

// One pull on the host over the listed vertices, with the device sweep's
// arithmetic over their in-edges. Every new value is computed from the
// values as they were (a Jacobi step) and written afterwards; the vertices
// whose value decreased go to *changed. Returns the edges read.
int64_t sparse_pull(sr_graph *g, int algo, uint32_t *val, const uint32_t *list, int64_t nl,
                    std::vector<uint32_t> *changed) {
  const int T = host_threads();
  const int use = (int)std::min<int64_t>((int64_t)T, std::max<int64_t>(1, nl / 1024));
  std::vector<std::vector<std::pair<uint32_t, uint32_t>>> upd(use);
  std::vector<int64_t> cnt(use, 0);
  auto work = [&](int t, int64_t lo, int64_t hi) {
    int64_t c = 0;
    for (int64_t i = lo; i < hi; ++i) {
      const uint32_t v = list[i];
      if (v >= (uint32_t)g->n) continue;
      uint32_t best = val[v];
      for (int64_t e = g->in_off[v]; e < g->in_off[v + 1]; ++e) {
        const uint32_t u = (uint32_t)g->in_src[e];
        best = std::min(best, relax_value(algo, val[u], g->weighted ? g->in_w[e] : 1u));
        ++c;
      }
      if (best < val[v]) upd[t].push_back({v, best});
    }
    cnt[t] = c;
  };
  if (use <= 1) {
    work(0, 0, nl);
  } else {
    std::vector<std::thread> th;
    for (int t = 0; t < use; ++t) th.emplace_back(work, t, nl * t / use, nl * (t + 1) / use);
    for (auto &x : th) x.join();
  }
  int64_t edges = 0;
  changed->clear();
  for (int t = 0; t < use; ++t) {
    edges += cnt[t];
    for (auto &kv : upd[t]) {
      val[kv.first] = kv.second;
      changed->push_back(kv.first);
    }
  }
  return edges;
}

}  // namespace sr

namespace sr {

// Bit of page p in a 64-bit page mask (pages share bits when P > 64, which
// only makes the dirty test more conservative).
static inline int page_bit(int32_t p, int32_t P) { return P <= 64 ? p : (int)((int64_t)p * 64 / P); }

void build_out_masks(sr_graph *g) {
  const int32_t P = (int32_t)g->pages.size();
  if (g->out_mask_parts == P && (int64_t)g->out_mask.size() == (int64_t)g->n) return;
  build_out_csr(g);
  std::vector<uint8_t> bit((size_t)g->n);
  for (int32_t p = 0; p < P; ++p) {
    const int b = page_bit(p, P);
    for (int32_t v = g->pages[p].hdr.v_begin; v < g->pages[p].hdr.v_begin + g->pages[p].hdr.n_p; ++v)
      bit[v] = (uint8_t)b;
  }
  g->out_mask.assign((size_t)g->n, 0ull);
  for (int32_t u = 0; u < g->n; ++u) {
    uint64_t m = 0;
    for (int64_t e = g->out_off[u]; e < g->out_off[u + 1]; ++e) m |= 1ull << bit[g->out_dst[e]];
    g->out_mask[u] = m;
  }
  g->out_mask_parts = P;
}

uint64_t frontier_pages(const sr_graph *g, const uint32_t *front, int64_t nf) {
  uint64_t m = 0;
  for (int64_t i = 0; i < nf; ++i)
    if (front[i] < (uint32_t)g->n) m |= g->out_mask[front[i]];
  return m;
}

}  // namespace sr
