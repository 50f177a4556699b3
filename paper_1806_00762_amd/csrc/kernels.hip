// kernels.hip -- gfx950 kernels of the subgraph sweep (Sections 3-4 of
// Li, arXiv 1806.00762): one launch pulls every vertex of the resident
// pages of a window ("super subgraph", Section 3.2), gated by predictive
// vertex updating (Section 4), and folds its counters into the device
// control block; the last block to finish closes the sweep (and the pass).
//
// Mapping: every block owns one (page, degree bin, item). Bins group
// vertices of similar in-degree so a fixed number of lanes serves each
// vertex: lane groups of 1..32 lanes for d < 64 (<= 2 edges per lane),
// one wavefront for 64 <= d <= HEAVY, wavefront-sized chunks for larger d.
// Reads of offsets, in-edge sources and weights are contiguous across the
// lanes of a group and across consecutive groups; the gather of neighbour
// values is the only random access. Pull updates write only the owning
// vertex, so no atomics are needed except for split (chunked) vertices and
// for the per-sweep counters (one set per block).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "kernels.hpp"

namespace sr {
namespace {

// ---------------------------------------------------------------- helpers

template <typename T>
__device__ inline T shfl_xor(T v, int m) { return __shfl_xor(v, m, 64); }

__device__ inline uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += shfl_xor(v, m);
  return v;
}
__device__ inline uint32_t wave_min_u32(uint32_t v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v = min(v, shfl_xor(v, m));
  return v;
}
__device__ inline double wave_sum_f64(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += shfl_xor(v, m);
  return v;
}

template <typename T>
__device__ inline T ld_agent(const T *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ inline void st_agent(T *p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

struct PageCtx {
  int32_t v_begin;
  const int32_t *off;
  const int32_t *bins;
  const Chunk *chunks;
  const int32_t *src;
  const uint32_t *w;
  int32_t bin_count, bin_start;
  uint32_t *partial, *arrive;
};

// Thread-local sweep counters, reduced per block at the end.
struct Acc {
  uint32_t changed = 0, attempted = 0, skipped = 0, mispred = 0, edges = 0;
  uint32_t min_changed = INF;
  double l1 = 0.0, ddelta = 0.0;
};

// Per-block view of the run state.
struct Run {
  int algo, pvu, phase, audit;
  uint32_t threshold;
  uint32_t *value;
  float *contrib;
  const float *inv_outdeg;
  uint8_t *status;
  const Diagram *dia;
  float damping, pr_eps, base_uniform, dangling;
  int32_t pr_seed;
  uint32_t *hist;  // LDS histogram of predictor states
};

// Gate: does vertex v attempt a pull this sweep? (Section 4.) Returns the
// old value and the predictor state.
struct Gate {
  bool attempt;
  uint8_t st;
  uint32_t old;
};

__device__ inline Gate gate_of(const Run &r, int32_t v) {
  Gate g;
  g.old = r.value[v];
  g.st = 0;
  if (r.phase == 1 || r.pvu == P_OFF) {
    g.attempt = true;
  } else if (r.pvu == P_STRONG) {
    // Table I: a vertex whose value is <= the threshold has converged.
    g.attempt = g.old > r.threshold;
  } else {
    g.st = r.status[v];
    g.attempt = (r.dia->attempt_mask >> g.st) & 1u;
  }
  return g;
}

// Contribution of one in-edge (u -> v, weight w) to the reduction.
template <int ALGO>
__device__ inline uint32_t edge_min(const uint32_t *value, int32_t u, uint32_t w) {
  uint32_t x = value[u];
  if (ALGO == A_CC) return x;
  if (x == INF) return INF;
  uint64_t c = (uint64_t)x + (ALGO == A_SSSP ? (uint64_t)w : 1ull);
  return c >= (uint64_t)INF ? INF : (uint32_t)c;
}

template <int ALGO>
constexpr bool is_pr() { return ALGO == A_PR || ALGO == A_PPR; }

// Reduction value: u32 min for BFS/SSSP/CC, f32 sum for PageRank.
template <int ALGO>
struct Red {
  using T = typename std::conditional<is_pr<ALGO>(), float, uint32_t>::type;
  __device__ static inline T identity() {
    if constexpr (is_pr<ALGO>()) return 0.0f; else return INF;
  }
  __device__ static inline T combine(T a, T b) {
    if constexpr (is_pr<ALGO>()) return a + b; else return min(a, b);
  }
  __device__ static inline T edge(const Run &r, int32_t u, uint32_t w) {
    if constexpr (is_pr<ALGO>()) return r.contrib[u];
    else return edge_min<ALGO>(r.value, u, w);
  }
  __device__ static inline uint32_t bits(T v) {
    if constexpr (is_pr<ALGO>()) return __float_as_uint(v); else return v;
  }
  __device__ static inline T from_bits(uint32_t b) {
    if constexpr (is_pr<ALGO>()) return __uint_as_float(b); else return b;
  }
};

// Epilogue of one vertex: compare, write, advance the predictor state,
// count. `computed` says whether red holds the pull result.
template <int ALGO>
__device__ inline void epilogue(const Run &r, int32_t v, const Gate &g, bool computed,
                                typename Red<ALGO>::T red, uint32_t deg, Acc &acc) {
  bool changed = false;
  if (computed) {
    if constexpr (is_pr<ALGO>()) {
      float t = r.pr_seed < 0 ? r.base_uniform : (v == r.pr_seed ? 1.0f : 0.0f);
      float oldf = __uint_as_float(g.old);
      float nv = (1.0f - r.damping) * t + r.damping * (red + r.dangling * t);
      float diff = nv - oldf;
      bool would = fabsf(diff) > r.pr_eps;
      if (g.attempt) {
        changed = would;
        r.value[v] = __float_as_uint(nv);
        float iod = r.inv_outdeg[v];
        r.contrib[v] = nv * iod;
        acc.l1 += fabs((double)nv - (double)oldf);
        if (iod == 0.0f) acc.ddelta += (double)nv - (double)oldf;
      } else if (would) {
        acc.mispred++;
      }
    } else {
      uint32_t nv = min(g.old, red);
      bool would = nv < g.old;
      if (g.attempt) {
        changed = would;
        if (changed) {
          r.value[v] = nv;
          acc.min_changed = min(acc.min_changed, nv);
        }
      } else if (would) {
        acc.mispred++;
      }
    }
  }
  if (g.attempt) {
    acc.attempted++;
    acc.edges += deg;
  } else {
    acc.skipped++;
  }
  if (changed) acc.changed++;
  // predictor state (Fig. 6): success/fail edge for attempting states, the
  // unconditional step for dormant ones; a verification pass resets the
  // vertices it changes to the initial state.
  if (r.phase == 1) {
    if (changed && r.pvu == P_WEAK) r.status[v] = (uint8_t)r.dia->initial;
  } else if (r.pvu == P_WEAK) {
    uint8_t nx = (g.attempt && changed) ? r.dia->succ[g.st] : r.dia->fail[g.st];
    if (nx != g.st) r.status[v] = nx;
    atomicAdd(&r.hist[g.st], 1u);
  }
}

// ---------------------------------------------------- bins 0..5 and bin 8
// G lanes per vertex (G = 1..32), each lane <= 2 in-edges; every group
// handles SMALL_ROUNDS vertices whose loads are all issued before use.
template <int ALGO, int G>
__device__ void sweep_small(const Run &r, const PageCtx &p, int item, Acc &acc) {
  using R = Red<ALGO>;
  using T = typename R::T;
  constexpr int NG = BLOCK / G;
  constexpr int RR = SMALL_ROUNDS;
  const int grp = threadIdx.x / G, lane = threadIdx.x % G;
  const int base = item * NG * RR + grp;
  int32_t vl[RR];
  int32_t beg[RR], end[RR];
  Gate gt[RR];
  bool comp[RR];
#pragma unroll
  for (int k = 0; k < RR; ++k) gt[k] = Gate{false, 0, 0u};
#pragma unroll
  for (int k = 0; k < RR; ++k) {
    int idx = base + k * NG;
    vl[k] = idx < p.bin_count ? p.bins[p.bin_start + idx] : -1;
  }
#pragma unroll
  for (int k = 0; k < RR; ++k) {
    beg[k] = 0; end[k] = 0; comp[k] = false;
    if (vl[k] >= 0) {
      beg[k] = p.off[vl[k]];
      end[k] = p.off[vl[k] + 1];
      gt[k] = gate_of(r, p.v_begin + vl[k]);
      comp[k] = gt[k].attempt || r.audit;
    }
  }
  T red[RR];
  if constexpr (G >= 1) {
    int32_t s0[RR], s1[RR];
    uint32_t w0[RR], w1[RR];
#pragma unroll
    for (int k = 0; k < RR; ++k) {
      int e0 = beg[k] + lane, e1 = e0 + G;
      bool a0 = comp[k] && e0 < end[k], a1 = comp[k] && e1 < end[k];
      s0[k] = a0 ? p.src[e0] : -1;
      s1[k] = a1 ? p.src[e1] : -1;
      if (ALGO == A_SSSP) {
        w0[k] = a0 ? p.w[e0] : 0u;
        w1[k] = a1 ? p.w[e1] : 0u;
      } else {
        w0[k] = w1[k] = 0u;
      }
    }
#pragma unroll
    for (int k = 0; k < RR; ++k) {
      T x = R::identity();
      if (s0[k] >= 0) x = R::combine(x, R::edge(r, s0[k], w0[k]));
      if (s1[k] >= 0) x = R::combine(x, R::edge(r, s1[k], w1[k]));
#pragma unroll
      for (int m = G / 2; m >= 1; m >>= 1) x = R::combine(x, shfl_xor(x, m));
      red[k] = x;
    }
  }
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < RR; ++k)
      if (vl[k] >= 0)
        epilogue<ALGO>(r, p.v_begin + vl[k], gt[k], comp[k], red[k], (uint32_t)(end[k] - beg[k]), acc);
  }
}

// ----------------------------------------------------------------- bin 6
// One wavefront per vertex, 64 <= d <= HEAVY; 4 loads in flight per lane.
template <int ALGO>
__device__ void sweep_wave(const Run &r, const PageCtx &p, int item, Acc &acc) {
  using R = Red<ALGO>;
  using T = typename R::T;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
#pragma unroll 1
  for (int k = 0; k < WAVE_ROUNDS; ++k) {
    int idx = (item * WAVE_ROUNDS + k) * WAVES + wave;
    if (idx >= p.bin_count) break;
    int32_t vl = p.bins[p.bin_start + idx];
    int32_t v = p.v_begin + vl;
    int32_t beg = p.off[vl], end = p.off[vl + 1];
    Gate g = gate_of(r, v);
    bool comp = g.attempt || r.audit;
    T x = R::identity();
    if (comp) {
      int e = beg + lane;
      for (; e + 192 < end; e += 256) {
        int32_t u0 = p.src[e], u1 = p.src[e + 64], u2 = p.src[e + 128], u3 = p.src[e + 192];
        uint32_t a0 = 0, a1 = 0, a2 = 0, a3 = 0;
        if (ALGO == A_SSSP) { a0 = p.w[e]; a1 = p.w[e + 64]; a2 = p.w[e + 128]; a3 = p.w[e + 192]; }
        T y0 = R::edge(r, u0, a0), y1 = R::edge(r, u1, a1), y2 = R::edge(r, u2, a2), y3 = R::edge(r, u3, a3);
        x = R::combine(x, R::combine(R::combine(y0, y1), R::combine(y2, y3)));
      }
      for (; e < end; e += 64) x = R::combine(x, R::edge(r, p.src[e], ALGO == A_SSSP ? p.w[e] : 0u));
#pragma unroll
      for (int m = 32; m >= 1; m >>= 1) x = R::combine(x, shfl_xor(x, m));
    }
    if (lane == 0) epilogue<ALGO>(r, v, g, comp, x, (uint32_t)(end - beg), acc);
  }
}

// ----------------------------------------------------------------- bin 7
// One wavefront per CHUNK edges of a heavy vertex; the last chunk of the
// vertex to arrive combines the partials in chunk order and runs the
// epilogue (fence + arrival counter, the classic last-block pattern).
template <int ALGO>
__device__ void sweep_chunk(const Run &r, const PageCtx &p, int item, Acc &acc) {
  using R = Red<ALGO>;
  using T = typename R::T;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  int idx = item * WAVES + wave;
  if (idx >= p.bin_count) return;
  Chunk c = p.chunks[idx];
  int32_t v = p.v_begin + c.vl;
  int first = (int)((uint32_t)c.first_count & 0xFFFFFu), count = (int)((uint32_t)c.first_count >> 20);
  Gate g = gate_of(r, v);
  bool comp = g.attempt || r.audit;
  T x = R::identity();
  if (comp) {
    int e = c.e_begin + lane;
    for (; e + 192 < c.e_end; e += 256) {
      int32_t u0 = p.src[e], u1 = p.src[e + 64], u2 = p.src[e + 128], u3 = p.src[e + 192];
      uint32_t a0 = 0, a1 = 0, a2 = 0, a3 = 0;
      if (ALGO == A_SSSP) { a0 = p.w[e]; a1 = p.w[e + 64]; a2 = p.w[e + 128]; a3 = p.w[e + 192]; }
      T y0 = R::edge(r, u0, a0), y1 = R::edge(r, u1, a1), y2 = R::edge(r, u2, a2), y3 = R::edge(r, u3, a3);
      x = R::combine(x, R::combine(R::combine(y0, y1), R::combine(y2, y3)));
    }
    for (; e < c.e_end; e += 64) x = R::combine(x, R::edge(r, p.src[e], ALGO == A_SSSP ? p.w[e] : 0u));
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) x = R::combine(x, shfl_xor(x, m));
  }
  if (lane != 0) return;
  int32_t beg = p.off[c.vl], end = p.off[c.vl + 1];
  if (count == 1) {
    epilogue<ALGO>(r, v, g, comp, x, (uint32_t)(end - beg), acc);
    return;
  }
  st_agent(&p.partial[idx], R::bits(x));
  __threadfence();
  uint32_t ticket = atomicAdd(&p.arrive[first], 1u);
  if (ticket != (uint32_t)(count - 1)) return;
  __threadfence();
  T tot = R::identity();
  for (int j = 0; j < count; ++j) tot = R::combine(tot, R::from_bits(ld_agent(&p.partial[first + j])));
  st_agent(&p.arrive[first], 0u);
  epilogue<ALGO>(r, v, g, comp, tot, (uint32_t)(end - beg), acc);
}

// ------------------------------------------------------ end of pass logic
// Table I thresholds, the verification pass that recovers weak
// mispredictions (Section 4.3), and the PageRank stop rule.
__device__ void close_pass(Ctl *c, SweepRecord *rec) {
  c->pass += 1;
  const bool minprog = c->algo == A_BFS || c->algo == A_SSSP || c->algo == A_CC;
  if (rec) rec->pass_l1_closed = c->pass_l1;
  if (minprog) {
    if (c->phase == 1) {
      if (c->pass_changed == 0) { c->done = 1; c->stop_reason = 1; }
      else c->phase = 0;
    } else if (c->pass_changed == 0) {
      if (c->pvu == P_WEAK) c->phase = 1;
      else { c->done = 1; c->stop_reason = 1; }
    }
    if (c->pvu == P_STRONG && !c->done) {
      // BFS: after k passes every level <= k is final. SSSP/CC: nothing
      // can drop below the smallest value changed in the last pass.
      if (c->algo == A_BFS) c->threshold = c->pass;
      else if (c->pass_changed > 0) c->threshold = c->pass_min_changed;
    }
  } else {
    const double l1 = c->pass_l1;
    if (c->phase == 1) {
      if (l1 < c->best_l1) { c->best_l1 = l1; c->no_improve = 0; }
      else c->no_improve += 1;
      if (l1 < c->tol_l1) { c->done = 1; c->stop_reason = 1; }
      else if (l1 < c->floor_cap && c->no_improve >= 3) { c->done = 1; c->stop_reason = 2; }
    } else {
      if (l1 < c->best_l1) { c->best_l1 = l1; c->no_improve = 0; }
      else c->no_improve += 1;
      if (l1 < c->tol_l1 || (l1 < c->floor_cap && c->no_improve >= 3)) {
        c->phase = 1;
        c->best_l1 = 1e300;
        c->no_improve = 0;
      }
    }
  }
  if (!c->done && (int32_t)c->pass >= c->max_passes) { c->done = 1; c->stop_reason = 3; }
  c->pass_changed = 0;
  c->pass_min_changed = INF;
  c->pass_l1 = 0.0;
  if (rec) {
    rec->done_after = c->done;
    rec->pass_after = c->pass;
    rec->stop_reason = c->stop_reason;
  }
}

// Fold the sweep accumulators into the pass and publish the sweep record.
__device__ void close_sweep(Ctl *c, SweepRecord *ring, uint32_t mask, int end_of_pass) {
  uint32_t seq = c->sweep_seq;
  SweepRecord *rec = ring ? &ring[seq & mask] : nullptr;
  unsigned long long changed = ld_agent(&c->sw_changed);
  uint32_t minc = ld_agent(&c->sw_min_changed);
  double l1 = ld_agent(&c->sw_l1), dd = ld_agent(&c->sw_ddelta);
  if (rec) {
    rec->seq = seq;
    rec->changed = changed;
    rec->edges = ld_agent(&c->sw_edges);
    rec->attempted = ld_agent(&c->sw_attempted);
    rec->skipped = ld_agent(&c->sw_skipped);
    rec->mispred = ld_agent(&c->sw_mispred);
    rec->l1 = l1;
    rec->min_changed = minc;
    rec->threshold = c->threshold;
    rec->phase = c->phase;
    for (int i = 0; i < 8; ++i) rec->hist[i] = ld_agent(&c->sw_hist[i]);
    rec->pass_l1_closed = -1.0;
  }
  c->pass_changed += changed;
  c->pass_min_changed = min(c->pass_min_changed, minc);
  c->pass_l1 += l1;
  c->dangling += dd;
  st_agent(&c->sw_changed, 0ull); st_agent(&c->sw_edges, 0ull);
  st_agent(&c->sw_attempted, 0ull); st_agent(&c->sw_skipped, 0ull);
  st_agent(&c->sw_mispred, 0ull);
  for (int i = 0; i < 8; ++i) st_agent(&c->sw_hist[i], 0ull);
  st_agent(&c->sw_min_changed, INF);
  st_agent(&c->sw_l1, 0.0); st_agent(&c->sw_ddelta, 0.0);
  c->sweep_seq = seq + 1;
  if (end_of_pass) close_pass(c, rec);
  if (rec) {
    if (!end_of_pass) { rec->done_after = c->done; rec->pass_after = c->pass; rec->stop_reason = c->stop_reason; }
    rec->dangling = c->dangling;
  }
  st_agent(&c->blocks_done, 0u);
  __threadfence_system();
}

// ------------------------------------------------------------ the sweep
template <int ALGO>
__global__ void __launch_bounds__(BLOCK) sweep_kernel(SweepArgs a) {
  Ctl *ctl = a.ctl;
  if (ctl->done) return;  // converged: every block leaves before counting
  __shared__ uint32_t s_hist[8];
  __shared__ uint32_t s_u32[WAVES][6];
  __shared__ double s_f64[WAVES][2];
  if (threadIdx.x < 8) s_hist[threadIdx.x] = 0;

  // locate (page, bin, item) of this block
  const int b = blockIdx.x;
  int lo = 0, hi = a.nent * NBINS;  // prefix[lo] <= b < prefix[hi]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (a.blk_prefix[mid] <= b) lo = mid; else hi = mid;
  }
  const int ent = lo / NBINS, bin = lo % NBINS, item = b - a.blk_prefix[lo];
  const char *base = a.base[ent];
  const PageHeader *h = reinterpret_cast<const PageHeader *>(base);
  PageCtx p;
  p.v_begin = h->v_begin;
  p.off = reinterpret_cast<const int32_t *>(base + h->off_offsets);
  p.bins = reinterpret_cast<const int32_t *>(base + h->off_bins);
  p.chunks = reinterpret_cast<const Chunk *>(base + h->off_chunks);
  p.src = reinterpret_cast<const int32_t *>(base + h->off_src);
  p.w = reinterpret_cast<const uint32_t *>(base + h->off_w);
  p.bin_count = h->bin_count[bin];
  p.bin_start = h->bin_start[bin];
  p.partial = a.partial[ent];
  p.arrive = a.arrive[ent];

  Run r;
  r.algo = ALGO;
  r.pvu = ctl->pvu;
  r.phase = ctl->phase;
  r.audit = a.audit && r.phase == 0 && r.pvu != P_OFF;
  r.threshold = ctl->threshold;
  r.value = a.value;
  r.contrib = a.contrib;
  r.inv_outdeg = a.inv_outdeg;
  r.status = a.status;
  r.dia = &a.dia;
  r.damping = a.damping;
  r.pr_eps = a.pr_eps;
  r.base_uniform = 1.0f / (float)a.n;
  r.dangling = (float)ctl->dangling;
  r.pr_seed = a.pr_seed;
  r.hist = s_hist;
  __syncthreads();

  Acc acc;
  // a launch over pages without any work still runs one block, so the
  // sweep (and the pass) is closed the same way
  const int active_bin = b < a.blk_prefix[a.nent * NBINS] ? bin : -1;
  switch (active_bin) {
    case -1: break;
    case 0: sweep_small<ALGO, 1>(r, p, item, acc); break;
    case 1: sweep_small<ALGO, 2>(r, p, item, acc); break;
    case 2: sweep_small<ALGO, 4>(r, p, item, acc); break;
    case 3: sweep_small<ALGO, 8>(r, p, item, acc); break;
    case 4: sweep_small<ALGO, 16>(r, p, item, acc); break;
    case 5: sweep_small<ALGO, 32>(r, p, item, acc); break;
    case BIN_WAVE: sweep_wave<ALGO>(r, p, item, acc); break;
    case BIN_CHUNK: sweep_chunk<ALGO>(r, p, item, acc); break;
    case BIN_ZERO:
      if constexpr (is_pr<ALGO>()) {
        // zero in-degree: the pull sum is empty, the value still follows D
        for (int k = 0; k < 4; ++k) {
          int idx = (item * 4 + k) * BLOCK + threadIdx.x;
          if (idx < p.bin_count) {
            int32_t v = p.v_begin + p.bins[p.bin_start + idx];
            Gate g = gate_of(r, v);
            epilogue<ALGO>(r, v, g, g.attempt || r.audit, 0.0f, 0u, acc);
          }
        }
      }
      break;
  }

  // block reduction of the counters, one set of atomics per block
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  uint32_t v0 = wave_sum_u32(acc.changed), v1 = wave_sum_u32(acc.attempted),
           v2 = wave_sum_u32(acc.skipped), v3 = wave_sum_u32(acc.mispred),
           v4 = wave_sum_u32(acc.edges), v5 = wave_min_u32(acc.min_changed);
  double f0 = 0.0, f1 = 0.0;
  if constexpr (is_pr<ALGO>()) { f0 = wave_sum_f64(acc.l1); f1 = wave_sum_f64(acc.ddelta); }
  if (lane == 0) {
    s_u32[wave][0] = v0; s_u32[wave][1] = v1; s_u32[wave][2] = v2;
    s_u32[wave][3] = v3; s_u32[wave][4] = v4; s_u32[wave][5] = v5;
    s_f64[wave][0] = f0; s_f64[wave][1] = f1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t0 = 0, t1 = 0, t2 = 0, t3 = 0, t4 = 0;
    uint32_t mn = INF;
    double g0 = 0.0, g1 = 0.0;
    for (int w = 0; w < WAVES; ++w) {
      t0 += s_u32[w][0]; t1 += s_u32[w][1]; t2 += s_u32[w][2]; t3 += s_u32[w][3]; t4 += s_u32[w][4];
      mn = min(mn, s_u32[w][5]);
      g0 += s_f64[w][0]; g1 += s_f64[w][1];
    }
    if (t0) atomicAdd(&ctl->sw_changed, t0);
    if (t1) atomicAdd(&ctl->sw_attempted, t1);
    if (t2) atomicAdd(&ctl->sw_skipped, t2);
    if (t3) atomicAdd(&ctl->sw_mispred, t3);
    if (t4) atomicAdd(&ctl->sw_edges, t4);
    if (mn != INF) atomicMin(&ctl->sw_min_changed, mn);
    if constexpr (is_pr<ALGO>()) {
      if (g0 != 0.0) atomicAdd(&ctl->sw_l1, g0);
      if (g1 != 0.0) atomicAdd(&ctl->sw_ddelta, g1);
    }
    for (int i = 0; i < 8; ++i)
      if (s_hist[i]) atomicAdd(&ctl->sw_hist[i], (unsigned long long)s_hist[i]);
    __threadfence();
    uint32_t ticket = atomicAdd(&ctl->blocks_done, 1u);
    if (ticket == (uint32_t)(a.nblocks - 1)) {
      __threadfence();
      close_sweep(ctl, a.ring, a.ring_mask, a.end_of_pass);
    }
  }
}

__global__ void end_pass_kernel(Ctl *ctl, SweepRecord *ring, uint32_t mask) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (ctl->done) return;
  // a pass closed on its own gets a record of its own (no sweep counters)
  uint32_t seq = ctl->sweep_seq;
  SweepRecord *rec = ring ? &ring[seq & mask] : nullptr;
  if (rec) {
    rec->seq = seq; rec->changed = 0; rec->edges = 0; rec->attempted = 0; rec->skipped = 0;
    rec->mispred = 0; rec->l1 = 0.0; rec->min_changed = INF; rec->threshold = ctl->threshold;
    rec->phase = ctl->phase;
    for (int i = 0; i < 8; ++i) rec->hist[i] = 0;
  }
  ctl->sweep_seq = seq + 1;
  close_pass(ctl, rec);
  if (rec) rec->dangling = ctl->dangling;
  __threadfence_system();
}

template <int ALGO>
__global__ void init_min_kernel(uint32_t *value, int32_t n, int32_t source) {
  int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  if (ALGO == A_CC) value[v] = (uint32_t)v;
  else value[v] = (v == source) ? 0u : INF;
}

__global__ void init_pr_kernel(float *rank, float *contrib, const float *inv_outdeg, int32_t n,
                               int32_t seed) {
  int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  float x = seed < 0 ? 1.0f / (float)n : (v == seed ? 1.0f : 0.0f);
  rank[v] = x;
  contrib[v] = x * inv_outdeg[v];
}

__global__ void fill_u8_kernel(uint8_t *p, uint8_t v, size_t count) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < count; i += stride) p[i] = v;
}

__global__ void fill_u32_kernel(uint32_t *p, uint32_t v, size_t count) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < count; i += stride) p[i] = v;
}

__global__ void init_ctl_kernel(Ctl *ctl, Ctl init) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *ctl = init;
}

}  // namespace

hipError_t launch_sweep(int algo, const SweepArgs &a, hipStream_t s) {
  if (a.nblocks <= 0) return hipErrorInvalidValue;
  dim3 grid(a.nblocks), block(BLOCK);
  switch (algo) {
    case A_BFS: hipLaunchKernelGGL(sweep_kernel<A_BFS>, grid, block, 0, s, a); break;
    case A_SSSP: hipLaunchKernelGGL(sweep_kernel<A_SSSP>, grid, block, 0, s, a); break;
    case A_CC: hipLaunchKernelGGL(sweep_kernel<A_CC>, grid, block, 0, s, a); break;
    case A_PR: hipLaunchKernelGGL(sweep_kernel<A_PR>, grid, block, 0, s, a); break;
    case A_PPR: hipLaunchKernelGGL(sweep_kernel<A_PPR>, grid, block, 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_end_pass(Ctl *ctl, SweepRecord *ring, uint32_t mask, hipStream_t s) {
  hipLaunchKernelGGL(end_pass_kernel, dim3(1), dim3(64), 0, s, ctl, ring, mask);
  return hipGetLastError();
}

hipError_t launch_init_min(int algo, uint32_t *value, int32_t n, int32_t source, hipStream_t s) {
  dim3 grid((n + 255) / 256), block(256);
  if (algo == A_CC) hipLaunchKernelGGL(init_min_kernel<A_CC>, grid, block, 0, s, value, n, source);
  else hipLaunchKernelGGL(init_min_kernel<A_SSSP>, grid, block, 0, s, value, n, source);
  return hipGetLastError();
}

hipError_t launch_init_pr(float *rank, float *contrib, const float *inv_outdeg, int32_t n,
                          int32_t seed, hipStream_t s) {
  hipLaunchKernelGGL(init_pr_kernel, dim3((n + 255) / 256), dim3(256), 0, s, rank, contrib,
                     inv_outdeg, n, seed);
  return hipGetLastError();
}

hipError_t launch_fill_u8(uint8_t *p, uint8_t v, size_t count, hipStream_t s) {
  if (!count) return hipSuccess;
  size_t blocks = (count + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(fill_u8_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, v, count);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, size_t count, hipStream_t s) {
  if (!count) return hipSuccess;
  size_t blocks = (count + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, v, count);
  return hipGetLastError();
}

hipError_t launch_init_ctl(Ctl *ctl, const Ctl &init, hipStream_t s) {
  hipLaunchKernelGGL(init_ctl_kernel, dim3(1), dim3(64), 0, s, ctl, init);
  return hipGetLastError();
}

}  // namespace sr
