// batch.hip -- multi-instance pull sweep for gfx950: K instances (K = 8 or
// 16; 32 for SSSP/BFS) of personalized PageRank, SSSP or BFS on resident graphs, several
// graphs in one persistent launch. A wavefront is split into 64/K edge
// lanes x K instance lanes: the K lanes of one edge lane load the same
// in-edge source (one broadcast load) and gather the K contiguous values of
// that neighbour (one 4K-byte access), so every index and weight read is
// shared by K instances. Blocks take work items from a device queue until
// it is empty and accumulate per-instance counters in LDS, flushed once per
// block. Heavy-vertex chunks fold their partials into per-vertex
// accumulators with device-scope atomics; a heavy-vertex kernel (one thread
// per vertex and instance) then runs their epilogues, and a one-block close
// kernel closes the sweep for every instance (convergence, thresholds,
// PageRank dangling mass). The three launches are replayed from a captured
// graph with no host work in between; no fence is executed inside the sweep.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "batch.hpp"

namespace sr {

namespace {
constexpr int MI_CLOSE_THREADS = 1024;

template <typename T>
__device__ inline T shfl_xor(T v, int m) { return __shfl_xor(v, m, 64); }
}  // namespace

// vertices (bins 0..6, 8) or chunks (bin 7) per work item of the multi-
// instance sweep with K instance lanes
// A heavy-vertex chunk is split over K/8 wavefronts (at least one): with
// 64/K edge lanes per wavefront, wide instance groups would otherwise leave
// one wavefront a long serial edge loop.
__host__ __device__ constexpr int mi_subchunks(int K) { return K >= 16 ? K / 8 : 1; }

// ROUNDS: rounds of vertices a wavefront takes per item in the small-degree
// bins (the items-per-block choice of the schedule)
__host__ __device__ inline int mi_items_per_block(int b, int K, int ROUNDS) {
  const int EL = 64 / K;
  if (b <= 5) {
    int GE = (1 << b) < EL ? (1 << b) : EL;
    return WAVES * ROUNDS * (EL / GE);
  }
  if (b == BIN_WAVE) return WAVES;
  if (b == BIN_CHUNK) return WAVES / mi_subchunks(K);  // chunks: WAVES sub-chunks per item
  return ROUNDS * (BLOCK / K);
}

namespace {

template <int ALGO>
constexpr bool mi_pr() { return ALGO == A_PPR; }

// Per-lane state of one instance column for the current item.
struct Lane {
  uint32_t active, unit, threshold;
  int32_t source;
  double dangling, inv_mass;
};

__device__ inline Lane lane_of(const MiInst &in) {
  Lane ln;
  ln.active = in.active;
  ln.unit = in.unit;
  ln.threshold = in.threshold;
  ln.source = in.source;
  ln.dangling = in.dangling;
  ln.inv_mass = in.mass > 0.0 ? 1.0 / in.mass : 1.0;
  return ln;
}

template <int ALGO, int K>
struct MiRed {
  using T = typename std::conditional<mi_pr<ALGO>(), float, uint32_t>::type;
  __device__ static inline T identity() {
    if constexpr (mi_pr<ALGO>()) return 0.0f; else return INF;
  }
  __device__ static inline T combine(T a, T b) {
    if constexpr (mi_pr<ALGO>()) return a + b; else return min(a, b);
  }
  __device__ static inline T edge(const MiGroup &g, int32_t u, uint32_t w, int k, const Lane &ln) {
    if constexpr (mi_pr<ALGO>()) {
      return g.contrib[(size_t)u * K + k];
    } else {
      uint32_t x = g.value[(size_t)u * K + k];
      if (x == INF) return INF;
      uint64_t c = (uint64_t)x + (ln.unit ? 1ull : (uint64_t)w);
      return c >= (uint64_t)INF ? INF : (uint32_t)c;
    }
  }
  __device__ static inline uint32_t bits(T v) {
    if constexpr (mi_pr<ALGO>()) return __float_as_uint(v); else return v;
  }
  __device__ static inline T from_bits(uint32_t b) {
    if constexpr (mi_pr<ALGO>()) return __uint_as_float(b); else return b;
  }
};

struct MiAcc {
  uint32_t changed = 0, min_changed = INF, edges = 0;
  double l1 = 0.0, ddelta = 0.0, dmass = 0.0;
};

// Per-instance counters of one block, in LDS (instance i = group * K + k).
struct MiLds {
  uint32_t changed, min_changed, edges, pad;
  double l1, ddelta, dmass;
};

__device__ inline void lds_clear(MiLds *lds, int n, int nthreads) {
  for (int i = threadIdx.x; i < n; i += nthreads) {
    lds[i].changed = 0;
    lds[i].min_changed = INF;
    lds[i].edges = 0;
    lds[i].pad = 0;
    lds[i].l1 = 0.0;
    lds[i].ddelta = 0.0;
    lds[i].dmass = 0.0;
  }
}

template <int ALGO>
__device__ inline void lds_add(MiLds &e, const MiAcc &acc) {
  if (acc.changed) atomicAdd(&e.changed, acc.changed);
  if (acc.min_changed != INF) atomicMin(&e.min_changed, acc.min_changed);
  if (acc.edges) atomicAdd(&e.edges, acc.edges);
  if constexpr (mi_pr<ALGO>()) {
    if (acc.l1 != 0.0) atomicAdd(&e.l1, acc.l1);
    if (acc.ddelta != 0.0) atomicAdd(&e.ddelta, acc.ddelta);
    if (acc.dmass != 0.0) atomicAdd(&e.dmass, acc.dmass);
  }
}

template <int ALGO, int K>
__device__ inline bool mi_attempt(const MiGroup &g, int32_t v, int k, const Lane &ln, uint32_t &old) {
  old = g.value[(size_t)v * K + k];
  if (!ln.active) return false;
  if constexpr (!mi_pr<ALGO>()) {
    if (g.pvu == P_STRONG && old <= ln.threshold) return false;  // Table I
  }
  return true;
}

template <int ALGO, int K>
__device__ inline void mi_epilogue(const MiGroup &g, int32_t v, int k, const Lane &ln, uint32_t old,
                                   typename MiRed<ALGO, K>::T red, uint32_t deg, double damping, MiAcc &acc) {
  acc.edges += deg;
  const size_t i = (size_t)v * K + k;
  if constexpr (mi_pr<ALGO>()) {
    // the update of x / mass (see the single-instance epilogue)
    const double t = (v == ln.source) ? 1.0 : 0.0;
    float oldf = __uint_as_float(old);
    float nv = (float)((1.0 - damping) * t + damping * ln.inv_mass * ((double)red + ln.dangling * t));
    g.value[i] = __float_as_uint(nv);
    float iod = g.inv_outdeg[v];
    g.contrib[i] = nv * iod;
    double dd = (double)nv - (double)oldf;
    acc.l1 += fabs(dd);
    acc.dmass += dd;
    if (iod == 0.0f) acc.ddelta += dd;
    if (nv != oldf) acc.changed++;
  } else {
    uint32_t nv = min(old, red);
    if (nv < old) {
      g.value[i] = nv;
      acc.changed++;
      acc.min_changed = min(acc.min_changed, nv);
    }
  }
}

// lanes with the same instance k reduce over the 64/K edge lanes; lanes
// 0..K-1 add the per-instance totals to the block's LDS counters
template <int ALGO, int K>
__device__ inline void mi_flush(MiLds *lds, int group, MiAcc &acc) {
  const int lane = threadIdx.x % 64;
#pragma unroll
  for (int m = K; m < 64; m <<= 1) {
    acc.changed += shfl_xor(acc.changed, m);
    acc.min_changed = min(acc.min_changed, shfl_xor(acc.min_changed, m));
    acc.edges += shfl_xor(acc.edges, m);
    if constexpr (mi_pr<ALGO>()) {
      acc.l1 += shfl_xor(acc.l1, m);
      acc.ddelta += shfl_xor(acc.ddelta, m);
      acc.dmass += shfl_xor(acc.dmass, m);
    }
  }
  if (lane < K) lds_add<ALGO>(lds[group * K + lane], acc);
  acc = MiAcc();
}

// bins 0..5: GE edge lanes per vertex (GE = min(2^b, 64/K)), ROUNDS
// rounds of 64/K/GE vertices per wavefront
// Weight of in-edge e with edge word q (1 for unweighted programs).
template <int ALGO>
__device__ inline uint32_t mi_weight(const MiGroup &g, uint32_t q, const uint32_t *wt, int32_t e) {
  if (ALGO != A_SSSP || !g.has_w) return 1u;
  return g.packed ? q >> 24 : wt[e];
}

template <int ALGO, int K, int GE, int ROUNDS>
__device__ void mi_small(const MiGroup &g, const char *base, const PageHeader *h, int bin, int item,
                         const Lane &ln, double damping, MiAcc &acc) {
  using R = MiRed<ALGO, K>;
  using T = typename R::T;
  constexpr int EL = 64 / K;
  constexpr int VPW = EL / GE;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int k = lane % K, el = lane / K, vs = el / GE, ein = el % GE;
  const int32_t *off = reinterpret_cast<const int32_t *>(base + h->off_offsets);
  const int32_t *bins = reinterpret_cast<const int32_t *>(base + h->off_bins) + h->bin_start[bin];
  const uint32_t *src = reinterpret_cast<const uint32_t *>(base + h->off_src);
  const uint32_t *wt = reinterpret_cast<const uint32_t *>(base + h->off_w);
  const int cnt = h->bin_count[bin];
  const int vb = h->v_begin;
  int32_t vl[ROUNDS], beg[ROUNDS], end[ROUNDS];
  uint32_t old[ROUNDS];
  bool att[ROUNDS];
#pragma unroll
  for (int r = 0; r < ROUNDS; ++r) {
    // loads are unconditional (lanes past the bin reread its first vertex)
    // so the rounds' bin, offset and value loads overlap
    const int idx = ((item * WAVES + wave) * ROUNDS + r) * VPW + vs;
    const bool ok = idx < cnt;
    vl[r] = cnt > 0 ? bins[ok ? idx : 0] : 0;  // an empty bin rereads the page's vertex 0
    beg[r] = off[vl[r]];
    end[r] = off[vl[r] + 1];
    old[r] = 0;
    att[r] = mi_attempt<ALGO, K>(g, vb + vl[r], k, ln, old[r]) && ok;
    if (!ok) vl[r] = -1;
  }
#pragma unroll
  for (int r = 0; r < ROUNDS; ++r) {
    T x = R::identity();
    if (att[r]) {
      // batches of 4 edges per lane: word loads, then gathers, in flight together
      for (int e0 = beg[r] + ein; e0 < end[r]; e0 += 4 * GE) {
        int32_t ei[4];
        uint32_t q[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          ei[j] = e0 + j * GE < end[r] ? e0 + j * GE : e0;
          q[j] = src[ei[j]];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const T y = R::edge(g, (int32_t)(q[j] & g.src_mask), mi_weight<ALGO>(g, q[j], wt, ei[j]), k, ln);
          if (e0 + j * GE < end[r]) x = R::combine(x, y);
        }
      }
    }
#pragma unroll
    for (int m = K; m < K * GE; m <<= 1) x = R::combine(x, shfl_xor(x, m));
    if (att[r] && ein == 0)
      mi_epilogue<ALGO, K>(g, vb + vl[r], k, ln, old[r], x, (uint32_t)(end[r] - beg[r]), damping, acc);
  }
}

// edge loop of bins 6 and 7: 64/K edge lanes, 8 edges in flight per lane
template <int ALGO, int K>
__device__ inline typename MiRed<ALGO, K>::T mi_edges(const MiGroup &g, const uint32_t *src, const uint32_t *wt,
                                                      int32_t e0, int32_t e1, int k, int el, const Lane &ln) {
  using R = MiRed<ALGO, K>;
  using T = typename R::T;
  constexpr int EL = 64 / K;
  T x = R::identity();
  constexpr int B = 8;
  for (int e = e0 + el; e < e1; e += B * EL) {
    int32_t ei[B];
    uint32_t q[B];
#pragma unroll
    for (int j = 0; j < B; ++j) {
      ei[j] = e + j * EL < e1 ? e + j * EL : e;  // past the range: reread a real edge
      q[j] = src[ei[j]];
    }
#pragma unroll
    for (int j = 0; j < B; ++j) {
      const T y = R::edge(g, (int32_t)(q[j] & g.src_mask), mi_weight<ALGO>(g, q[j], wt, ei[j]), k, ln);
      if (e + j * EL < e1) x = R::combine(x, y);
    }
  }
#pragma unroll
  for (int m = K; m < 64; m <<= 1) x = R::combine(x, shfl_xor(x, m));
  return x;
}

// bin 6: one wavefront per vertex
template <int ALGO, int K>
__device__ void mi_wave(const MiGroup &g, const char *base, const PageHeader *h, int item, const Lane &ln,
                        double damping, MiAcc &acc) {
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64, k = lane % K, el = lane / K;
  int idx = item * WAVES + wave;
  if (idx >= h->bin_count[BIN_WAVE]) return;
  const int32_t *off = reinterpret_cast<const int32_t *>(base + h->off_offsets);
  const int32_t vl = reinterpret_cast<const int32_t *>(base + h->off_bins)[h->bin_start[BIN_WAVE] + idx];
  const uint32_t *src = reinterpret_cast<const uint32_t *>(base + h->off_src);
  const uint32_t *wt = reinterpret_cast<const uint32_t *>(base + h->off_w);
  const int32_t v = h->v_begin + vl;
  uint32_t old;
  bool att = mi_attempt<ALGO, K>(g, v, k, ln, old);
  if (!__any(att)) return;  // lanes of other instances still share the index loads
  auto x = mi_edges<ALGO, K>(g, src, wt, off[vl], off[vl + 1], k, el, ln);
  if (att && el == 0) mi_epilogue<ALGO, K>(g, v, k, ln, old, x, (uint32_t)(off[vl + 1] - off[vl]), damping, acc);
}

// bin 7: one wavefront per chunk; each instance column folds its partial
// into the heavy vertex's accumulator
template <int ALGO, int K>
__device__ void mi_chunk(const MiGroup &g, const MiUnit &u, const char *base, const PageHeader *h, int item,
                         const Lane &ln) {
  using R = MiRed<ALGO, K>;
  using T = typename R::T;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64, k = lane % K, el = lane / K;
  constexpr int S = mi_subchunks(K);
  const int sidx = item * WAVES + wave;
  const int idx = sidx / S, sub = sidx % S;
  if (idx >= h->bin_count[BIN_CHUNK]) return;
  const Chunk c = reinterpret_cast<const Chunk *>(base + h->off_chunks)[idx];
  const int32_t len = (c.e_end - c.e_begin + S - 1) / S;
  const int32_t sb = c.e_begin + sub * len, se = min(c.e_end, sb + len);
  if (sb >= se) return;
  const uint32_t *src = reinterpret_cast<const uint32_t *>(base + h->off_src);
  const uint32_t *wt = reinterpret_cast<const uint32_t *>(base + h->off_w);
  const int32_t v = h->v_begin + c.vl;
  uint32_t old;
  bool att = mi_attempt<ALGO, K>(g, v, k, ln, old);
  T x = R::identity();
  if (__any(att)) x = mi_edges<ALGO, K>(g, src, wt, sb, se, k, el, ln);
  // fold into the vertex's accumulator (one device-scope atomic per chunk
  // and instance); the heavy-vertex kernel takes it after the sweep
  if (el == 0 && att) {
    unsigned long long *slot = &u.acc[(size_t)((uint32_t)c.first_count & 0xFFFFFu) * K + k];
    if constexpr (mi_pr<ALGO>()) atomicAdd(slot, (unsigned long long)llrint((double)x * FIX_ONE));
    else if (x != INF) atomicMin(reinterpret_cast<uint32_t *>(slot), (uint32_t)x);
  }
}

// bin 8 (PPR only): zero in-degree, the value still follows the teleport term
template <int ALGO, int K, int ROUNDS>
__device__ void mi_zero(const MiGroup &g, const char *base, const PageHeader *h, int item, const Lane &ln,
                        double damping, MiAcc &acc) {
  const int k = threadIdx.x % K, vs = threadIdx.x / K;
  const int32_t *bins = reinterpret_cast<const int32_t *>(base + h->off_bins) + h->bin_start[BIN_ZERO];
  const int cnt = h->bin_count[BIN_ZERO];
  for (int r = 0; r < ROUNDS; ++r) {
    int idx = (item * ROUNDS + r) * (BLOCK / K) + vs;
    if (idx >= cnt) break;
    int32_t v = h->v_begin + bins[idx];
    uint32_t old;
    if (mi_attempt<ALGO, K>(g, v, k, ln, old))
      mi_epilogue<ALGO, K>(g, v, k, ln, old, typename MiRed<ALGO, K>::T(0), 0u, damping, acc);
  }
}

template <int ALGO, int K, int ROUNDS>
__global__ void __launch_bounds__(BLOCK) mi_sweep_kernel(MiArgs a) {
  if (a.ctl->remaining == 0 && !a.tuning) return;  // everything converged: replays are no-ops
  extern __shared__ MiLds lds[];
  __shared__ int32_t s_base;
  const int ninst = a.ngroups * K;
  lds_clear(lds, ninst, BLOCK);
  const int lane = threadIdx.x % 64, k = lane % K;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) s_base = (int32_t)atomicAdd(&a.ctl->queue, (uint32_t)a.grab);
    __syncthreads();
    const int32_t base = s_base;
    if (base >= a.total_items) break;
    const int32_t end = min(base + a.grab, a.total_items);
    for (int32_t it = base; it < end; ++it) {
      int lo = 0, hi = a.nunits;  // unit_prefix[lo] <= it < unit_prefix[hi]
      while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (a.unit_prefix[mid] <= it) lo = mid; else hi = mid;
      }
      const MiUnit &u = a.units[lo];
      if (a.group_active[u.group] == 0) continue;  // no live instance in this group
      const MiGroup &g = a.groups[u.group];
      const int local = it - a.unit_prefix[lo];
      int bin = 0;
      while (bin < NBINS - 1 && u.blk_prefix[bin + 1] <= local) ++bin;
      const int item = local - u.blk_prefix[bin];
      const char *bp = u.page;
      const PageHeader *h = reinterpret_cast<const PageHeader *>(bp);
      const Lane ln = lane_of(g.inst[k]);
      MiAcc acc;
      switch (bin) {
        case 0: mi_small<ALGO, K, 1, ROUNDS>(g, bp, h, 0, item, ln, a.damping, acc); break;
        case 1: mi_small<ALGO, K, (2 < 64 / K ? 2 : 64 / K), ROUNDS>(g, bp, h, 1, item, ln, a.damping, acc); break;
        case 2: mi_small<ALGO, K, (4 < 64 / K ? 4 : 64 / K), ROUNDS>(g, bp, h, 2, item, ln, a.damping, acc); break;
        case 3: mi_small<ALGO, K, (8 < 64 / K ? 8 : 64 / K), ROUNDS>(g, bp, h, 3, item, ln, a.damping, acc); break;
        case 4: mi_small<ALGO, K, (16 < 64 / K ? 16 : 64 / K), ROUNDS>(g, bp, h, 4, item, ln, a.damping, acc); break;
        case 5: mi_small<ALGO, K, (32 < 64 / K ? 32 : 64 / K), ROUNDS>(g, bp, h, 5, item, ln, a.damping, acc); break;
        case BIN_WAVE: mi_wave<ALGO, K>(g, bp, h, item, ln, a.damping, acc); break;
        case BIN_CHUNK: mi_chunk<ALGO, K>(g, u, bp, h, item, ln); break;
        default:
          if constexpr (mi_pr<ALGO>()) mi_zero<ALGO, K, ROUNDS>(g, bp, h, item, ln, a.damping, acc);
          break;
      }
      mi_flush<ALGO, K>(lds, u.group, acc);
    }
  }
  // publish this block's per-instance counters (device-scope atomics on
  // distinct instance records; the close kernel reads them after the sweep)
  __syncthreads();
  for (int i = threadIdx.x; i < ninst; i += BLOCK) {
    const MiLds &e = lds[i];
    if (e.changed == 0 && e.edges == 0 && e.min_changed == INF && e.l1 == 0.0 && e.ddelta == 0.0 &&
        e.dmass == 0.0)
      continue;
    MiInst &in = a.groups[i / K].inst[i % K];
    if (e.changed) atomicAdd(&in.sw_changed, e.changed);
    if (e.min_changed != INF) atomicMin(&in.sw_min_changed, e.min_changed);
    if (e.edges) atomicAdd(&in.sw_edges, (unsigned long long)e.edges);
    if constexpr (mi_pr<ALGO>()) {
      if (e.l1 != 0.0) atomicAdd(&in.sw_l1, e.l1);
      if (e.ddelta != 0.0) atomicAdd(&in.sw_ddelta, e.ddelta);
      if (e.dmass != 0.0) atomicAdd(&in.sw_dmass, e.dmass);
    }
  }
}

// Heavy vertices after a sweep: one thread per (heavy vertex, instance)
// takes the vertex's accumulator with an exchange (leaving the identity),
// runs the epilogue and adds its counters to the instance's sweep totals.
template <int ALGO, int K>
__global__ void __launch_bounds__(BLOCK) mi_heavy_kernel(MiArgs a) {
  using R = MiRed<ALGO, K>;
  using T = typename R::T;
  if (a.ctl->remaining == 0 && !a.tuning) return;
  const int64_t p = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  const int32_t hh = (int32_t)(p / K), k = (int32_t)(p % K);
  if (hh >= a.total_heavy) return;
  int lo = 0, hi = a.nunits;  // units[lo].heavy_base <= hh < units[lo + 1].heavy_base
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (a.units[mid].heavy_base <= hh) lo = mid; else hi = mid;
  }
  const MiUnit &u = a.units[lo];
  if (a.group_active[u.group] == 0) return;  // the sweep skipped the group: accumulators untouched
  const MiGroup &g = a.groups[u.group];
  const PageHeader *h = reinterpret_cast<const PageHeader *>(u.page);
  const Heavy x = reinterpret_cast<const Heavy *>(u.page + h->off_heavy)[hh - u.heavy_base];
  const int32_t *off = reinterpret_cast<const int32_t *>(u.page + h->off_offsets);
  unsigned long long *slot = &u.acc[(size_t)((uint32_t)x.first_count & 0xFFFFFu) * K + k];
  T t;
  if constexpr (mi_pr<ALGO>()) t = (float)((double)(long long)atomicExch(slot, 0ull) / FIX_ONE);
  else t = atomicExch(reinterpret_cast<uint32_t *>(slot), INF);
  const int32_t v = h->v_begin + x.vl;
  const Lane ln = lane_of(g.inst[k]);
  uint32_t old;
  if (!mi_attempt<ALGO, K>(g, v, k, ln, old)) return;
  MiAcc acc;
  mi_epilogue<ALGO, K>(g, v, k, ln, old, t, (uint32_t)(off[x.vl + 1] - off[x.vl]), a.damping, acc);
  MiInst &in = g.inst[k];
  if (acc.changed) atomicAdd(&in.sw_changed, acc.changed);
  if (acc.min_changed != INF) atomicMin(&in.sw_min_changed, acc.min_changed);
  if (acc.edges) atomicAdd(&in.sw_edges, (unsigned long long)acc.edges);
  if constexpr (mi_pr<ALGO>()) {
    if (acc.l1 != 0.0) atomicAdd(&in.sw_l1, acc.l1);
    if (acc.ddelta != 0.0) atomicAdd(&in.sw_ddelta, acc.ddelta);
    if (acc.dmass != 0.0) atomicAdd(&in.sw_dmass, acc.dmass);
  }
}

// Close a sweep: close every instance (convergence, thresholds, dangling
// mass) from its sweep totals and reset the queue. One block, after the
// sweep and the heavy-vertex kernel.
template <int ALGO, int K>
__global__ void __launch_bounds__(MI_CLOSE_THREADS) mi_close_kernel(MiArgs a) {
  if (a.ctl->remaining == 0 && !a.tuning) return;
  __shared__ uint32_t s_rem;
  const int ninst = a.ngroups * K;
  if (threadIdx.x == 0) s_rem = 0;
  for (int gi = threadIdx.x; gi < a.ngroups; gi += MI_CLOSE_THREADS) a.group_active[gi] = 0;
  __syncthreads();
  for (int i = threadIdx.x; i < ninst; i += MI_CLOSE_THREADS) {
    MiInst &in = a.groups[i / K].inst[i % K];
    if (!in.active) continue;
    const uint32_t changed = in.sw_changed;
    const uint32_t minc = in.sw_min_changed;
    const double l1 = in.sw_l1, dd = in.sw_ddelta, dm = in.sw_dmass;
    in.edges_total += in.sw_edges;
    in.sweeps += 1;
    bool done = false;
    if constexpr (mi_pr<ALGO>()) {
      in.dangling += dd;
      in.mass += dm;
      in.last_l1 = l1;
      // FP32 floor: an improvement is an L1 at least 10% below the best so far
      const bool better = l1 < 0.9 * in.best_l1;
      in.no_improve = better ? 0 : in.no_improve + 1;
      in.best_l1 = better ? l1 : fmin(in.best_l1, l1);
      if (l1 < a.tol_l1) { done = true; in.stop_reason = 1; }
      else if (l1 < a.floor_cap && in.no_improve >= 3) { done = true; in.stop_reason = 2; }
    } else {
      if (changed == 0) { done = true; in.stop_reason = 1; }
      else if (a.groups[i / K].pvu == P_STRONG) in.threshold = in.unit ? in.sweeps : minc;
    }
    if (!done && (int32_t)in.sweeps >= a.max_sweeps) { done = true; in.stop_reason = 3; }
    if (a.tuning) done = false;
    in.sw_changed = 0;
    in.sw_min_changed = INF;
    in.sw_edges = 0;
    in.sw_l1 = 0.0;
    in.sw_ddelta = 0.0;
    in.sw_dmass = 0.0;
    if (done) { in.done = 1; in.active = 0; }
    else { atomicAdd(&s_rem, 1u); atomicAdd(&a.group_active[i / K], 1u); }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    a.ctl->remaining = s_rem;
    a.ctl->sweeps += 1;
    a.ctl->queue = 0;
    if (a.host_remaining) *a.host_remaining = s_rem;
    __threadfence_system();
  }
}

template <int ALGO, int K>
__global__ void mi_init_column_kernel(uint32_t *value, float *contrib, const float *inv_outdeg, int32_t n,
                                      int32_t col, int32_t source) {
  int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  size_t i = (size_t)v * K + col;
  if constexpr (mi_pr<ALGO>()) {
    float x = v == source ? 1.0f : 0.0f;
    value[i] = __float_as_uint(x);
    contrib[i] = x * inv_outdeg[v];
  } else {
    value[i] = v == source ? 0u : INF;
  }
}

__global__ void mi_set_inst_kernel(MiInst *dst, MiInst val) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dst = val;
}

__global__ void mi_set_ctl_kernel(MiCtl *dst, MiCtl val) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dst = val;
}

// Several columns in one pass: the columns of a vertex share its row of
// 4K bytes, so the row is fetched from memory once for all of them.
template <int K>
__global__ void mi_extract_kernel(uint32_t *value, int32_t n, MiExtract x, int32_t reset, uint32_t reset_to,
                                  const int32_t *rank) {
  int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  uint32_t *row = value + (size_t)(rank ? rank[v] : v) * K;
  for (int j = 0; j < x.count; ++j) {
    x.out[j][v] = row[x.col[j]];
    if (reset) row[x.col[j]] = reset_to;
  }
}

template <int ALGO, int K>
void mi_pair(const MiArgs &a, hipStream_t s) {
  const size_t lds = sizeof(MiLds) * (size_t)a.ngroups * K;
  if (a.rounds == 2) hipLaunchKernelGGL((mi_sweep_kernel<ALGO, K, 2>), dim3(a.nblocks), dim3(BLOCK), lds, s, a);
  else if (a.rounds == 8) hipLaunchKernelGGL((mi_sweep_kernel<ALGO, K, 8>), dim3(a.nblocks), dim3(BLOCK), lds, s, a);
  else hipLaunchKernelGGL((mi_sweep_kernel<ALGO, K, 4>), dim3(a.nblocks), dim3(BLOCK), lds, s, a);
  hipLaunchKernelGGL((mi_heavy_kernel<ALGO, K>), dim3(a.heavy_blocks), dim3(BLOCK), 0, s, a);
  hipLaunchKernelGGL((mi_close_kernel<ALGO, K>), dim3(1), dim3(MI_CLOSE_THREADS), 0, s, a);
}

}  // namespace

int mi_items_per_block_host(int b, int K, int rounds) { return mi_items_per_block(b, K, rounds); }

hipError_t launch_mi_sweep(int algo, int K, const MiArgs &a, hipStream_t s) {
  if (a.nblocks <= 0) return hipErrorInvalidValue;
  if (a.ngroups * K > MI_MAX_INSTANCES) return hipErrorInvalidValue;
  if (a.rounds != 2 && a.rounds != 4 && a.rounds != 8) return hipErrorInvalidValue;
  if (algo == A_PPR && K == 8) mi_pair<A_PPR, 8>(a, s);
  else if (algo == A_PPR && K == 16) mi_pair<A_PPR, 16>(a, s);
  else if (algo == A_SSSP && K == 8) mi_pair<A_SSSP, 8>(a, s);
  else if (algo == A_SSSP && K == 16) mi_pair<A_SSSP, 16>(a, s);
  else if (algo == A_SSSP && K == 32) mi_pair<A_SSSP, 32>(a, s);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_mi_init_column(int algo, int K, uint32_t *value, float *contrib, const float *inv_outdeg,
                                 int32_t n, int32_t col, int32_t source, hipStream_t s) {
  dim3 grid((n + 255) / 256), block(256);
  if (algo == A_PPR && K == 8) hipLaunchKernelGGL((mi_init_column_kernel<A_PPR, 8>), grid, block, 0, s, value, contrib, inv_outdeg, n, col, source);
  else if (algo == A_PPR && K == 16) hipLaunchKernelGGL((mi_init_column_kernel<A_PPR, 16>), grid, block, 0, s, value, contrib, inv_outdeg, n, col, source);
  else if (algo == A_SSSP && K == 8) hipLaunchKernelGGL((mi_init_column_kernel<A_SSSP, 8>), grid, block, 0, s, value, contrib, inv_outdeg, n, col, source);
  else if (algo == A_SSSP && K == 16) hipLaunchKernelGGL((mi_init_column_kernel<A_SSSP, 16>), grid, block, 0, s, value, contrib, inv_outdeg, n, col, source);
  else if (algo == A_SSSP && K == 32) hipLaunchKernelGGL((mi_init_column_kernel<A_SSSP, 32>), grid, block, 0, s, value, contrib, inv_outdeg, n, col, source);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_mi_extract(int K, uint32_t *value, int32_t n, const MiExtract &x, hipStream_t s,
                             bool reset, uint32_t reset_to, const int32_t *rank) {
  if (x.count < 1 || x.count > MI_EXTRACT_MAX) return hipErrorInvalidValue;
  for (int j = 0; j < x.count; ++j)
    if (x.col[j] < 0 || x.col[j] >= K || !x.out[j]) return hipErrorInvalidValue;
  if (n <= 0) return hipSuccess;
  dim3 grid((n + 255) / 256), block(256);
  const int32_t r = reset ? 1 : 0;
  if (K == 8) hipLaunchKernelGGL(mi_extract_kernel<8>, grid, block, 0, s, value, n, x, r, reset_to, rank);
  else if (K == 16) hipLaunchKernelGGL(mi_extract_kernel<16>, grid, block, 0, s, value, n, x, r, reset_to, rank);
  else if (K == 32) hipLaunchKernelGGL(mi_extract_kernel<32>, grid, block, 0, s, value, n, x, r, reset_to, rank);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_mi_set_inst(MiInst *dst, const MiInst &val, hipStream_t s) {
  hipLaunchKernelGGL(mi_set_inst_kernel, dim3(1), dim3(64), 0, s, dst, val);
  return hipGetLastError();
}

hipError_t launch_mi_set_ctl(MiCtl *dst, const MiCtl &val, hipStream_t s) {
  hipLaunchKernelGGL(mi_set_ctl_kernel, dim3(1), dim3(64), 0, s, dst, val);
  return hipGetLastError();
}

}  // namespace sr
