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

#include <algorithm>
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

// SSSP/BFS columns whose values are stored as 16 bits ([n][K] u16, 0xFFFF =
// unreached): rows half as wide. A candidate of CAP16 or more is
// not stored (the vertex keeps its old value) and sets the column's overflow
// flag; the caller then completes that column exactly on the host.
constexpr int A_MIN16 = 100;
template <int ALGO>
constexpr bool mi_narrow() { return ALGO == A_MIN16; }
constexpr uint32_t INF16 = 0xFFFFu;
constexpr uint32_t CAP16 = 0x7FFFu;  // stored 16-bit values are below this

// Loads through pointers the compiler cannot place (they come from the
// group and unit tables): declared global, so they compile to global loads
// whose waits count vector memory only, not to flat loads.
typedef __attribute__((address_space(1))) const uint32_t g_u32;
typedef __attribute__((address_space(1))) const uint16_t g_u16;
typedef __attribute__((address_space(1))) const int32_t g_i32;
typedef __attribute__((address_space(1))) const float g_f32;
__device__ inline uint32_t ldg(const uint32_t *p) { return *(g_u32 *)p; }
__device__ inline uint32_t ldg(const uint16_t *p) { return *(g_u16 *)p; }
__device__ inline int32_t ldg(const int32_t *p) { return *(g_i32 *)p; }
__device__ inline float ldg(const float *p) { return *(g_f32 *)p; }

// Stored value of column k at row i (16 or 32 bits), and its u32-domain
// reading (INF for an unreached vertex).
template <int ALGO>
__device__ inline uint32_t mi_ld_raw(const MiGroup &g, size_t i) {
  if constexpr (mi_narrow<ALGO>()) return ldg(reinterpret_cast<const uint16_t *>(g.value) + i);
  else return ldg(g.value + i);
}
template <int ALGO>
__device__ inline uint32_t mi_cvt(uint32_t x) {
  if constexpr (mi_narrow<ALGO>()) return x == INF16 ? INF : x;
  else return x;
}
template <int ALGO>
__device__ inline uint32_t mi_ld(const MiGroup &g, size_t i) {
  return mi_cvt<ALGO>(mi_ld_raw<ALGO>(g, i));
}

// Weight of an in-edge, by the group's weight mode (fixed per work item, so
// the edge loops have no branch around a load): 0 unit weights (BFS columns
// and PageRank ignore it), 1 packed in the top byte of the edge word, 2 a
// separate u32 weight array.
template <int WM>
__device__ inline uint32_t mi_w(uint32_t q, const uint32_t *wt, int32_t e) {
  if constexpr (WM == 1) return q >> 24;
  else if constexpr (WM == 2) return ldg(wt + e);
  else return 1u;
}
template <int ALGO>
__device__ inline int mi_wmode(const MiGroup &g) {
  if constexpr (ALGO == A_SSSP || ALGO == A_MIN16) return g.has_w ? (g.packed ? 1 : 2) : 0;
  else return 0;
}

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
    return cand(raw(g, u, k), w, ln);
  }
  // the gathered value of in-neighbour u as stored (the load alone); the
  // row offset is 32-bit (plans keep every [n][K] array below 4 GiB), so
  // the load takes the group's base from scalar registers ...
  __device__ static inline uint32_t raw(const MiGroup &g, int32_t u, int k) {
    const uint32_t i = (uint32_t)u * (uint32_t)K + (uint32_t)k;
    if constexpr (mi_pr<ALGO>()) {
      return __float_as_uint(ldg(reinterpret_cast<const float *>(reinterpret_cast<const char *>(g.contrib) + 4u * i)));
    } else {
      return ldg(reinterpret_cast<const uint32_t *>(reinterpret_cast<const char *>(g.value) + 4u * i));
    }
  }
  // ... and its contribution through an edge of weight w
  __device__ static inline T cand(uint32_t xs, uint32_t w, const Lane &ln) {
    if constexpr (mi_pr<ALGO>()) {
      return __uint_as_float(xs);
    } else {
      const uint32_t x = mi_cvt<ALGO>(xs);
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
  old = mi_ld<ALGO>(g, (size_t)v * K + k);
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
      if (mi_narrow<ALGO>() && nv >= CAP16) {
        // not representable: the vertex stays unreached in this column
        atomicOr(&g.inst[k].overflow, 1u);
      } else {
        if constexpr (mi_narrow<ALGO>()) reinterpret_cast<uint16_t *>(g.value)[i] = (uint16_t)nv;
        else g.value[i] = nv;
        acc.changed++;
        acc.min_changed = min(acc.min_changed, nv);
      }
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
template <int ALGO, int K, int GE, int ROUNDS, int WM>
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
    vl[r] = cnt > 0 ? ldg(bins + (ok ? idx : 0)) : 0;  // an empty bin rereads the page's vertex 0
    beg[r] = ldg(off + vl[r]);
    end[r] = ldg(off + vl[r] + 1);
    old[r] = 0;
    att[r] = mi_attempt<ALGO, K>(g, vb + vl[r], k, ln, old[r]) && ok;
    if (!ok) vl[r] = -1;
  }
  // The rounds' edges in lockstep: each step loads EB edge words of every
  // round that still has edges (a finished or non-attempting round rereads
  // its vertex's first edge, masked), then all their value gathers, so
  // ROUNDS * EB gathers are in flight together instead of one round's.
  constexpr int EB = ROUNDS >= 8 ? 1 : (ROUNDS >= 4 ? 2 : 4);
  int32_t ec[ROUNDS];
  T x[ROUNDS];
#pragma unroll
  for (int r = 0; r < ROUNDS; ++r) {
    x[r] = R::identity();
    ec[r] = beg[r] + ein;
  }
  for (;;) {
    bool more = false;
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r) more |= att[r] && ec[r] < end[r];
    if (!more) break;
    int32_t ei[ROUNDS][EB];
    uint32_t q[ROUNDS][EB], xr[ROUNDS][EB];
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r)
#pragma unroll
      for (int j = 0; j < EB; ++j) {
        const int e = ec[r] + j * GE;
        ei[r][j] = att[r] && e < end[r] ? e : beg[r];
        q[r][j] = ldg(src + ei[r][j]);
      }
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r)
#pragma unroll
      for (int j = 0; j < EB; ++j) xr[r][j] = R::raw(g, (int32_t)(q[r][j] & g.src_mask), k);
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r) {
#pragma unroll
      for (int j = 0; j < EB; ++j)
        if (att[r] && ec[r] + j * GE < end[r])
          x[r] = R::combine(x[r], R::cand(xr[r][j], mi_w<WM>(q[r][j], wt, ei[r][j]), ln));
      ec[r] += EB * GE;
    }
  }
#pragma unroll
  for (int r = 0; r < ROUNDS; ++r) {
#pragma unroll
    for (int m = K; m < K * GE; m <<= 1) x[r] = R::combine(x[r], shfl_xor(x[r], m));
    if (att[r] && ein == 0)
      mi_epilogue<ALGO, K>(g, vb + vl[r], k, ln, old[r], x[r], (uint32_t)(end[r] - beg[r]), damping, acc);
  }
}

// edge loop of bins 6 and 7: 64/K edge lanes, 8 edges in flight per lane.
// Software-pipelined: the edge words of the next batch are loaded while the
// value rows of this batch are gathered, so a batch costs one memory round
// trip instead of two (words, then the rows they name).
template <int ALGO, int K, int WM>
__device__ inline typename MiRed<ALGO, K>::T mi_edges(const MiGroup &g, const uint32_t *src, const uint32_t *wt,
                                                      int32_t e0, int32_t e1, int k, int el, const Lane &ln) {
  using R = MiRed<ALGO, K>;
  using T = typename R::T;
  constexpr int EL = 64 / K;
  constexpr int B = 8;
  // (callers pass e0 < e1; lanes that start past the range load its first
  // edge and skip the loop, and every lane reaches the final reduction)
  T x = R::identity();
  int e = e0 + el;
  const int eb = e < e1 ? e : e0;
  int32_t ei[B];
  uint32_t q[B];
#pragma unroll
  for (int j = 0; j < B; ++j) {
    ei[j] = e + j * EL < e1 ? e + j * EL : eb;  // past the range: reread a real edge
    q[j] = ldg(src + ei[j]);
  }
  for (; e < e1; e += B * EL) {
    // the next batch's words, then this batch's gathers: both in flight
    // together, so the wait for the gathers also covers the next words
    const int en = e + B * EL;
    int32_t ein[B];
    uint32_t qn[B];
#pragma unroll
    for (int j = 0; j < B; ++j) {
      ein[j] = en + j * EL < e1 ? en + j * EL : e;  // past the range: reread this batch's first edge
      qn[j] = ldg(src + ein[j]);
    }
    uint32_t xr[B], w[B];
#pragma unroll
    for (int j = 0; j < B; ++j) {
      xr[j] = R::raw(g, (int32_t)(q[j] & g.src_mask), k);
      w[j] = mi_w<WM>(q[j], wt, ei[j]);
    }
#pragma unroll
    for (int j = 0; j < B; ++j)
      if (e + j * EL < e1) x = R::combine(x, R::cand(xr[j], w[j], ln));
#pragma unroll
    for (int j = 0; j < B; ++j) {
      ei[j] = ein[j];
      q[j] = qn[j];
    }
  }
#pragma unroll
  for (int m = K; m < 64; m <<= 1) x = R::combine(x, shfl_xor(x, m));
  return x;
}

// bin 6: one wavefront per vertex
template <int ALGO, int K, int WM>
__device__ void mi_wave(const MiGroup &g, const char *base, const PageHeader *h, int item, const Lane &ln,
                        double damping, MiAcc &acc) {
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64, k = lane % K, el = lane / K;
  int idx = item * WAVES + wave;
  if (idx >= h->bin_count[BIN_WAVE]) return;
  const int32_t *off = reinterpret_cast<const int32_t *>(base + h->off_offsets);
  const int32_t vl = ldg(reinterpret_cast<const int32_t *>(base + h->off_bins) + h->bin_start[BIN_WAVE] + idx);
  const uint32_t *src = reinterpret_cast<const uint32_t *>(base + h->off_src);
  const uint32_t *wt = reinterpret_cast<const uint32_t *>(base + h->off_w);
  const int32_t v = h->v_begin + vl;
  uint32_t old;
  bool att = mi_attempt<ALGO, K>(g, v, k, ln, old);
  if (!__any(att)) return;  // lanes of other instances still share the index loads
  const int32_t b0 = ldg(off + vl), b1 = ldg(off + vl + 1);
  auto x = mi_edges<ALGO, K, WM>(g, src, wt, b0, b1, k, el, ln);
  if (att && el == 0) mi_epilogue<ALGO, K>(g, v, k, ln, old, x, (uint32_t)(b1 - b0), damping, acc);
}

// bin 7: one wavefront per chunk; each instance column folds its partial
// into the heavy vertex's accumulator
template <int ALGO, int K, int WM>
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
  if (__any(att)) x = mi_edges<ALGO, K, WM>(g, src, wt, sb, se, k, el, ln);
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

// ---------------------------------------------------------------------------
// 16-bit SSSP/BFS columns, four per lane. A lane holds columns 4c..4c+3 of a
// row as two u16 pairs (one 8-byte load) and relaxes them with packed 16-bit
// saturating adds and mins, so the index, address and weight work of an
// in-edge is shared by four columns and a wavefront covers 64 / (K/4) edges
// per step. Values stored are below CAP16; 0xFFFF is unreached and stays so
// under the saturating add. Weights are clamped to CAP16 (a candidate through
// a heavier edge is at least CAP16 either way), so a reached value plus a
// weight never saturates and every candidate of CAP16 or more is seen as
// such: it is not stored and flags the column's overflow. Row n of every
// group is a sentinel of unreached values: an edge lane past its range
// gathers it and needs no mask.

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
__device__ inline uint32_t pk_addsat(uint32_t x, uint32_t y) {
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_add_sat(__builtin_bit_cast(u16x2, x),
                                                                     __builtin_bit_cast(u16x2, y)));
}
__device__ inline uint32_t pk_min(uint32_t x, uint32_t y) {
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_min(__builtin_bit_cast(u16x2, x),
                                                                 __builtin_bit_cast(u16x2, y)));
}
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) const u32x2 g_u32x2;
// columns 4c..4c+3 of row u (byte offset below 4 GiB)
template <int K>
__device__ inline uint2 mp_row(const MiGroup &g, uint32_t u, int c) {
  const u32x2 x = *(g_u32x2 *)(reinterpret_cast<const char *>(g.value) + (u * (uint32_t)(2 * K) + 8u * (uint32_t)c));
  return make_uint2(x.x, x.y);
}
__device__ inline uint32_t half16(uint2 x, int j) {
  const uint32_t w = j < 2 ? x.x : x.y;
  return (j & 1) ? w >> 16 : w & 0xFFFFu;
}

// Per-lane state of four instance columns.
struct Lane4 {
  uint32_t thr[4];      // a column attempts a vertex whose value exceeds thr (0xFFFF: inactive)
  uint32_t wm01, wa01;  // pair weight of columns 0, 1: w * wm + wa (unit columns: 1)
  uint32_t wm23, wa23;
};

// (ungated: every active column attempts every vertex but its source, as in
// the autotuner's timing sweeps, whose cost must not depend on the state the
// previous candidates left)
template <int K>
__device__ inline Lane4 lane4_of(const MiGroup &g, int c, bool ungated) {
  Lane4 l;
  uint32_t unit[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const MiInst &in = g.inst[4 * c + j];
    unit[j] = in.unit;
    // Table I: under strong prediction a value at or below the threshold is
    // final; otherwise every vertex is attempted (the source, at 0, cannot
    // improve and is left out)
    l.thr[j] = !in.active ? 0xFFFFu : (g.pvu == P_STRONG && !ungated ? min(in.threshold, 0xFFFEu) : 0u);
  }
  l.wm01 = (unit[0] ? 0u : 1u) | (unit[1] ? 0u : 0x10000u);
  l.wa01 = (unit[0] ? 1u : 0u) | (unit[1] ? 0x10000u : 0u);
  l.wm23 = (unit[2] ? 0u : 1u) | (unit[3] ? 0u : 0x10000u);
  l.wa23 = (unit[2] ? 1u : 0u) | (unit[3] ? 0x10000u : 0u);
  return l;
}

__device__ inline uint32_t mp_attempt(const Lane4 &ln, uint2 old) {
  uint32_t m = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) m |= (half16(old, j) > ln.thr[j] ? 1u : 0u) << j;
  return m;
}

// weight of an in-edge as the clamped value the packed add takes
template <int WM>
__device__ inline uint32_t mp_w(uint32_t q, const uint32_t *wt, int32_t e) {
  if constexpr (WM == 1) return q >> 24;
  else if constexpr (WM == 2) return min(ldg(wt + e), CAP16);
  else return 1u;
}

// relax the four columns of one gathered row through an edge of weight w
__device__ inline void mp_relax(uint2 row, uint32_t w, const Lane4 &ln, uint32_t &x01, uint32_t &x23) {
  x01 = pk_min(x01, pk_addsat(row.x, __umul24(w, ln.wm01) + ln.wa01));
  x23 = pk_min(x23, pk_addsat(row.y, __umul24(w, ln.wm23) + ln.wa23));
}

struct Acc4 {
  uint32_t changed[4] = {0, 0, 0, 0};
  uint32_t min_changed[4] = {INF, INF, INF, INF};
  uint32_t edges[4] = {0, 0, 0, 0};
};

template <int K>
__device__ inline void mp_epilogue(const MiGroup &g, int32_t v, int c, uint32_t attm, uint2 old, uint32_t x01,
                                   uint32_t x23, uint32_t deg, Acc4 &acc) {
  const uint2 red = make_uint2(x01, x23);
  uint32_t nw[4];
  bool any = false;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const uint32_t o = half16(old, j), r = half16(red, j);
    nw[j] = o;
    if (!((attm >> j) & 1u)) continue;
    acc.edges[j] += deg;
    if (r < o) {
      if (r >= CAP16) {
        atomicOr(&g.inst[4 * c + j].overflow, 1u);
      } else {
        nw[j] = r;
        acc.changed[j]++;
        acc.min_changed[j] = min(acc.min_changed[j], r);
        any = true;
      }
    }
  }
  if (any)
    *reinterpret_cast<uint2 *>(reinterpret_cast<char *>(g.value) + ((uint32_t)v * (uint32_t)(2 * K) + 8u * (uint32_t)c)) =
        make_uint2(nw[0] | (nw[1] << 16), nw[2] | (nw[3] << 16));
}

// lanes of the same column quad reduce over the edge lanes; lanes 0..K/4-1
// add the totals of their four columns to the block's LDS counters
template <int K>
__device__ inline void mp_flush(MiLds *lds, int group, Acc4 &acc) {
  constexpr int KL = K / 4;
  const int lane = threadIdx.x % 64;
#pragma unroll
  for (int m = KL; m < 64; m <<= 1)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      acc.changed[j] += shfl_xor(acc.changed[j], m);
      acc.min_changed[j] = min(acc.min_changed[j], shfl_xor(acc.min_changed[j], m));
      acc.edges[j] += shfl_xor(acc.edges[j], m);
    }
  if (lane < KL) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      MiLds &e = lds[group * K + 4 * lane + j];
      if (acc.changed[j]) atomicAdd(&e.changed, acc.changed[j]);
      if (acc.min_changed[j] != INF) atomicMin(&e.min_changed, acc.min_changed[j]);
      if (acc.edges[j]) atomicAdd(&e.edges, acc.edges[j]);
    }
  }
  acc = Acc4();
}

// bins 0..5: GE edge lanes per vertex, ROUNDS rounds of EL/GE vertices per
// wavefront, the rounds' edges in lockstep (as mi_small)
template <int K, int GE, int ROUNDS, int WM>
__device__ void mp_small(const MiGroup &g, const char *base, const PageHeader *h, int bin, int item,
                         const Lane4 &ln, Acc4 &acc) {
  constexpr int KL = K / 4, EL = 64 / KL, VPW = EL / GE;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int c = lane % KL, el = lane / KL, vs = el / GE, ein = el % GE;
  const int32_t *off = reinterpret_cast<const int32_t *>(base + h->off_offsets);
  const int32_t *bins = reinterpret_cast<const int32_t *>(base + h->off_bins) + h->bin_start[bin];
  const uint32_t *src = reinterpret_cast<const uint32_t *>(base + h->off_src);
  const uint32_t *wt = reinterpret_cast<const uint32_t *>(base + h->off_w);
  const int cnt = h->bin_count[bin];
  const int vb = h->v_begin;
  const uint32_t sentinel = (uint32_t)g.n;
  int32_t vl[ROUNDS], beg[ROUNDS], end[ROUNDS];
  uint2 old[ROUNDS];
  uint32_t attm[ROUNDS];
#pragma unroll
  for (int r = 0; r < ROUNDS; ++r) {
    const int idx = ((item * WAVES + wave) * ROUNDS + r) * VPW + vs;
    const bool ok = idx < cnt;
    vl[r] = cnt > 0 ? ldg(bins + (ok ? idx : 0)) : 0;  // an empty bin rereads the page's vertex 0
    beg[r] = ldg(off + vl[r]);
    end[r] = ldg(off + vl[r] + 1);
    old[r] = mp_row<K>(g, (uint32_t)(vb + vl[r]), c);
    attm[r] = ok ? mp_attempt(ln, old[r]) : 0u;
  }
  constexpr int EB = ROUNDS >= 8 ? 1 : (ROUNDS >= 4 ? 2 : 4);
  int32_t ec[ROUNDS];
  uint32_t x01[ROUNDS], x23[ROUNDS];
#pragma unroll
  for (int r = 0; r < ROUNDS; ++r) {
    x01[r] = 0xFFFFFFFFu;
    x23[r] = 0xFFFFFFFFu;
    ec[r] = beg[r] + ein;
  }
  for (;;) {
    bool more = false;
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r) more |= attm[r] != 0u && ec[r] < end[r];
    if (!more) break;
    int32_t ei[ROUNDS][EB];
    uint32_t q[ROUNDS][EB];
    uint2 row[ROUNDS][EB];
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r)
#pragma unroll
      for (int j = 0; j < EB; ++j) {
        const int e = ec[r] + j * GE;
        ei[r][j] = attm[r] != 0u && e < end[r] ? e : -1;
        q[r][j] = ldg(src + (ei[r][j] >= 0 ? ei[r][j] : beg[r]));
      }
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r)
#pragma unroll
      for (int j = 0; j < EB; ++j)
        row[r][j] = mp_row<K>(g, ei[r][j] >= 0 ? (q[r][j] & g.src_mask) : sentinel, c);
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r) {
#pragma unroll
      for (int j = 0; j < EB; ++j)
        mp_relax(row[r][j], mp_w<WM>(q[r][j], wt, ei[r][j] >= 0 ? ei[r][j] : beg[r]), ln, x01[r], x23[r]);
      ec[r] += EB * GE;
    }
  }
#pragma unroll
  for (int r = 0; r < ROUNDS; ++r) {
#pragma unroll
    for (int m = KL; m < KL * GE; m <<= 1) {
      x01[r] = pk_min(x01[r], shfl_xor(x01[r], m));
      x23[r] = pk_min(x23[r], shfl_xor(x23[r], m));
    }
    if (attm[r] != 0u && ein == 0)
      mp_epilogue<K>(g, vb + vl[r], c, attm[r], old[r], x01[r], x23[r], (uint32_t)(end[r] - beg[r]), acc);
  }
}

// edge loop of bins 6 and 7 (as mi_edges): EL edge lanes, 8 edges in flight
// per lane, the next batch's words loaded while this batch's rows are gathered
template <int K, int WM>
__device__ inline void mp_edges(const MiGroup &g, const uint32_t *src, const uint32_t *wt, int32_t e0, int32_t e1,
                                int c, int el, bool live, const Lane4 &ln, uint32_t &x01, uint32_t &x23) {
  constexpr int KL = K / 4, EL = 64 / KL, B = 8;
  const uint32_t sentinel = (uint32_t)g.n;
  x01 = 0xFFFFFFFFu;
  x23 = 0xFFFFFFFFu;
  int e = e0 + el;
  const int eb = e < e1 ? e : e0;
  int32_t ei[B];
  uint32_t q[B];
#pragma unroll
  for (int j = 0; j < B; ++j) {
    ei[j] = e + j * EL < e1 ? e + j * EL : eb;
    q[j] = ldg(src + ei[j]);
  }
  for (; e < e1; e += B * EL) {
    const int en = e + B * EL;
    int32_t ein[B];
    uint32_t qn[B];
#pragma unroll
    for (int j = 0; j < B; ++j) {
      ein[j] = en + j * EL < e1 ? en + j * EL : e;
      qn[j] = ldg(src + ein[j]);
    }
    uint2 row[B];
#pragma unroll
    for (int j = 0; j < B; ++j) row[j] = mp_row<K>(g, live && e + j * EL < e1 ? (q[j] & g.src_mask) : sentinel, c);
#pragma unroll
    for (int j = 0; j < B; ++j) mp_relax(row[j], mp_w<WM>(q[j], wt, ei[j]), ln, x01, x23);
#pragma unroll
    for (int j = 0; j < B; ++j) {
      ei[j] = ein[j];
      q[j] = qn[j];
    }
  }
#pragma unroll
  for (int m = KL; m < 64; m <<= 1) {
    x01 = pk_min(x01, shfl_xor(x01, m));
    x23 = pk_min(x23, shfl_xor(x23, m));
  }
}

// bin 6: one wavefront per vertex
template <int K, int WM>
__device__ void mp_wave(const MiGroup &g, const char *base, const PageHeader *h, int item, const Lane4 &ln,
                        Acc4 &acc) {
  constexpr int KL = K / 4;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64, c = lane % KL, el = lane / KL;
  const int idx = item * WAVES + wave;
  if (idx >= h->bin_count[BIN_WAVE]) return;
  const int32_t *off = reinterpret_cast<const int32_t *>(base + h->off_offsets);
  const int32_t vl = ldg(reinterpret_cast<const int32_t *>(base + h->off_bins) + h->bin_start[BIN_WAVE] + idx);
  const uint32_t *src = reinterpret_cast<const uint32_t *>(base + h->off_src);
  const uint32_t *wt = reinterpret_cast<const uint32_t *>(base + h->off_w);
  const int32_t v = h->v_begin + vl;
  const uint2 old = mp_row<K>(g, (uint32_t)v, c);
  const uint32_t attm = mp_attempt(ln, old);
  if (!__any(attm != 0u)) return;
  const int32_t b0 = ldg(off + vl), b1 = ldg(off + vl + 1);
  uint32_t x01, x23;
  mp_edges<K, WM>(g, src, wt, b0, b1, c, el, attm != 0u, ln, x01, x23);
  if (attm != 0u && el == 0) mp_epilogue<K>(g, v, c, attm, old, x01, x23, (uint32_t)(b1 - b0), acc);
}

// bin 7: one wavefront per sub-chunk; each column folds its partial into the
// heavy vertex's accumulator (the heavy-vertex kernel runs the epilogue)
template <int K, int WM>
__device__ void mp_chunk(const MiGroup &g, const MiUnit &u, const char *base, const PageHeader *h, int item,
                         const Lane4 &ln) {
  constexpr int KL = K / 4;
  constexpr int S = mi_subchunks(KL);
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64, c = lane % KL, el = lane / KL;
  const int sidx = item * WAVES + wave;
  const int idx = sidx / S, sub = sidx % S;
  if (idx >= h->bin_count[BIN_CHUNK]) return;
  const Chunk ch = reinterpret_cast<const Chunk *>(base + h->off_chunks)[idx];
  const int32_t len = (ch.e_end - ch.e_begin + S - 1) / S;
  const int32_t sb = ch.e_begin + sub * len, se = min(ch.e_end, sb + len);
  if (sb >= se) return;
  const uint32_t *src = reinterpret_cast<const uint32_t *>(base + h->off_src);
  const uint32_t *wt = reinterpret_cast<const uint32_t *>(base + h->off_w);
  const int32_t v = h->v_begin + ch.vl;
  const uint2 old = mp_row<K>(g, (uint32_t)v, c);
  const uint32_t attm = mp_attempt(ln, old);
  if (!__any(attm != 0u)) return;
  uint32_t x01, x23;
  mp_edges<K, WM>(g, src, wt, sb, se, c, el, attm != 0u, ln, x01, x23);
  if (el == 0 && attm != 0u) {
    const uint2 red = make_uint2(x01, x23);
    unsigned long long *slot = &u.acc[(size_t)((uint32_t)ch.first_count & 0xFFFFFu) * K + 4 * c];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t r = half16(red, j);
      if (((attm >> j) & 1u) && r != INF16) atomicMin(reinterpret_cast<uint32_t *>(slot + j), r);
    }
  }
}

// WMK: the weight mode of every group of the plan (0, 1, 2), or 3 when the
// groups differ (then chosen per work item; that kernel needs the registers
// of the widest mode)
template <int ALGO, int K, int ROUNDS, int WMK>
__global__ void __launch_bounds__(BLOCK) mi_sweep_kernel(MiArgs a) {
  if (a.ctl->remaining == 0 && !a.tuning) return;  // everything converged: replays are no-ops
  extern __shared__ MiLds lds[];
  __shared__ int32_t s_base;
  const int ninst = a.ngroups * K;
  lds_clear(lds, ninst, BLOCK);
  const int lane = threadIdx.x % 64, k = lane % K;
  // the lanes' instance state (gate thresholds, weights, PageRank terms),
  // taken once per block into LDS after the counters when the launch has
  // the room (lane_lds): items read it there instead of from the records
  Lane *lanes = reinterpret_cast<Lane *>(lds + ninst);
  Lane4 *lanes4 = reinterpret_cast<Lane4 *>(lds + ninst);
  if (a.lane_lds) {
    if constexpr (mi_narrow<ALGO>()) {
      for (int i = threadIdx.x; i < a.ngroups * (K / 4); i += BLOCK)
        lanes4[i] = lane4_of<K>(a.groups[i / (K / 4)], i % (K / 4), a.tuning != 0);
    } else {
      for (int i = threadIdx.x; i < ninst; i += BLOCK) lanes[i] = lane_of(a.groups[i / K].inst[i % K]);
    }
  }
  // consecutive items of a block mostly lie in one unit: its item range
  // carries over from item to item (the search runs only when an item leaves it)
  int32_t cu = 0, cu_lo = 0, cu_hi = -1;  // the last unit and its items [cu_lo, cu_hi)
  // per-instance counters of the items so far, added to LDS when the group
  // changes or the block ends
  int acc_group = -1;
  MiAcc acc;
  Acc4 acc4;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) s_base = (int32_t)atomicAdd(&a.ctl->queue, (uint32_t)a.grab);
    __syncthreads();
    const int32_t base = s_base;
    if (base >= a.total_items) break;
    const int32_t end = min(base + a.grab, a.total_items);
    for (int32_t qi = base; qi < end; ++qi) {
      const int32_t it = a.descending ? a.total_items - 1 - qi : qi;
      if (it < cu_lo || it >= cu_hi) {
        int lo = 0, hi = a.nunits;  // unit_prefix[lo] <= it < unit_prefix[hi]
        while (hi - lo > 1) {
          int mid = (lo + hi) >> 1;
          if (a.unit_prefix[mid] <= it) lo = mid; else hi = mid;
        }
        cu = lo;
        cu_lo = a.unit_prefix[lo];
        cu_hi = a.unit_prefix[lo + 1];
      }
      const MiUnit &u = a.units[cu];
      if (a.group_active[u.group] == 0) continue;  // no live instance in this group
      const MiGroup &g = a.groups[u.group];
      if (u.group != acc_group) {
        if (acc_group >= 0) {
          if constexpr (mi_narrow<ALGO>()) mp_flush<K>(lds, acc_group, acc4);
          else mi_flush<ALGO, K>(lds, acc_group, acc);
        }
        acc_group = u.group;
      }
      const int local = it - cu_lo;
      // the item's bin: the unit's bin starts loaded together, then counted
      // (they grow with the bin), with no chain of dependent loads
      int32_t pf[NBINS];
#pragma unroll
      for (int b = 0; b < NBINS; ++b) pf[b] = u.blk_prefix[b];
      int bin = 0;
      int32_t first = 0;
#pragma unroll
      for (int b = 1; b < NBINS; ++b)
        if (pf[b] <= local) { bin = b; first = pf[b]; }
      const int item = local - first;
      const char *bp = u.page;
      const PageHeader *h = reinterpret_cast<const PageHeader *>(bp);
      // the weight mode: the plan's, or the group's when the plan mixes them
      const int wm = WMK < 3 ? WMK : mi_wmode<ALGO>(g);
#define MI_WM(CALL)                                                                 \
  do {                                                                              \
    if constexpr (WMK < 3) { constexpr int WM = mi_pr<ALGO>() ? 0 : WMK; CALL; }    \
    else if (wm == 1) { constexpr int WM = mi_pr<ALGO>() ? 0 : 1; CALL; }           \
    else if (wm == 2) { constexpr int WM = mi_pr<ALGO>() ? 0 : 2; CALL; }           \
    else { constexpr int WM = 0; CALL; }                                            \
  } while (0)
      if constexpr (mi_narrow<ALGO>()) {
        constexpr int EL4 = 256 / K;  // edge lanes with four columns per lane
        const Lane4 ln4 = a.lane_lds ? lanes4[u.group * (K / 4) + lane % (K / 4)]
                                     : lane4_of<K>(g, lane % (K / 4), a.tuning != 0);
        switch (bin) {
          case 0: MI_WM((mp_small<K, 1, ROUNDS, WM>(g, bp, h, 0, item, ln4, acc4))); break;
          case 1: MI_WM((mp_small<K, (2 < EL4 ? 2 : EL4), ROUNDS, WM>(g, bp, h, 1, item, ln4, acc4))); break;
          case 2: MI_WM((mp_small<K, (4 < EL4 ? 4 : EL4), ROUNDS, WM>(g, bp, h, 2, item, ln4, acc4))); break;
          case 3: MI_WM((mp_small<K, (8 < EL4 ? 8 : EL4), ROUNDS, WM>(g, bp, h, 3, item, ln4, acc4))); break;
          case 4: MI_WM((mp_small<K, (16 < EL4 ? 16 : EL4), ROUNDS, WM>(g, bp, h, 4, item, ln4, acc4))); break;
          case 5: MI_WM((mp_small<K, (32 < EL4 ? 32 : EL4), ROUNDS, WM>(g, bp, h, 5, item, ln4, acc4))); break;
          case BIN_WAVE: MI_WM((mp_wave<K, WM>(g, bp, h, item, ln4, acc4))); break;
          case BIN_CHUNK: MI_WM((mp_chunk<K, WM>(g, u, bp, h, item, ln4))); break;
          default: break;  // no zero in-degree bin outside PageRank
        }
      } else {
        const Lane ln = a.lane_lds ? lanes[u.group * K + k] : lane_of(g.inst[k]);
        switch (bin) {
          case 0: MI_WM((mi_small<ALGO, K, 1, ROUNDS, WM>(g, bp, h, 0, item, ln, a.damping, acc))); break;
          case 1: MI_WM((mi_small<ALGO, K, (2 < 64 / K ? 2 : 64 / K), ROUNDS, WM>(g, bp, h, 1, item, ln, a.damping, acc))); break;
          case 2: MI_WM((mi_small<ALGO, K, (4 < 64 / K ? 4 : 64 / K), ROUNDS, WM>(g, bp, h, 2, item, ln, a.damping, acc))); break;
          case 3: MI_WM((mi_small<ALGO, K, (8 < 64 / K ? 8 : 64 / K), ROUNDS, WM>(g, bp, h, 3, item, ln, a.damping, acc))); break;
          case 4: MI_WM((mi_small<ALGO, K, (16 < 64 / K ? 16 : 64 / K), ROUNDS, WM>(g, bp, h, 4, item, ln, a.damping, acc))); break;
          case 5: MI_WM((mi_small<ALGO, K, (32 < 64 / K ? 32 : 64 / K), ROUNDS, WM>(g, bp, h, 5, item, ln, a.damping, acc))); break;
          case BIN_WAVE: MI_WM((mi_wave<ALGO, K, WM>(g, bp, h, item, ln, a.damping, acc))); break;
          case BIN_CHUNK: MI_WM((mi_chunk<ALGO, K, WM>(g, u, bp, h, item, ln))); break;
          default:
            if constexpr (mi_pr<ALGO>()) mi_zero<ALGO, K, ROUNDS>(g, bp, h, item, ln, a.damping, acc);
            break;
        }
      }
#undef MI_WM
    }
  }
  if (acc_group >= 0) {
    if constexpr (mi_narrow<ALGO>()) mp_flush<K>(lds, acc_group, acc4);
    else mi_flush<ALGO, K>(lds, acc_group, acc);
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

// Heavy vertices after a sweep: each thread serves one instance column of
// a run of MI_HEAVY_RUN consecutive heavy vertices: it takes each vertex's
// accumulator with an exchange (leaving the identity) and runs the
// epilogue. The counters go to the block's LDS copy and then once per block
// and instance to the instance record, so the instance records do not take
// one device atomic per heavy vertex.
template <int ALGO, int K>
__global__ void __launch_bounds__(BLOCK) mi_heavy_kernel(MiArgs a) {
  using R = MiRed<ALGO, K>;
  using T = typename R::T;
  if (a.ctl->remaining == 0 && !a.tuning) return;
  extern __shared__ MiLds hlds[];
  const int ninst = a.ngroups * K;
  lds_clear(hlds, ninst, BLOCK);
  __syncthreads();
  const int64_t p = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  const int32_t k = (int32_t)(p % K);
  const int32_t h0 = (int32_t)(p / K) * MI_HEAVY_RUN;
  const int32_t h1 = min(h0 + MI_HEAVY_RUN, a.total_heavy);
  int lo = 0;
  for (int32_t hh = h0; hh < h1; ++hh) {
    // units[lo].heavy_base <= hh < units[lo + 1].heavy_base (runs move forward)
    if (hh == h0) {
      int hi = a.nunits;
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (a.units[mid].heavy_base <= hh) lo = mid; else hi = mid;
      }
    } else {
      while (lo + 1 < a.nunits && a.units[lo + 1].heavy_base <= hh) ++lo;
    }
    const MiUnit &u = a.units[lo];
    if (a.group_active[u.group] == 0) continue;  // the sweep skipped the group: accumulators untouched
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
    if (!mi_attempt<ALGO, K>(g, v, k, ln, old)) continue;
    MiAcc acc;
    mi_epilogue<ALGO, K>(g, v, k, ln, old, t, (uint32_t)(off[x.vl + 1] - off[x.vl]), a.damping, acc);
    lds_add<ALGO>(hlds[u.group * K + k], acc);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < ninst; i += BLOCK) {
    const MiLds &e = hlds[i];
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
  } else if constexpr (mi_narrow<ALGO>()) {
    reinterpret_cast<uint16_t *>(value)[i] = v == source ? (uint16_t)0 : (uint16_t)INF16;
  } else {
    value[i] = v == source ? 0u : INF;
  }
}

// One entry of a 16-bit column (the source of an admitted query).
__global__ void mi_set_u16_kernel(uint32_t *value, size_t index, uint32_t v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) reinterpret_cast<uint16_t *>(value)[index] = (uint16_t)v;
}

__global__ void mi_set_inst_kernel(MiInst *dst, MiInst val) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dst = val;
}

__global__ void mi_set_ctl_kernel(MiCtl *dst, MiCtl val) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dst = val;
}

// Several columns in one pass: the columns of a vertex share its row of
// 4K bytes, so the row is fetched from memory once for all of them.
// NARROW: 16-bit columns, widened to u32 (0xFFFF -> INF) on the way out.
template <int K, bool NARROW>
__global__ void mi_extract_kernel(uint32_t *value, int32_t n, MiExtract x, int32_t reset, uint32_t reset_to,
                                  const int32_t *rank) {
  int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const size_t r = (size_t)(rank ? rank[v] : v) * K;
  for (int j = 0; j < x.count; ++j) {
    if constexpr (NARROW) {
      uint16_t *row = reinterpret_cast<uint16_t *>(value) + r;
      const uint32_t y = row[x.col[j]];
      x.out[j][v] = y == INF16 ? INF : y;
      if (reset) row[x.col[j]] = (uint16_t)(reset_to >= INF16 ? INF16 : reset_to);
    } else {
      uint32_t *row = value + r;
      x.out[j][v] = row[x.col[j]];
      if (reset) row[x.col[j]] = reset_to;
    }
  }
}

template <int ALGO, int K, int ROUNDS>
void mi_sweep_wm(const MiArgs &a, hipStream_t s, size_t lds) {
  if constexpr (mi_pr<ALGO>()) {
    hipLaunchKernelGGL((mi_sweep_kernel<ALGO, K, ROUNDS, 0>), dim3(a.nblocks), dim3(BLOCK), lds, s, a);
  } else {
    if (a.wmode == 0) hipLaunchKernelGGL((mi_sweep_kernel<ALGO, K, ROUNDS, 0>), dim3(a.nblocks), dim3(BLOCK), lds, s, a);
    else if (a.wmode == 1) hipLaunchKernelGGL((mi_sweep_kernel<ALGO, K, ROUNDS, 1>), dim3(a.nblocks), dim3(BLOCK), lds, s, a);
    else if (a.wmode == 2) hipLaunchKernelGGL((mi_sweep_kernel<ALGO, K, ROUNDS, 2>), dim3(a.nblocks), dim3(BLOCK), lds, s, a);
    else hipLaunchKernelGGL((mi_sweep_kernel<ALGO, K, ROUNDS, 3>), dim3(a.nblocks), dim3(BLOCK), lds, s, a);
  }
}

template <int ALGO, int K>
void mi_pair(const MiArgs &a, hipStream_t s) {
  // LDS: per-instance counters (the heavy kernel too), then the sweep's lane
  // states when both fit 64 KiB
  const size_t lds = sizeof(MiLds) * (size_t)a.ngroups * K;
  const size_t lanes = mi_narrow<ALGO>() ? sizeof(Lane4) * (size_t)a.ngroups * (K / 4) : sizeof(Lane) * (size_t)a.ngroups * K;
  MiArgs b = a;
  b.lane_lds = lds + lanes <= 65536 ? 1 : 0;
  const size_t sweep_lds = b.lane_lds ? lds + lanes : lds;
  if (a.rounds == 2) mi_sweep_wm<ALGO, K, 2>(b, s, sweep_lds);
  else if (a.rounds == 8) mi_sweep_wm<ALGO, K, 8>(b, s, sweep_lds);
  else mi_sweep_wm<ALGO, K, 4>(b, s, sweep_lds);
  hipLaunchKernelGGL((mi_heavy_kernel<ALGO, K>), dim3(a.heavy_blocks), dim3(BLOCK), lds, s, a);
  hipLaunchKernelGGL((mi_close_kernel<ALGO, K>), dim3(1), dim3(MI_CLOSE_THREADS), 0, s, a);
}

}  // namespace

int mi_items_per_block_host(int b, int K, int rounds) { return mi_items_per_block(b, K, rounds); }

hipError_t launch_mi_sweep(int algo, int K, const MiArgs &a, hipStream_t s) {
  if (a.nblocks <= 0) return hipErrorInvalidValue;
  if (a.ngroups * K > MI_MAX_INSTANCES) return hipErrorInvalidValue;
  if (a.rounds != 2 && a.rounds != 4 && a.rounds != 8) return hipErrorInvalidValue;
  if (a.wmode < 0 || a.wmode > 3) return hipErrorInvalidValue;
  if (algo == A_PPR && K == 8) mi_pair<A_PPR, 8>(a, s);
  else if (algo == A_PPR && K == 16) mi_pair<A_PPR, 16>(a, s);
  else if (algo == A_SSSP && a.narrow && K == 8) mi_pair<A_MIN16, 8>(a, s);
  else if (algo == A_SSSP && a.narrow && K == 16) mi_pair<A_MIN16, 16>(a, s);
  else if (algo == A_SSSP && a.narrow && K == 32) mi_pair<A_MIN16, 32>(a, s);
  else if (algo == A_SSSP && a.narrow && K == 64) mi_pair<A_MIN16, 64>(a, s);
  else if (algo == A_SSSP && K == 8) mi_pair<A_SSSP, 8>(a, s);
  else if (algo == A_SSSP && K == 16) mi_pair<A_SSSP, 16>(a, s);
  else if (algo == A_SSSP && K == 32) mi_pair<A_SSSP, 32>(a, s);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_mi_init_column(int algo, int K, uint32_t *value, float *contrib, const float *inv_outdeg,
                                 int32_t n, int32_t col, int32_t source, hipStream_t s, bool narrow) {
  dim3 grid((n + 255) / 256), block(256);
  if (narrow) {
    if (algo != A_SSSP) return hipErrorInvalidValue;
    if (K == 8) hipLaunchKernelGGL((mi_init_column_kernel<A_MIN16, 8>), grid, block, 0, s, value, contrib, inv_outdeg, n, col, source);
    else if (K == 16) hipLaunchKernelGGL((mi_init_column_kernel<A_MIN16, 16>), grid, block, 0, s, value, contrib, inv_outdeg, n, col, source);
    else if (K == 32) hipLaunchKernelGGL((mi_init_column_kernel<A_MIN16, 32>), grid, block, 0, s, value, contrib, inv_outdeg, n, col, source);
    else if (K == 64) hipLaunchKernelGGL((mi_init_column_kernel<A_MIN16, 64>), grid, block, 0, s, value, contrib, inv_outdeg, n, col, source);
    else return hipErrorInvalidValue;
    return hipGetLastError();
  }
  if (algo == A_PPR && K == 8) hipLaunchKernelGGL((mi_init_column_kernel<A_PPR, 8>), grid, block, 0, s, value, contrib, inv_outdeg, n, col, source);
  else if (algo == A_PPR && K == 16) hipLaunchKernelGGL((mi_init_column_kernel<A_PPR, 16>), grid, block, 0, s, value, contrib, inv_outdeg, n, col, source);
  else if (algo == A_SSSP && K == 8) hipLaunchKernelGGL((mi_init_column_kernel<A_SSSP, 8>), grid, block, 0, s, value, contrib, inv_outdeg, n, col, source);
  else if (algo == A_SSSP && K == 16) hipLaunchKernelGGL((mi_init_column_kernel<A_SSSP, 16>), grid, block, 0, s, value, contrib, inv_outdeg, n, col, source);
  else if (algo == A_SSSP && K == 32) hipLaunchKernelGGL((mi_init_column_kernel<A_SSSP, 32>), grid, block, 0, s, value, contrib, inv_outdeg, n, col, source);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_mi_extract(int K, uint32_t *value, int32_t n, const MiExtract &x, hipStream_t s,
                             bool reset, uint32_t reset_to, const int32_t *rank, bool narrow) {
  if (x.count < 1 || x.count > MI_EXTRACT_MAX) return hipErrorInvalidValue;
  for (int j = 0; j < x.count; ++j)
    if (x.col[j] < 0 || x.col[j] >= K || !x.out[j]) return hipErrorInvalidValue;
  if (n <= 0) return hipSuccess;
  dim3 grid((n + 255) / 256), block(256);
  const int32_t r = reset ? 1 : 0;
  if (narrow) {
    if (K == 8) hipLaunchKernelGGL((mi_extract_kernel<8, true>), grid, block, 0, s, value, n, x, r, reset_to, rank);
    else if (K == 16) hipLaunchKernelGGL((mi_extract_kernel<16, true>), grid, block, 0, s, value, n, x, r, reset_to, rank);
    else if (K == 32) hipLaunchKernelGGL((mi_extract_kernel<32, true>), grid, block, 0, s, value, n, x, r, reset_to, rank);
    else if (K == 64) hipLaunchKernelGGL((mi_extract_kernel<64, true>), grid, block, 0, s, value, n, x, r, reset_to, rank);
    else return hipErrorInvalidValue;
    return hipGetLastError();
  }
  if (K == 8) hipLaunchKernelGGL((mi_extract_kernel<8, false>), grid, block, 0, s, value, n, x, r, reset_to, rank);
  else if (K == 16) hipLaunchKernelGGL((mi_extract_kernel<16, false>), grid, block, 0, s, value, n, x, r, reset_to, rank);
  else if (K == 32) hipLaunchKernelGGL((mi_extract_kernel<32, false>), grid, block, 0, s, value, n, x, r, reset_to, rank);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_mi_set_u16(uint32_t *value, size_t index, uint32_t v, hipStream_t s) {
  hipLaunchKernelGGL(mi_set_u16_kernel, dim3(1), dim3(64), 0, s, value, index, v);
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

namespace {
__global__ void __launch_bounds__(256) mi_setup_kernel(const MiGroup *groups, const uint32_t *buf, int32_t ngroups,
                                                       int32_t nadmit, uint32_t remaining, MiCtl *ctl,
                                                       uint32_t *group_active, int32_t K, int32_t narrow) {
  const int32_t i = (int32_t)(blockIdx.x * 256 + threadIdx.x);
  if (i == 0) {
    ctl->queue = 0;
    ctl->pad = 0;
    ctl->remaining = remaining;
    ctl->sweeps = 0;
  }
  if (i < ngroups) group_active[i] = buf[i];
  if (i >= nadmit) return;
  const MiAdmit ad = reinterpret_cast<const MiAdmit *>(buf + ngroups)[i];
  const MiGroup &g = groups[ad.group];
  const size_t idx = (size_t)ad.source * (size_t)K + (size_t)ad.col;
  if (narrow) reinterpret_cast<uint16_t *>(g.value)[idx] = 0;
  else g.value[idx] = 0u;
  // the record a fresh column starts from (as the host's column set-up)
  MiInst in;
  in.active = 1;
  in.unit = ad.unit;
  in.source = ad.source;
  in.threshold = 0;  // value 0 (the source) is final from the start
  in.sweeps = 0;
  in.done = 0;
  in.stop_reason = 0;
  in.no_improve = 0;
  in.sw_changed = 0;
  in.sw_min_changed = INF;
  in.sw_edges = 0;
  in.sw_l1 = 0.0;
  in.sw_ddelta = 0.0;
  in.sw_dmass = 0.0;
  in.dangling = 0.0;
  in.mass = 0.0;
  in.best_l1 = 1e300;
  in.last_l1 = -1.0;
  in.edges_total = 0;
  in.overflow = 0;
  in.pad = 0;
  g.inst[ad.col] = in;
}
}  // namespace

hipError_t launch_mi_setup(const MiGroup *groups, const uint32_t *buf, int32_t ngroups, int32_t nadmit,
                           uint32_t remaining, MiCtl *ctl, uint32_t *group_active, int32_t K, bool narrow,
                           hipStream_t s) {
  const int32_t n = std::max(1, std::max(ngroups, nadmit));
  hipLaunchKernelGGL(mi_setup_kernel, dim3((n + 255) / 256), dim3(256), 0, s, groups, buf, ngroups, nadmit, remaining,
                     ctl, group_active, K, narrow ? 1 : 0);
  return hipGetLastError();
}

}  // namespace sr
