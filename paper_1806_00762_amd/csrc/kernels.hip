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

#include <mutex>
#include <type_traits>
#include <vector>

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
  const int32_t *tiles;
  const Chunk *chunks;
  const uint32_t *src;       // edge words: source id, or source | weight << 24 when packed
  const uint32_t *w;         // separate u32 weights (unpacked weighted pages)
  const uint32_t *vpk;       // split images: per-vertex tile-relative ends, or heavy index
  const int2 *tbase;         // split images: per-tile bases
  const int4 *hside;         // split images: heavy-vertex table
  const uint16_t *hsrc;      // split images: narrow source ids
  const uint8_t *hw;         // split images: narrow weights
  int32_t bin_count, bin_start;
  unsigned long long *partial;  // heavy-vertex accumulators, at each vertex's first chunk
};

// Wide in-edge e of a split image: its edge word, or (W3: the image of an
// unweighted graph stores 3-byte ids back to back, 8 bytes of padding
// after the last) the id, taken from the two aligned words around it.
template <bool W3>
__device__ inline uint32_t wide_word(const PageCtx &p, int32_t e) {
  if constexpr (W3) {
    const uint32_t b = 3u * (uint32_t)e;
    const uint32_t *w = reinterpret_cast<const uint32_t *>(reinterpret_cast<const char *>(p.src) + (b & ~3u));
    return __builtin_amdgcn_alignbyte(w[1], w[0], b & 3u) & 0xFFFFFFu;
  } else {
    return p.src[e];
  }
}

// Thread-local sweep counters, reduced per block at the end.
struct Acc {
  uint32_t changed = 0, attempted = 0, skipped = 0, mispred = 0, edges = 0;
  uint32_t narrow = 0;  // scanned edges read from the narrow section of a split image
  uint32_t min_changed = INF;
  double l1 = 0.0, ddelta = 0.0, dmass = 0.0;
};

// Per-block view of the run state.
struct Run {
  int algo, pvu, phase, audit;
  int early;  // BFS early break (strong prediction, normal phase)
  uint32_t threshold;
  uint32_t *value;
  float *contrib;    // gathered terms (a snapshot under deterministic sweeps)
  float *contrib_w;  // where a pull writes its vertex's new term (contrib, or the snapshot's next buffer)
  const float *inv_outdeg;
  uint8_t *status;
  const Diagram *dia;
  double damping, dangling, inv_mass;
  float pr_eps, base_uniform;
  int32_t pr_seed;
  int delta;       // PageRank-delta phase: residual propagation (dangling = mass sent last pass)
  float *resid;
  uint32_t *hist;  // LDS histogram of predictor states
  // frontier of the pass (vertices that changed), for the host sparse stage
  int32_t collect;
  uint32_t *frontier, *fr_count;
  uint32_t fr_cap;
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

// Source and weight of page-local in-edge e from its edge word.
// PACKED: the word is source | weight << 24; else the source id, with the
// weight (SSSP) in the separate u32 section.
template <bool PACKED>
__device__ inline int32_t src_of(uint32_t word) { return (int32_t)(PACKED ? word & PACKED_SRC_MASK : word); }
template <bool PACKED>
__device__ inline uint32_t weight_of(const PageCtx &p, uint32_t word, int32_t e) {
  if constexpr (PACKED) return word >> 24;
  else return p.w[e];
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

// Pull result handed to the epilogue: the u32 minimum, or the PageRank sum
// in double (exact for a float sum, and for the fixed-point sums of
// deterministic sweeps and heavy-vertex chunks).
template <int ALGO>
using RedArg = typename std::conditional<is_pr<ALGO>(), double, uint32_t>::type;

// Epilogue of one vertex: compare, write, advance the predictor state,
// count. `computed` says whether red holds the pull result.
template <int ALGO>
__device__ inline bool epilogue(const Run &r, int32_t v, const Gate &g, bool computed,
                                RedArg<ALGO> red, uint32_t deg, Acc &acc) {
  bool changed = false;
  if constexpr (is_pr<ALGO>()) {
    if (r.delta) {
      // PageRank-delta (Section 4.3's data-driven PageRank), as residual
      // propagation: the gathered sum holds d r_u / outdeg(u) of every
      // in-neighbour that sent in the last pass, and the dangling vertices'
      // sent mass reaches every vertex through the teleport vector. A vertex
      // whose residual exceeds pr_eps applies it to its rank and sends it
      // (success in Fig. 6); otherwise it keeps it. A vertex that does not
      // pull (weak prediction) drops this pass's in-delta: the rank-form
      // verification passes that end the run recover it.
      const uint32_t att = g.attempt ? 1u : 0u;
      if (computed && g.attempt) {
        const double t = r.pr_seed < 0 ? (double)r.base_uniform : (v == r.pr_seed ? 1.0 : 0.0);
        const float rv = (float)((double)r.resid[v] + red + r.damping * r.dangling * t);
        const float iod = r.inv_outdeg[v];
        if (fabsf(rv) > r.pr_eps) {
          changed = true;
          r.value[v] = __float_as_uint(__uint_as_float(g.old) + rv);
          r.contrib_w[v] = (float)(r.damping * (double)rv * (double)iod);
          r.resid[v] = 0.0f;
          acc.l1 += fabs((double)rv);
          acc.dmass += (double)rv;
          if (iod == 0.0f) acc.ddelta += (double)rv;
        } else {
          r.resid[v] = rv;
          r.contrib_w[v] = 0.0f;
        }
      } else {
        r.contrib_w[v] = 0.0f;
      }
      acc.attempted += att;
      acc.skipped += 1u - att;
      acc.edges += att * deg;
      acc.changed += changed ? 1u : 0u;
      if (r.pvu == P_WEAK) {
        uint8_t nx = (g.attempt && changed) ? r.dia->succ[g.st] : r.dia->fail[g.st];
        if (nx != g.st) r.status[v] = nx;
        atomicAdd(&r.hist[g.st], 1u);
      }
      return changed;
    }
  }
  if (computed) {
    if constexpr (is_pr<ALGO>()) {
      // x = (1 - d) t + d (P^T x + D t) applied to x / mass: in-place
      // sweeps do not keep the rank sum at 1, and the drift would otherwise
      // decay only at rate d; the fixed point (mass 1) is the same
      const double t = r.pr_seed < 0 ? (double)r.base_uniform : (v == r.pr_seed ? 1.0 : 0.0);
      float oldf = __uint_as_float(g.old);
      float nv = (float)((1.0 - r.damping) * t + r.damping * r.inv_mass * (red + r.dangling * t));
      float diff = nv - oldf;
      bool would = fabsf(diff) > r.pr_eps;
      if (g.attempt) {
        changed = would;
        r.value[v] = __float_as_uint(nv);
        float iod = r.inv_outdeg[v];
        r.contrib_w[v] = nv * iod;
        acc.l1 += fabs((double)nv - (double)oldf);
        acc.dmass += (double)nv - (double)oldf;
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
  const uint32_t att = g.attempt ? 1u : 0u;
  acc.attempted += att;
  acc.skipped += 1u - att;
  acc.edges += att * deg;
  acc.changed += changed ? 1u : 0u;
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
  return changed;
}

// Append the changed vertices of the active lanes to the pass frontier:
// one counter atomic per wavefront; entries past the capacity are counted
// but dropped (the host then knows the frontier is incomplete). Call from
// converged control flow of the wavefront.
__device__ inline void frontier_push(const Run &r, bool changed, int32_t v) {
  if (!r.collect) return;
  const unsigned long long m = __ballot(changed);
  if (m == 0ull) return;
  const int lane = threadIdx.x % 64;
  const int leader = __ffsll((long long)m) - 1;
  uint32_t base = 0;
  if (lane == leader) base = atomicAdd(r.fr_count, (uint32_t)__popcll(m));
  base = __shfl(base, leader, 64);
  if (changed) {
    const uint32_t i = base + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
    if (i < r.fr_cap) r.frontier[i] = (uint32_t)v;
  }
}

// ------------------------------------------------------------------ tiles
// One block per tile of consecutive vertices (<= TILE_V vertices, <= TILE_E
// in-edges). Phase 1 gates the vertices (two consecutive ones per thread)
// and compacts the attempting ones with a block-wide scan into LDS. Phase 2
// gives every thread TILE_E/256 positions of the compacted edge list in
// short groups of consecutive ones, so each load instruction of a wavefront
// reads one contiguous range and a thread keeps all its gathers in flight;
// runs of edges of the same vertex are reduced in registers before one LDS
// atomic. Phase 3 runs the epilogues.

template <bool SPLIT_, bool DET_ = false, bool W3_ = false>
struct TileLds {
  static constexpr bool SPLIT = SPLIT_;
  static constexpr bool DET = DET_;
  static constexpr bool W3 = W3_;  // split image of an unweighted graph: wide ids of 3 bytes
  int32_t pos[TILE_V + 1];  // first compacted (wide) edge position of each attempting vertex
  int32_t eb[TILE_V];       // its first (wide) in-edge (page-local) minus that position
  // split images: the same for the narrow list (one unused entry otherwise)
  int32_t pos_n[SPLIT ? TILE_V + 1 : 1];
  int32_t eb_n[SPLIT ? TILE_V : 1];
  int32_t vl[TILE_V];       // its page-local vertex id
  uint32_t acc[TILE_V];     // reduction (u32 min, or f32 sum bits)
  // deterministic PageRank sweeps: the sum in 2^-54 fixed point (exact, order-free)
  unsigned long long acc64[DET_ ? TILE_V : 1];
  uint32_t old[TILE_V];
  uint8_t att[TILE_V];
  uint8_t st[TILE_V];
  int32_t wsum[WAVES][3];
  uint32_t wmax[WAVES];
  // position -> covering vertex: k for the narrow list, TILE_V + k for the
  // wide one (split images put the narrow positions first)
  __attribute__((aligned(16))) uint16_t map[TILE_E];
};

// Builds s.map over the tile's An + At compacted positions: the start of
// every non-empty edge range is marked with its (list, vertex) code, and an
// inclusive max-scan carries each mark over its range (codes grow with the
// position, since the wide codes lie above the narrow ones). Called by every
// thread of the block.
template <typename L>
__device__ inline void tile_map(L &s, int An, int At, int Kt) {
  constexpr bool SPLIT = L::SPLIT;
  constexpr int PER = TILE_E / BLOCK;  // consecutive entries per thread in the scan
  static_assert(PER == 16, "two 16-byte LDS words per thread");
  const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
  const int Ac = An + At;
  uint4 *m4 = reinterpret_cast<uint4 *>(s.map);
  if (tid * PER < Ac) { m4[2 * tid] = make_uint4(0, 0, 0, 0); m4[2 * tid + 1] = make_uint4(0, 0, 0, 0); }
  __syncthreads();
  for (int k = tid; k < Kt; k += BLOCK) {
    if constexpr (SPLIT) {
      if (s.pos_n[k] < s.pos_n[k + 1]) s.map[s.pos_n[k]] = (uint16_t)k;
    }
    if (s.pos[k] < s.pos[k + 1]) s.map[An + s.pos[k]] = (uint16_t)(TILE_V + k);
  }
  __syncthreads();
  uint32_t v[PER];
  uint32_t run = 0;
  if (tid * PER < Ac) {
    const uint4 a = m4[2 * tid], b = m4[2 * tid + 1];
    const uint32_t w[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      run = max(run, w[i] & 0xFFFFu); v[2 * i] = run;
      run = max(run, w[i] >> 16);     v[2 * i + 1] = run;
    }
  }
  uint32_t inc = run;
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) {
    const uint32_t o = __shfl_up(inc, m, 64);
    if (lane >= m) inc = max(inc, o);
  }
  if (lane == 63) s.wmax[wave] = inc;
  __syncthreads();
  uint32_t pre = __shfl_up(inc, 1, 64);
  if (lane == 0) pre = 0;
  for (int w = 0; w < wave; ++w) pre = max(pre, s.wmax[w]);
  if (tid * PER < Ac) {
    uint32_t w[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) w[i] = max(v[2 * i], pre) | max(v[2 * i + 1], pre) << 16;
    m4[2 * tid] = make_uint4(w[0], w[1], w[2], w[3]);
    m4[2 * tid + 1] = make_uint4(w[4], w[5], w[6], w[7]);
  }
  __syncthreads();
}

// Folds a thread's gathered values into the LDS accumulators: runs of one
// vertex (kk) within a group are combined in registers first.
template <int ALGO, int EPT, int RUN, typename L>
__device__ inline void tile_fold(L &s, const int (&kk)[EPT], const typename Red<ALGO>::T (&x)[EPT]) {
  using R = Red<ALGO>;
  using T = typename R::T;
  constexpr int G = EPT / RUN;
  if constexpr (is_pr<ALGO>() && L::DET) {
    // each term rounded to fixed point once, so the sum does not depend on
    // which thread adds which run, or in which order
#pragma unroll
    for (int gi = 0; gi < G; ++gi) {
      int ck = kk[gi * RUN];
      unsigned long long cur = (unsigned long long)llrint((double)x[gi * RUN] * FIX_ONE);
#pragma unroll
      for (int i = 1; i < RUN; ++i) {
        const int j = gi * RUN + i;
        const unsigned long long q = (unsigned long long)llrint((double)x[j] * FIX_ONE);
        if (kk[j] == ck) {
          cur += q;
        } else {
          if (ck >= 0) atomicAdd(&s.acc64[ck], cur);
          ck = kk[j];
          cur = q;
        }
      }
      if (ck >= 0) atomicAdd(&s.acc64[ck], cur);
    }
    return;
  }
#pragma unroll
  for (int gi = 0; gi < G; ++gi) {
    int ck = kk[gi * RUN];
    T cur = x[gi * RUN];
#pragma unroll
    for (int i = 1; i < RUN; ++i) {
      const int j = gi * RUN + i;
      if (kk[j] == ck) {
        cur = R::combine(cur, x[j]);
      } else {
        if (ck >= 0) {
          if constexpr (is_pr<ALGO>()) atomicAdd(reinterpret_cast<float *>(&s.acc[ck]), cur);
          else atomicMin(&s.acc[ck], cur);
        }
        ck = kk[j];
        cur = x[j];
      }
    }
    if (ck >= 0) {
      if constexpr (is_pr<ALGO>()) atomicAdd(reinterpret_cast<float *>(&s.acc[ck]), cur);
      else atomicMin(&s.acc[ck], cur);
    }
  }
}

// Phase 2 of a tile over its compacted edge list (pos/eb in LDS, At
// positions, Kt vertices): EDGES_PER_THREAD positions per thread, in groups
// of RUN consecutive ones; group g of thread t starts at g * BLOCK * RUN +
// t * RUN, so a load instruction of a wavefront covers 64 * RUN consecutive
// positions and each thread keeps EDGES_PER_THREAD gathers in flight. A
// group finds its first position's vertex by binary search (monotone over
// the groups) and walks forward; runs of one vertex within a group are
// reduced in registers before one LDS atomic.
template <int ALGO, int EPT, bool PACKED, typename L>
__device__ inline void tile_gather(const Run &r, const PageCtx &p, L &s, int At, int Kt) {
  using R = Red<ALGO>;
  using T = typename R::T;
  const int tid = threadIdx.x;
  constexpr int RUN = 2;
  constexpr int G = EPT / RUN;
  static_assert(EPT % RUN == 0, "groups of RUN positions");
  tile_map(s, 0, At, Kt);
  int kk[EPT];
  int32_t e[EPT];
#pragma unroll
  for (int gi = 0; gi < G; ++gi) {
#pragma unroll
    for (int i = 0; i < RUN; ++i) {
      const int q = gi * BLOCK * RUN + tid * RUN + i;
      const int j = gi * RUN + i;
      kk[j] = -1;
      e[j] = 0;
      if (q < At) {
        const int k = (int)s.map[q] - TILE_V;
        kk[j] = k;
        e[j] = s.eb[k] + q;
      }
    }
  }
  if (tid * RUN >= At) return;
  // unconditional loads: positions past the list reread the thread's first
  // edge (a real one, since its first position is below At)
#pragma unroll
  for (int j = 0; j < EPT; ++j) e[j] = kk[j] >= 0 ? e[j] : e[0];
  T x[EPT];
  uint32_t word[EPT];
#pragma unroll
  for (int j = 0; j < EPT; ++j) word[j] = p.src[e[j]];
#pragma unroll
  for (int j = 0; j < EPT; ++j) {
    const uint32_t w = ALGO == A_SSSP ? weight_of<PACKED>(p, word[j], e[j]) : 0u;
    const T y = R::edge(r, src_of<PACKED>(word[j]), w);
    x[j] = kk[j] >= 0 ? y : R::identity();
  }
  tile_fold<ALGO, EPT, RUN>(s, kk, x);
}

// Phase 2 of a tile of a split image: its narrow list (u16 ids at positions
// [0, An)) and its wide list (edge words at [An, An + At)) form one position
// space covered as above, so a thread's gathers of both lists are in flight
// together. Every position issues one aligned 32-bit load: the edge word, or
// the word holding the u16 id; SSSP also loads the u8 weight of narrow
// positions (wide positions read the first one, unused).
template <int ALGO, int EPT, typename L>
__device__ inline void tile_gather_split(const Run &r, const PageCtx &p, L &s, int An, int At, int Kt) {
  using R = Red<ALGO>;
  using T = typename R::T;
  const int tid = threadIdx.x;
  constexpr int RUN = 2;
  constexpr int G = EPT / RUN;
  const int Ac = An + At;
  tile_map(s, An, At, Kt);
  int kk[EPT];
  int32_t e[EPT];
  bool nar[EPT];
#pragma unroll
  for (int gi = 0; gi < G; ++gi) {
#pragma unroll
    for (int i = 0; i < RUN; ++i) {
      const int q = gi * BLOCK * RUN + tid * RUN + i, j = gi * RUN + i;
      kk[j] = -1;
      e[j] = 0;
      nar[j] = false;
      if (q < Ac) {
        const int code = s.map[q];
        const bool qn = code < TILE_V;
        const int k = qn ? code : code - TILE_V;
        kk[j] = k;
        nar[j] = qn;
        e[j] = qn ? s.eb_n[k] + q : s.eb[k] + (q - An);
      }
    }
  }
  if (tid * RUN >= Ac) return;
#pragma unroll
  for (int j = 0; j < EPT; ++j) {
    e[j] = kk[j] >= 0 ? e[j] : e[0];
    nar[j] = kk[j] >= 0 ? nar[j] : nar[0];
  }
  const char *hs = reinterpret_cast<const char *>(p.hsrc);
  const char *ws = reinterpret_cast<const char *>(p.src);
  uint32_t word[EPT], wt[EPT];
  // 3-byte wide ids: the second aligned word after the first (a narrow
  // position rereads its own word)
  uint32_t word2[L::W3 ? EPT : 1];
#pragma unroll
  for (int j = 0; j < EPT; ++j) {
    if constexpr (L::W3) {
      const char *a = nar[j] ? hs + ((2 * e[j]) & ~3) : ws + ((3u * (uint32_t)e[j]) & ~3u);
      word[j] = *reinterpret_cast<const uint32_t *>(a);
      word2[j] = *reinterpret_cast<const uint32_t *>(nar[j] ? a : a + 4);
    } else {
      const char *a = nar[j] ? hs + ((2 * e[j]) & ~3) : ws + 4 * e[j];
      word[j] = *reinterpret_cast<const uint32_t *>(a);
    }
  }
  if constexpr (ALGO == A_SSSP) {
    // a wavefront's group covers 128 consecutive positions, so it is
    // narrow or wide as a whole except at the lists' boundary: a wholly
    // wide group loads no weights
#pragma unroll
    for (int gi = 0; gi < G; ++gi) {
      const bool any = __ballot(nar[gi * RUN] || nar[gi * RUN + 1]) != 0ull;
#pragma unroll
      for (int i = 0; i < RUN; ++i) {
        const int j = gi * RUN + i;
        wt[j] = any ? (uint32_t)p.hw[nar[j] ? e[j] : 0] : 0u;
      }
    }
  }
  T x[EPT];
#pragma unroll
  for (int j = 0; j < EPT; ++j) {
    const uint32_t un = (word[j] >> (16 * (e[j] & 1))) & 0xFFFFu;
    uint32_t uw;
    if constexpr (L::W3) uw = __builtin_amdgcn_alignbyte(word2[j], word[j], (3u * (uint32_t)e[j]) & 3u) & 0xFFFFFFu;
    else uw = src_of<true>(word[j]);
    const uint32_t u = nar[j] ? un : uw;
    uint32_t w = 0u;
    if constexpr (ALGO == A_SSSP) w = nar[j] ? wt[j] : (word[j] >> 24);
    const T y = R::edge(r, (int32_t)u, w);
    x[j] = kk[j] >= 0 ? y : R::identity();
  }
  tile_fold<ALGO, EPT, RUN>(s, kk, x);
}

template <int ALGO, int EDGES_PER_THREAD, bool PACKED, typename L>
__device__ void sweep_tile(const Run &r, const PageCtx &p, int item, Acc &acc, L &s) {
  constexpr bool SPLIT = L::SPLIT;
  using R = Red<ALGO>;
  const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
  const int32_t t0 = p.tiles[2 * item], t1 = p.tiles[2 * item + 1];
  const int nv = t1 - t0;
  // phase 1: gate, degrees, block scan of (attempting vertices, their edges)
  // (split images: narrow edges [nb, nb + dn) and wide edges [eb, eb + d))
  int32_t lv[2], eb[2], d[2], nb[2] = {0, 0}, dn[2] = {0, 0};
  Gate gt[2];
  bool act[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    // loads are unconditional (lanes past the tile reread its first vertex)
    // so the offset, value and state loads of both vertices overlap
    const int i = 2 * tid + j;
    const bool in = i < nv;
    lv[j] = t0 + (in ? i : 0);
    if constexpr (SPLIT) {
      // ends of this vertex and of the one before it (0 at the tile's start),
      // narrow in the low and wide in the high 16 bits
      const int2 tb = p.tbase[item];  // (in-edges, narrow edges) before the tile
      const uint32_t e1 = p.vpk[lv[j]];
      const uint32_t e0r = p.vpk[lv[j] > 0 ? lv[j] - 1 : 0];
      const uint32_t e0 = lv[j] > t0 ? e0r : 0u;
      nb[j] = tb.y + (int32_t)(e0 & 0xFFFFu);
      dn[j] = (int32_t)(e1 & 0xFFFFu) - (int32_t)(e0 & 0xFFFFu);
      eb[j] = tb.x - tb.y + (int32_t)(e0 >> 16);  // wide edges before the vertex
      d[j] = (int32_t)(e1 >> 16) - (int32_t)(e0 >> 16);
    } else {
      eb[j] = p.off[lv[j]];
      d[j] = p.off[lv[j] + 1] - eb[j];
    }
    gt[j] = gate_of(r, p.v_begin + lv[j]);
    act[j] = in && (gt[j].attempt || r.audit) && (d[j] + dn[j] > 0 || is_pr<ALGO>());
  }
  // BFS early break (Section 5.5): after the threshold's k passes every level <= k is
  // final and every other vertex is at level >= k + 1, so a vertex whose
  // first in-neighbour (the smallest internal id: the highest-degree one
  // under degree numbering) is at level k is at level k + 1 and its other
  // in-edges are not read. Otherwise the probed edge seeds the reduction
  // and the scan starts after it, so no edge is read twice.
  uint32_t seed[2] = {INF, INF};
  if constexpr (ALGO == A_BFS) {
    if (r.early) {
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        if (act[j]) {
          const bool nar = SPLIT && dn[j] > 0;
          const int32_t u = nar ? (int32_t)p.hsrc[nb[j]] : src_of<PACKED>(wide_word<SPLIT && L::W3>(p, eb[j]));
          const uint32_t x = r.value[u];
          acc.edges += 1;
          if (nar) acc.narrow += 1;
          seed[j] = x == INF ? INF : x + 1u;
          if (nar) { nb[j] += 1; dn[j] -= 1; } else { eb[j] += 1; d[j] -= 1; }
          if (x == r.threshold) { d[j] = 0; dn[j] = 0; }
        }
      }
    }
  }
  int na = (int)act[0] + (int)act[1];
  int ne = (act[0] ? d[0] : 0) + (act[1] ? d[1] : 0);
  int nn = (act[0] ? dn[0] : 0) + (act[1] ? dn[1] : 0);
  int ina = na, ine = ne, inn = nn;  // inclusive scan within the wavefront
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) {
    int a = __shfl_up(ina, m, 64), b = __shfl_up(ine, m, 64);
    int c = SPLIT ? __shfl_up(inn, m, 64) : 0;
    if (lane >= m) { ina += a; ine += b; inn += c; }
  }
  if (lane == 63) { s.wsum[wave][0] = ina; s.wsum[wave][1] = ine; s.wsum[wave][2] = inn; }
  __syncthreads();
  int ka = 0, pe = 0, pn = 0, Kt = 0, At = 0, An = 0;
  for (int w = 0; w < WAVES; ++w) {
    if (w < wave) { ka += s.wsum[w][0]; pe += s.wsum[w][1]; pn += s.wsum[w][2]; }
    Kt += s.wsum[w][0];
    At += s.wsum[w][1];
    An += s.wsum[w][2];
  }
  ka += ina - na;
  pe += ine - ne;
  pn += inn - nn;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    if (act[j]) {
      s.pos[ka] = pe;
      s.eb[ka] = eb[j] - pe;  // so that a position's edge is eb + position
      if constexpr (SPLIT) {
        s.pos_n[ka] = pn;
        s.eb_n[ka] = nb[j] - pn;
      }
      s.vl[ka] = lv[j];
      // the early break's probe (BFS) seeds the reduction
      s.acc[ka] = ALGO == A_BFS ? seed[j] : R::bits(R::identity());
      if constexpr (L::DET) s.acc64[ka] = 0ull;
      s.old[ka] = gt[j].old;
      s.att[ka] = gt[j].attempt ? 1 : 0;
      s.st[ka] = gt[j].st;
      ++ka;
      pe += d[j];
      pn += dn[j];
    } else if (2 * tid + j < nv) {
      // not pulled this sweep: skipped by the predictor, or no in-edge
      epilogue<ALGO>(r, p.v_begin + lv[j], gt[j], false, R::identity(), (uint32_t)(d[j] + dn[j]), acc);
    }
  }
  if (tid == 0) {
    s.pos[Kt] = At;
    if constexpr (SPLIT) s.pos_n[Kt] = An;
  }
  __syncthreads();
  // phase 2: the wide edges, then (split images) the narrow ones
  if constexpr (SPLIT) tile_gather_split<ALGO, EDGES_PER_THREAD>(r, p, s, An, At, Kt);
  else tile_gather<ALGO, EDGES_PER_THREAD, PACKED>(r, p, s, At, Kt);
  __syncthreads();
  // phase 3: epilogues of the pulled vertices
  for (int k = tid; k < Kt; k += BLOCK) {
    Gate g{s.att[k] != 0, s.st[k], s.old[k]};
    uint32_t dn_k = 0u;
    if constexpr (SPLIT) dn_k = (uint32_t)(s.pos_n[k + 1] - s.pos_n[k]);
    if (SPLIT && g.attempt) acc.narrow += dn_k;
    RedArg<ALGO> red;
    if constexpr (L::DET && is_pr<ALGO>()) red = (double)s.acc64[k] / FIX_ONE;
    else red = R::from_bits(s.acc[k]);
    const bool ch = epilogue<ALGO>(r, p.v_begin + s.vl[k], g, true, red,
                                   (uint32_t)(s.pos[k + 1] - s.pos[k]) + dn_k, acc);
    frontier_push(r, ch, p.v_begin + s.vl[k]);
  }
}

// ----------------------------------------------------------------- bin 7
// One wavefront per CHUNK edges of a heavy vertex. Each chunk folds its
// partial into the vertex's accumulator with one device-scope atomic (min,
// or an exact fixed-point add for PageRank sums); the close kernel, after
// the sweep has finished, takes the accumulator (resetting it) and runs the
// vertex's epilogue, so no fence or arrival counter is needed in the sweep.
// Edges [a, b) of one chunk list, lanes strided, batches of B per lane:
// B loads, then B gathers, all in flight together (lanes past the range
// reread its first edge). NARROW: u16 ids and u8 weights of a split image.
template <int ALGO, bool PACKED, bool NARROW, bool W3 = false>
__device__ inline typename Red<ALGO>::T chunk_range(const Run &r, const PageCtx &p, int32_t a, int32_t b,
                                                    typename Red<ALGO>::T x) {
  using R = Red<ALGO>;
  using T = typename R::T;
  const int lane = threadIdx.x % 64;
  constexpr int B = 8;
  for (int e0 = a + lane; e0 < b; e0 += B * 64) {
    int32_t ei[B];
    uint32_t q[B], w[B];
#pragma unroll
    for (int j = 0; j < B; ++j) {
      ei[j] = e0 + j * 64 < b ? e0 + j * 64 : a;
      if constexpr (NARROW) {
        q[j] = p.hsrc[ei[j]];
        w[j] = ALGO == A_SSSP ? (uint32_t)p.hw[ei[j]] : 0u;
      } else {
        q[j] = wide_word<W3>(p, ei[j]);
      }
    }
#pragma unroll
    for (int j = 0; j < B; ++j) {
      T y;
      if constexpr (NARROW) y = R::edge(r, (int32_t)q[j], w[j]);
      else y = R::edge(r, src_of<PACKED>(q[j]), ALGO == A_SSSP ? weight_of<PACKED>(p, q[j], ei[j]) : 0u);
      if (e0 + j * 64 < b) x = R::combine(x, y);
    }
  }
  return x;
}

template <int ALGO, bool PACKED, bool SPLIT, bool W3 = false>
__device__ void sweep_chunk(const Run &r, const PageCtx &p, int item) {
  using R = Red<ALGO>;
  using T = typename R::T;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  int idx = item * WAVES + wave;
  if (idx >= p.bin_count) return;
  Chunk c = p.chunks[idx];
  int32_t v = p.v_begin + c.vl;
  Gate g = gate_of(r, v);
  bool comp = g.attempt || r.audit;
  T x = R::identity();
  // split images: the vertex's edges are its narrow ones, then its wide
  // ones; the chunk covers [e_begin, e_end) of that order
  int32_t v0 = 0, nb = 0, dn = 0;
  if constexpr (SPLIT) {
    const int4 hs = p.hside[p.vpk[c.vl]];
    v0 = hs.x;
    nb = hs.y;
    dn = hs.z;
  }
  bool scan = comp;
  if constexpr (ALGO == A_BFS) {
    // early break, as in tiles: every chunk of the vertex probes its first in-edge
    if (comp && r.early) {
      int32_t u;
      if (SPLIT && dn > 0) u = (int32_t)p.hsrc[nb];
      else if (SPLIT) u = src_of<PACKED>(wide_word<W3>(p, v0 - nb));
      else u = src_of<PACKED>(p.src[p.off[c.vl]]);
      if (r.value[u] == r.threshold) {
        x = r.threshold + 1u;
        scan = false;
      }
    }
  }
  if (scan) {
    if constexpr (SPLIT) {
      // narrow part: combined positions [v0, v0 + dn) -> narrow entries from nb
      const int32_t na = max(c.e_begin, v0), nz = min(c.e_end, v0 + dn);
      if (na < nz) x = chunk_range<ALGO, PACKED, true>(r, p, nb + (na - v0), nb + (nz - v0), x);
      // wide part: combined positions [v0 + dn, ...) -> wide words from v0 - nb
      const int32_t wa = max(c.e_begin, v0 + dn), wz = c.e_end;
      if (wa < wz) x = chunk_range<ALGO, PACKED, false, W3>(r, p, wa - nb - dn, wz - nb - dn, x);
    } else {
      x = chunk_range<ALGO, PACKED, false>(r, p, c.e_begin, c.e_end, x);
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) x = R::combine(x, shfl_xor(x, m));
  }
  if (comp && lane == 0) {
    unsigned long long *slot = &p.partial[(uint32_t)c.first_count & 0xFFFFFu];
    if constexpr (is_pr<ALGO>()) atomicAdd(slot, (unsigned long long)llrint((double)x * FIX_ONE));
    else atomicMin(reinterpret_cast<uint32_t *>(slot), R::bits(x));
  }
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
    if (c->delta) {
      // the dangling mass sent in this pass is received in the next one
      c->dangling = c->dangling_next;
      c->dangling_next = 0.0;
    }
    // FP32 floor: a pass counts as an improvement only when its L1 falls at
    // least 10% below the best so far (smaller steps are rounding noise)
    const bool better = l1 < 0.9 * c->best_l1;
    c->no_improve = better ? 0 : c->no_improve + 1;
    c->best_l1 = better ? l1 : fmin(c->best_l1, l1);
    if (c->phase == 1) {
      if (l1 < c->tol_l1) { c->done = 1; c->stop_reason = 1; }
      else if (l1 < c->floor_cap && c->no_improve >= 3) { c->done = 1; c->stop_reason = 2; }
    } else {
      if (l1 < c->tol_l1 || (l1 < c->floor_cap && c->no_improve >= 3)) {
        // PageRank-delta leaves its residual phase here; the host turns the
        // ranks into rank-form terms before the verification passes
        c->phase = 1;
        c->delta = 0;
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

// Totals of one sweep, as reduced by the close kernel.
struct SweepTotals {
  unsigned long long changed, edges, attempted, skipped, mispred, hist[8], narrow;
  uint32_t min_changed;
  double l1, ddelta, dmass;
};

// Fold a sweep into the pass (one thread) and fill its record in `rec`
// (LDS); the caller copies the record to the host ring with wide stores.
__device__ void close_sweep(Ctl *c, SweepRecord *rec, int end_of_pass, const SweepTotals &t) {
  const uint32_t seq = c->sweep_seq;
  rec->seq = seq;
  rec->changed = t.changed;
  rec->edges = t.edges;
  rec->edges_narrow = t.narrow;
  rec->attempted = t.attempted;
  rec->skipped = t.skipped;
  rec->mispred = t.mispred;
  rec->l1 = t.l1;
  rec->min_changed = t.min_changed;
  rec->threshold = c->threshold;
  rec->phase = c->phase;
  for (int i = 0; i < 8; ++i) rec->hist[i] = t.hist[i];
  rec->pass_l1_closed = -1.0;
  c->pass_changed += t.changed;
  c->pass_min_changed = min(c->pass_min_changed, t.min_changed);
  c->pass_l1 += t.l1;
  if (c->delta) c->dangling_next += t.ddelta;  // sent mass, received in the next pass
  else c->dangling += t.ddelta;
  c->mass += t.dmass;
  c->win_quiet = t.changed == 0 ? 1u : 0u;
  c->sweep_seq = seq + 1;
  if (end_of_pass) close_pass(c, rec);
  if (!end_of_pass) { rec->done_after = c->done; rec->pass_after = c->pass; rec->stop_reason = c->stop_reason; }
  rec->dangling = c->dangling;
  rec->phase_after = c->phase;
  rec->pad_ = 0;
}

// Copy a record staged in LDS to the host-mapped ring: one 16-byte store
// per thread of the first wavefront, so the PCIe writes go out together.
__device__ inline void publish_record(const SweepRecord *src, SweepRecord *dst) {
  static_assert(sizeof(SweepRecord) % 16 == 0, "record is a whole number of 16-byte words");
  constexpr int WORDS = sizeof(SweepRecord) / 16;
  static_assert(WORDS <= 64, "one wavefront writes the record");
  if (threadIdx.x < WORDS)
    reinterpret_cast<uint4 *>(dst)[threadIdx.x] = reinterpret_cast<const uint4 *>(src)[threadIdx.x];
}

// ------------------------------------------------------------ the sweep
template <int ALGO, int EPT, bool PACKED, bool SPLIT, bool DET = false, bool W3 = false>
__global__ void __launch_bounds__(BLOCK) sweep_kernel(SweepArgs a) {
  Ctl *ctl = a.ctl;
  // converged, or a later sweep of a window whose last sweep changed
  // nothing: every block leaves before counting
  if (ctl->done || (a.win_skip && !a.win_first && ctl->win_quiet)) return;
  __shared__ uint32_t s_hist[8];
  __shared__ uint32_t s_u32[WAVES][7];
  __shared__ double s_f64[WAVES][3];
  __shared__ TileLds<SPLIT, DET, W3> s_tile;
  if (threadIdx.x < 8) s_hist[threadIdx.x] = 0;

  // locate (page, section, item) of this block: section 0 = tiles, 1 = chunks
  const int b = blockIdx.x;
  int lo = 0, hi = a.nent * NSEC;  // prefix[lo] <= b < prefix[hi]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (a.blk_prefix[mid] <= b) lo = mid; else hi = mid;
  }
  const int ent = lo / NSEC, sec = lo % NSEC, item = b - a.blk_prefix[lo];
  const char *base = a.base[ent];
  const PageHeader *h = reinterpret_cast<const PageHeader *>(base);
  PageCtx p;
  p.v_begin = h->v_begin;
  p.off = reinterpret_cast<const int32_t *>(base + h->off_offsets);
  p.bins = reinterpret_cast<const int32_t *>(base + h->off_bins);
  p.tiles = reinterpret_cast<const int32_t *>(base + h->off_tiles);
  p.chunks = reinterpret_cast<const Chunk *>(base + h->off_chunks);
  p.src = reinterpret_cast<const uint32_t *>(base + h->off_src);
  p.w = reinterpret_cast<const uint32_t *>(base + h->off_w);
  p.vpk = reinterpret_cast<const uint32_t *>(base + h->off_vpk);
  p.tbase = reinterpret_cast<const int2 *>(base + h->off_tbase);
  p.hside = reinterpret_cast<const int4 *>(base + h->off_hside);
  p.hsrc = reinterpret_cast<const uint16_t *>(base + h->off_hsrc);
  p.hw = reinterpret_cast<const uint8_t *>(base + h->off_w);
  p.bin_count = h->bin_count[BIN_CHUNK];
  p.bin_start = 0;
  p.partial = a.partial[ent];

  Run r;
  r.algo = ALGO;
  r.pvu = ctl->pvu;
  r.phase = ctl->phase;
  r.audit = a.audit && r.phase == 0 && r.pvu != P_OFF;
  r.early = ALGO == A_BFS && a.early && !a.audit && r.phase == 0 && r.pvu == P_STRONG;
  r.threshold = ctl->threshold;
  r.value = a.value;
  r.delta = a.delta && ctl->delta;
  r.resid = a.resid;
  r.contrib = a.contrib;
  r.contrib_w = (a.det || r.delta) ? a.contrib_next : a.contrib;
  r.inv_outdeg = a.inv_outdeg;
  r.status = a.status;
  r.dia = &a.dia;
  r.damping = a.damping;
  r.pr_eps = a.pr_eps;
  r.base_uniform = 1.0f / (float)a.n;
  r.dangling = ctl->dangling;
  r.inv_mass = 1.0 / ctl->mass;
  r.pr_seed = a.pr_seed;
  r.hist = s_hist;
  r.collect = a.collect;
  r.frontier = a.frontier;
  r.fr_count = a.fr_count;
  r.fr_cap = a.fr_cap;
  __syncthreads();

  Acc acc;
  // a launch over pages without any work still runs one block, so the
  // sweep (and the pass) is closed the same way
  if (b < a.blk_prefix[a.nent * NSEC]) {
    if (sec == 0) sweep_tile<ALGO, EPT, PACKED>(r, p, item, acc, s_tile);
    else sweep_chunk<ALGO, PACKED, SPLIT, W3>(r, p, item);
  }

  // block reduction of the counters, then one set of device-scope atomics
  // into this block's stripe (no block waits for another)
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  uint32_t v0 = wave_sum_u32(acc.changed), v1 = wave_sum_u32(acc.attempted),
           v2 = wave_sum_u32(acc.skipped), v3 = wave_sum_u32(acc.mispred),
           v4 = wave_sum_u32(acc.edges), v5 = wave_min_u32(acc.min_changed),
           v6 = SPLIT ? wave_sum_u32(acc.narrow) : 0u;
  double f0 = 0.0, f1 = 0.0, f2 = 0.0;
  if constexpr (is_pr<ALGO>()) {
    f0 = wave_sum_f64(acc.l1); f1 = wave_sum_f64(acc.ddelta); f2 = wave_sum_f64(acc.dmass);
  }
  if (lane == 0) {
    s_u32[wave][0] = v0; s_u32[wave][1] = v1; s_u32[wave][2] = v2;
    s_u32[wave][3] = v3; s_u32[wave][4] = v4; s_u32[wave][5] = v5; s_u32[wave][6] = v6;
    s_f64[wave][0] = f0; s_f64[wave][1] = f1; s_f64[wave][2] = f2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long ch = 0, at = 0, sk = 0, mp = 0, ed = 0, nr = 0;
    uint32_t mn = INF;
    double l1 = 0.0, dd = 0.0, dm = 0.0;
    for (int w = 0; w < WAVES; ++w) {
      ch += s_u32[w][0]; at += s_u32[w][1]; sk += s_u32[w][2]; mp += s_u32[w][3]; ed += s_u32[w][4];
      mn = min(mn, s_u32[w][5]);
      nr += s_u32[w][6];
      l1 += s_f64[w][0]; dd += s_f64[w][1]; dm += s_f64[w][2];
    }
    Stripe &st = a.stripes[blockIdx.x % NSTRIPE];
    if (ch | at) atomicAdd(&st.ca, ch | at << 32);
    if (sk | mp) atomicAdd(&st.sm, sk | mp << 32);
    if (ed) atomicAdd(&st.edges, ed);
    if (nr) atomicAdd(&st.narrow, nr);
    if (mn != INF) atomicMin(&st.min_changed, mn);
    if constexpr (is_pr<ALGO>()) {
      if (l1 != 0.0) atomicAdd(&st.l1, (unsigned long long)llrint(l1 * FIX_ONE));
      if (dd != 0.0) atomicAdd(&st.dd, (unsigned long long)llrint(dd * FIX_ONE));
      if (dm != 0.0) atomicAdd(&st.dm, (unsigned long long)llrint(dm * FIX_ONE));
    }
  }
  if (r.pvu == P_WEAK && threadIdx.x < 4) {
    const unsigned long long hw = (unsigned long long)s_hist[2 * threadIdx.x] |
                                  (unsigned long long)s_hist[2 * threadIdx.x + 1] << 32;
    if (hw) atomicAdd(&a.stripes[blockIdx.x % NSTRIPE].hist[threadIdx.x], hw);
  }
}

// Close a sweep: take the accumulator of every heavy vertex (resetting it)
// and run its epilogue, take the counter stripes (resetting them), and fold
// the totals into the control block (and close the pass). One block of
// CLOSE_THREADS threads, after the sweep.
constexpr int CLOSE_THREADS = 1024;

template <int ALGO>
__global__ void __launch_bounds__(CLOSE_THREADS) close_kernel(SweepArgs a) {
  using R = Red<ALGO>;
  using T = typename R::T;
  constexpr int CW = sizeof(Ctl) / 4;
  static_assert(CW <= 64 && NSTRIPE <= 64, "the first wavefront stages the control block, the second takes the stripes");
  __shared__ Ctl s_ctl;
  __shared__ uint32_t s_hist[8];
  __shared__ unsigned long long s_red[CLOSE_THREADS / 64][6];
  __shared__ uint32_t s_min[CLOSE_THREADS / 64];
  __shared__ double s_fl[CLOSE_THREADS / 64][3];
  __shared__ __align__(16) SweepRecord s_rec;
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64, nw = CLOSE_THREADS / 64;
  // independent loads first: the control block is staged in LDS (all of the
  // close logic then runs on the copy), and the second wavefront takes the
  // counter stripes (a stripe is the identity when its sweep did nothing)
  if (tid < CW) reinterpret_cast<uint32_t *>(&s_ctl)[tid] = reinterpret_cast<const uint32_t *>(a.ctl)[tid];
  if (tid < 8) s_hist[tid] = 0;
  unsigned long long c0 = 0, c1 = 0, c2 = 0, c3 = 0, c4 = 0, c5 = 0, hw[4] = {0, 0, 0, 0};
  uint32_t mn = INF;
  double l1 = 0.0, dd = 0.0, dm = 0.0;
  if (wave == 1 && lane < NSTRIPE) {
    Stripe &st = a.stripes[lane];
    const unsigned long long ca = atomicExch(&st.ca, 0ull), sm = atomicExch(&st.sm, 0ull);
    c0 = ca & 0xFFFFFFFFull; c1 = ca >> 32;
    c2 = sm & 0xFFFFFFFFull; c3 = sm >> 32;
    c4 = atomicExch(&st.edges, 0ull);
    c5 = atomicExch(&st.narrow, 0ull);
    mn = atomicExch(&st.min_changed, INF);
    if constexpr (is_pr<ALGO>()) {
      l1 = (double)atomicExch(&st.l1, 0ull) / FIX_ONE;
      dd = (double)(long long)atomicExch(&st.dd, 0ull) / FIX_ONE;
      dm = (double)(long long)atomicExch(&st.dm, 0ull) / FIX_ONE;
    }
    for (int k = 0; k < 4; ++k) hw[k] = atomicExch(&st.hist[k], 0ull);
  }
  __syncthreads();
  if (s_ctl.done) return;  // the sweep was a no-op as well
  if (a.win_skip && !a.win_first && s_ctl.win_quiet) {
    // a sweep its window skipped still leaves a record (no counts), so the
    // records number the launches and a host that has waited for launch k
    // reads records up to k only
    if (tid == 0) {
      SweepRecord &rec = s_rec;
      rec = SweepRecord{};
      rec.seq = s_ctl.sweep_seq;
      rec.min_changed = INF;
      rec.threshold = s_ctl.threshold;
      rec.phase = s_ctl.phase;
      rec.done_after = s_ctl.done;
      rec.pass_after = s_ctl.pass;
      rec.stop_reason = s_ctl.stop_reason;
      rec.dangling = s_ctl.dangling;
      rec.pass_l1_closed = -1.0;
      rec.phase_after = s_ctl.phase;
      a.ctl->sweep_seq = s_ctl.sweep_seq + 1;
    }
    __syncthreads();
    if (a.ring) publish_record(&s_rec, &a.ring[s_rec.seq & a.ring_mask]);
    return;
  }
  Run r;
  r.algo = ALGO;
  r.pvu = s_ctl.pvu;
  r.phase = s_ctl.phase;
  r.audit = a.audit && r.phase == 0 && r.pvu != P_OFF;
  r.threshold = s_ctl.threshold;
  r.value = a.value;
  r.delta = a.delta && s_ctl.delta;
  r.resid = a.resid;
  r.contrib = a.contrib;
  r.contrib_w = (a.det || r.delta) ? a.contrib_next : a.contrib;
  r.inv_outdeg = a.inv_outdeg;
  r.status = a.status;
  r.dia = &a.dia;
  r.damping = a.damping;
  r.pr_eps = a.pr_eps;
  r.base_uniform = 1.0f / (float)a.n;
  r.dangling = s_ctl.dangling;
  r.inv_mass = 1.0 / s_ctl.mass;
  r.pr_seed = a.pr_seed;
  r.hist = s_hist;
  r.collect = a.collect;
  r.frontier = a.frontier;
  r.fr_count = a.fr_count;
  r.fr_cap = a.fr_cap;
  for (int k = 0; k < 4; ++k) {
    if (hw[k]) {
      atomicAdd(&s_hist[2 * k], (uint32_t)(hw[k] & 0xFFFFFFFFull));
      atomicAdd(&s_hist[2 * k + 1], (uint32_t)(hw[k] >> 32));
    }
  }
  Acc acc;
  // one thread per heavy vertex: one exchange takes its accumulated
  // reduction and leaves the identity for the next sweep
  for (int ent = 0; ent < a.nent; ++ent) {
    const char *base = a.base[ent];
    const PageHeader *h = reinterpret_cast<const PageHeader *>(base);
    const Heavy *hv = reinterpret_cast<const Heavy *>(base + h->off_heavy);
    const int32_t *off = reinterpret_cast<const int32_t *>(base + h->off_offsets);
    const int4 *hside = reinterpret_cast<const int4 *>(base + h->off_hside);
    const bool split = h->split != 0;
    unsigned long long *part = a.partial[ent];
    for (int i = tid; i < h->n_heavy; i += CLOSE_THREADS) {
      const Heavy x = hv[i];
      const uint32_t first = (uint32_t)x.first_count & 0xFFFFFu;
      const int32_t v = h->v_begin + x.vl;
      // taken even when the gate says skip, so every accumulator is back at
      // the identity when the next sweep starts
      RedArg<ALGO> t;
      if constexpr (is_pr<ALGO>()) t = (double)(long long)atomicExch(&part[first], 0ull) / FIX_ONE;
      else t = R::from_bits(atomicExch(reinterpret_cast<uint32_t *>(&part[first]), INF));
      Gate g = gate_of(r, v);
      bool comp = g.attempt || r.audit;
      if (!comp) t = R::identity();
      // split images have no offsets: the heavy table holds the in-degree
      int4 hs = make_int4(0, 0, 0, 0);
      if (split) hs = hside[i];
      if (split && g.attempt) acc.narrow += (uint32_t)hs.z;
      const uint32_t deg = split ? (uint32_t)hs.w : (uint32_t)(off[x.vl + 1] - off[x.vl]);
      const bool ch = epilogue<ALGO>(r, v, g, comp, t, deg, acc);
      frontier_push(r, ch, v);
    }
  }
  c0 += acc.changed; c1 += acc.attempted; c2 += acc.skipped; c3 += acc.mispred; c4 += acc.edges;
  c5 += acc.narrow;
  mn = min(mn, acc.min_changed);
  l1 += acc.l1; dd += acc.ddelta; dm += acc.dmass;
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    c0 += shfl_xor(c0, m); c1 += shfl_xor(c1, m); c2 += shfl_xor(c2, m);
    c3 += shfl_xor(c3, m); c4 += shfl_xor(c4, m); c5 += shfl_xor(c5, m);
    mn = min(mn, shfl_xor(mn, m));
    l1 += shfl_xor(l1, m); dd += shfl_xor(dd, m); dm += shfl_xor(dm, m);
  }
  if (lane == 0) {
    s_red[wave][0] = c0; s_red[wave][1] = c1; s_red[wave][2] = c2; s_red[wave][3] = c3; s_red[wave][4] = c4;
    s_red[wave][5] = c5;
    s_min[wave] = mn;
    s_fl[wave][0] = l1; s_fl[wave][1] = dd; s_fl[wave][2] = dm;
  }
  __syncthreads();
  if (tid == 0) {
    SweepTotals t{};
    t.min_changed = INF;
    for (int w = 0; w < nw; ++w) {
      t.changed += s_red[w][0]; t.attempted += s_red[w][1]; t.skipped += s_red[w][2];
      t.mispred += s_red[w][3]; t.edges += s_red[w][4]; t.narrow += s_red[w][5];
      t.min_changed = min(t.min_changed, s_min[w]);
      t.l1 += s_fl[w][0]; t.ddelta += s_fl[w][1]; t.dmass += s_fl[w][2];
    }
    for (int k = 0; k < 8; ++k) t.hist[k] = s_hist[k];  // sweep blocks and heavy vertices
    close_sweep(&s_ctl, &s_rec, a.end_of_pass, t);
  }
  __syncthreads();
  if (tid < CW) reinterpret_cast<uint32_t *>(a.ctl)[tid] = reinterpret_cast<const uint32_t *>(&s_ctl)[tid];
  if (a.ring) publish_record(&s_rec, &a.ring[s_rec.seq & a.ring_mask]);
}

// Deterministic PageRank sweeps: copy the terms the sweep wrote for the
// window's vertices back into the gathered array. contrib_next equals
// contrib everywhere outside a sweep (it starts as a copy and every sweep is
// followed by this copy), so a sweep that did nothing copies equal values.
// Grid: x strides over a page's vertices, y = page of the window.
__global__ void __launch_bounds__(BLOCK) det_commit_kernel(SweepArgs a) {
  const int ent = blockIdx.y;
  if (ent >= a.nent) return;
  const PageHeader *h = reinterpret_cast<const PageHeader *>(a.base[ent]);
  const int32_t v0 = h->v_begin, v1 = h->v_begin + h->n_p;
  for (int32_t v = v0 + (int32_t)(blockIdx.x * BLOCK + threadIdx.x); v < v1; v += (int32_t)(gridDim.x * BLOCK))
    a.contrib[v] = a.contrib_next[v];
}

// The vertices the next pass would attempt under strong prediction: an
// in-edge and a value above the Table I threshold (every other vertex is
// final or cannot change). Appended to list up to cap; *count receives how
// many there are. In a verification phase every vertex with an in-edge is
// attempted.
__global__ void __launch_bounds__(BLOCK) open_list_kernel(const uint32_t *value, const uint32_t *has_in, int32_t n,
                                                          const Ctl *ctl, uint32_t *list, uint32_t cap,
                                                          uint32_t *count) {
  const int32_t v = (int32_t)(blockIdx.x * BLOCK + threadIdx.x);
  bool open = false;
  if (v < n) {
    const bool in = (has_in[v >> 5] >> (v & 31)) & 1u;
    open = in && (ctl->phase != 0 || value[v] > ctl->threshold);
  }
  const unsigned long long b = __ballot(open);
  if (b == 0ull) return;
  const int lane = threadIdx.x % 64;
  uint32_t base = 0;
  if (lane == 0) base = atomicAdd(count, (uint32_t)__popcll(b));
  base = __shfl(base, 0, 64);
  const uint32_t idx = base + (uint32_t)__popcll(b & ((1ull << lane) - 1ull));
  if (open && idx < cap) list[idx] = (uint32_t)v;
}

// A guess for the copy schedule near a pass end: of the vertices below
// v_limit (the pages the pass has finished), those the next pass would
// attempt if the pass ended now (its smallest change so far as the SSSP/CC
// threshold; BFS: the next pass count). Counting only.
__global__ void __launch_bounds__(BLOCK) open_guess_kernel(const uint32_t *value, const uint32_t *has_in,
                                                           int32_t v_limit, const Ctl *ctl, uint32_t *count) {
  const int32_t v = (int32_t)(blockIdx.x * BLOCK + threadIdx.x);
  bool open = false;
  if (v < v_limit) {
    const uint32_t thr = ctl->algo == A_BFS ? ctl->pass + 1u
                                            : (ctl->pass_changed > 0 ? ctl->pass_min_changed : ctl->threshold);
    const bool in = (has_in[v >> 5] >> (v & 31)) & 1u;
    open = in && (ctl->phase != 0 || value[v] > thr);
  }
  const unsigned long long b = __ballot(open);
  if (b != 0ull && threadIdx.x % 64 == 0) atomicAdd(count, (uint32_t)__popcll(b));
}

__global__ void end_pass_kernel(Ctl *ctl, SweepRecord *ring, uint32_t mask) {
  // a pass closed on its own gets a record of its own (no sweep counters)
  __shared__ __align__(16) SweepRecord s_rec;
  if (ctl->done) return;
  if (threadIdx.x == 0) {
    const uint32_t seq = ctl->sweep_seq;
    SweepRecord &rec = s_rec;
    rec.seq = seq; rec.changed = 0; rec.edges = 0; rec.attempted = 0; rec.skipped = 0;
    rec.mispred = 0; rec.l1 = 0.0; rec.min_changed = INF; rec.threshold = ctl->threshold;
    rec.phase = ctl->phase;
    for (int i = 0; i < 8; ++i) rec.hist[i] = 0;
    rec.edges_narrow = 0;
    rec.pad_ = 0;
    ctl->sweep_seq = seq + 1;
    close_pass(ctl, &rec);
    rec.dangling = ctl->dangling;
    rec.phase_after = ctl->phase;
  }
  __syncthreads();
  if (ring) publish_record(&s_rec, &ring[s_rec.seq & mask]);
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

__global__ void init_prd_kernel(float *rank, float *resid, float *contrib, float *contrib_next, int32_t n,
                                int32_t seed, double damping) {
  int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const double t = seed < 0 ? 1.0 / (double)n : (v == seed ? 1.0 : 0.0);
  rank[v] = 0.0f;
  resid[v] = (float)((1.0 - damping) * t);
  contrib[v] = 0.0f;
  contrib_next[v] = 0.0f;
}

__global__ void rank_terms_kernel(const float *rank, float *contrib, const float *inv_outdeg, int32_t n) {
  int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  contrib[v] = rank[v] * inv_outdeg[v];
}

// Gather-rate probe: the sweep's tiling (TILE_E words per block; thread t
// takes groups of 2 consecutive words starting at g * BLOCK * 2 + t * 2,
// loads issued together) over a plain word array, every word's value
// gathered and summed; one add per block.
__global__ void __launch_bounds__(BLOCK) gather_probe_kernel(const uint32_t *src, int64_t m, uint32_t mask,
                                                             const uint32_t *val, int32_t n,
                                                             unsigned long long *sink) {
  constexpr int EPT = TILE_E / BLOCK;
  constexpr int RUN = 2;
  __shared__ unsigned long long s[WAVES];
  const int64_t b0 = (int64_t)blockIdx.x * TILE_E;
  const int64_t first = b0 + (int64_t)threadIdx.x * RUN;
  unsigned long long acc = 0;
  if (first < m) {
    int64_t e[EPT];
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
      const int64_t q = b0 + (int64_t)(j / RUN) * (BLOCK * RUN) + (int64_t)threadIdx.x * RUN + (j % RUN);
      e[j] = q < m ? q : -1;
    }
    uint32_t w[EPT];
#pragma unroll
    for (int j = 0; j < EPT; ++j) w[j] = src[e[j] >= 0 ? e[j] : first];
    uint32_t x[EPT];
#pragma unroll
    for (int j = 0; j < EPT; ++j) x[j] = val[min(w[j] & mask, (uint32_t)(n - 1))];
#pragma unroll
    for (int j = 0; j < EPT; ++j) acc += e[j] >= 0 ? x[j] : 0u;
  }
#pragma unroll
  for (int k = 32; k >= 1; k >>= 1) acc += shfl_xor(acc, k);
  if (threadIdx.x % 64 == 0) s[threadIdx.x / 64] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int w = 0; w < WAVES; ++w) t += s[w];
    atomicAdd(sink, t);
  }
}

// PageRank run start: the rank sum and the dangling sum of the current
// ranks (fresh or resumed) into the control block. One block; FP64 sums.
constexpr int SUMS_THREADS = 1024;
__global__ void __launch_bounds__(SUMS_THREADS) pr_sums_kernel(const float *rank, const float *inv_outdeg,
                                                               int32_t n, Ctl *ctl) {
  __shared__ double s[SUMS_THREADS / 64][2];
  double m = 0.0, dg = 0.0;
  for (int32_t v = threadIdx.x; v < n; v += SUMS_THREADS) {
    const double x = (double)rank[v];
    m += x;
    if (inv_outdeg[v] == 0.0f) dg += x;
  }
  m = wave_sum_f64(m);
  dg = wave_sum_f64(dg);
  if (threadIdx.x % 64 == 0) { s[threadIdx.x / 64][0] = m; s[threadIdx.x / 64][1] = dg; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double tm = 0.0, td = 0.0;
    for (int w = 0; w < SUMS_THREADS / 64; ++w) { tm += s[w][0]; td += s[w][1]; }
    ctl->mass = tm;
    ctl->dangling = td;
  }
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

__global__ void init_stripes_kernel(Stripe *s) {
  const int i = threadIdx.x;
  if (i < NSTRIPE) {
    Stripe z;
    z.ca = z.sm = z.edges = z.l1 = z.dd = z.dm = z.narrow = 0ull;
    for (int k = 0; k < 4; ++k) z.hist[k] = 0ull;
    z.min_changed = INF;
    s[i] = z;
  }
}

__global__ void init_ctl_kernel(Ctl *ctl, Ctl init) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *ctl = init;
}

// The host's density switch (Section 3.1) under weak prediction: the next
// pass is a verification pass (prediction off), so every vertex is pulled
// once before the sparse stage takes over.
__global__ void set_phase_kernel(Ctl *ctl, uint32_t phase) {
  if (threadIdx.x == 0 && blockIdx.x == 0 && !ctl->done) ctl->phase = phase;
}

}  // namespace

template <int ALGO>
static void launch_pair(const SweepArgs &a, hipStream_t s, hipEvent_t mid) {
  constexpr int EPT = TILE_E / BLOCK;
  // split-width images serve only the min programs, and their wide edge
  // words are always packed
  constexpr bool CAN_SPLIT = ALGO == A_BFS || ALGO == A_SSSP || ALGO == A_CC;
  constexpr bool PR = ALGO == A_PR || ALGO == A_PPR;
  if (PR && a.det) {
    if (a.packed) hipLaunchKernelGGL((sweep_kernel<ALGO, EPT, true, false, PR>), dim3(a.nblocks), dim3(BLOCK), 0, s, a);
    else hipLaunchKernelGGL((sweep_kernel<ALGO, EPT, false, false, PR>), dim3(a.nblocks), dim3(BLOCK), 0, s, a);
    if (mid) (void)hipEventRecord(mid, s);
    hipLaunchKernelGGL(close_kernel<ALGO>, dim3(1), dim3(CLOSE_THREADS), 0, s, a);
    if (a.nent > 0) hipLaunchKernelGGL(det_commit_kernel, dim3(64, a.nent), dim3(BLOCK), 0, s, a);
    return;
  }
  // (images of unweighted graphs hold 3-byte wide ids)
  constexpr bool CAN_W3 = ALGO == A_BFS || ALGO == A_CC;
  if (CAN_W3 && a.split && a.packed && a.wide3) {
    hipLaunchKernelGGL((sweep_kernel<ALGO, EPT, true, CAN_SPLIT, false, CAN_W3>), dim3(a.nblocks), dim3(BLOCK), 0, s, a);
  } else if (CAN_SPLIT && a.split && a.packed) {
    hipLaunchKernelGGL((sweep_kernel<ALGO, EPT, true, CAN_SPLIT>), dim3(a.nblocks), dim3(BLOCK), 0, s, a);
  } else if (a.packed) {
    hipLaunchKernelGGL((sweep_kernel<ALGO, EPT, true, false>), dim3(a.nblocks), dim3(BLOCK), 0, s, a);
  } else {
    hipLaunchKernelGGL((sweep_kernel<ALGO, EPT, false, false>), dim3(a.nblocks), dim3(BLOCK), 0, s, a);
  }
  if (mid) (void)hipEventRecord(mid, s);
  hipLaunchKernelGGL(close_kernel<ALGO>, dim3(1), dim3(CLOSE_THREADS), 0, s, a);
}

hipError_t launch_sweep(int algo, const SweepArgs &a, hipStream_t s, hipEvent_t mid) {
  if (a.nblocks <= 0) return hipErrorInvalidValue;
  switch (algo) {
    case A_BFS: launch_pair<A_BFS>(a, s, mid); break;
    case A_SSSP: launch_pair<A_SSSP>(a, s, mid); break;
    case A_CC: launch_pair<A_CC>(a, s, mid); break;
    case A_PR: launch_pair<A_PR>(a, s, mid); break;
    case A_PPR: launch_pair<A_PPR>(a, s, mid); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_open_list(const uint32_t *value, const uint32_t *has_in, int32_t n, const Ctl *ctl,
                            uint32_t *list, uint32_t cap, uint32_t *count, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(open_list_kernel, dim3((n + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, s, value, has_in, n, ctl,
                     list, cap, count);
  return hipGetLastError();
}

hipError_t launch_open_guess(const uint32_t *value, const uint32_t *has_in, int32_t v_limit, const Ctl *ctl,
                             uint32_t *count, hipStream_t s) {
  if (v_limit <= 0) return hipSuccess;
  hipLaunchKernelGGL(open_guess_kernel, dim3((v_limit + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, s, value, has_in,
                     v_limit, ctl, count);
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

hipError_t launch_gather_probe(const uint32_t *src, int64_t m, uint32_t mask, const uint32_t *val, int32_t n,
                               unsigned long long *sink, hipStream_t s) {
  const int64_t blocks = (m + TILE_E - 1) / TILE_E;
  if (m < 1 || n < 1 || blocks > 0x7FFFFFFF) return hipErrorInvalidValue;
  hipLaunchKernelGGL(gather_probe_kernel, dim3((unsigned)blocks), dim3(BLOCK), 0, s, src, m, mask, val, n, sink);
  return hipGetLastError();
}

hipError_t launch_pr_sums(const float *rank, const float *inv_outdeg, int32_t n, Ctl *ctl, hipStream_t s) {
  hipLaunchKernelGGL(pr_sums_kernel, dim3(1), dim3(SUMS_THREADS), 0, s, rank, inv_outdeg, n, ctl);
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

hipError_t launch_init_stripes(Stripe *s, hipStream_t st) {
  hipLaunchKernelGGL(init_stripes_kernel, dim3(1), dim3(NSTRIPE), 0, st, s);
  return hipGetLastError();
}

hipError_t launch_init_prd(float *rank, float *resid, float *contrib, float *contrib_next, int32_t n,
                           int32_t seed, double damping, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(init_prd_kernel, dim3((n + 255) / 256), dim3(256), 0, s, rank, resid, contrib, contrib_next,
                     n, seed, damping);
  return hipGetLastError();
}

hipError_t launch_rank_terms(const float *rank, float *contrib, const float *inv_outdeg, int32_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(rank_terms_kernel, dim3((n + 255) / 256), dim3(256), 0, s, rank, contrib, inv_outdeg, n);
  return hipGetLastError();
}

hipError_t launch_set_phase(Ctl *ctl, uint32_t phase, hipStream_t s) {
  hipLaunchKernelGGL(set_phase_kernel, dim3(1), dim3(64), 0, s, ctl, phase);
  return hipGetLastError();
}

hipError_t launch_init_ctl(Ctl *ctl, const Ctl &init, hipStream_t s) {
  hipLaunchKernelGGL(init_ctl_kernel, dim3(1), dim3(64), 0, s, ctl, init);
  return hipGetLastError();
}

// Per-run scratch of the allocation-free solve: the control block and the
// counter stripes, in a static array every device holds from library load
// to process end. Host code never passes the array's name to a kernel (on
// the host it is only a stand-in for the symbol): it takes the device
// address hipGetSymbolAddress gives, once per device, with that device
// current, and hands that address to the kernels.
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];
static_assert(sizeof(Ctl) <= NOALLOC_CTL_BYTES, "control block fits its scratch section");
static_assert(NOALLOC_CTL_BYTES + sizeof(Stripe) * NSTRIPE <= NOALLOC_SCRATCH_BYTES,
              "control block and stripes fit the scratch array");

hipError_t noalloc_scratch(int device, void **out) {
  static std::mutex mu;
  static std::vector<void *> ptr;  // per device, null until looked up
  std::lock_guard<std::mutex> lk(mu);
  if (device < 0) return hipErrorInvalidDevice;
  if ((size_t)device >= ptr.size()) ptr.resize((size_t)device + 1, nullptr);
  if (!ptr[device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    ptr[device] = p;
  }
  *out = ptr[device];
  return hipSuccess;
}

}  // namespace sr
