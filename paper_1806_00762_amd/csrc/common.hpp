// common.hpp -- internal layout shared by the host runtime and the gfx950
// kernels of libseraph: page buffer format, degree bins, sweep control
// block, per-sweep records. Not part of the public ABI (include/seraph.h).
#pragma once

#include <cstddef>
#include <cstdint>

namespace sr {

constexpr uint32_t INF = 0xFFFFFFFFu;
constexpr uint32_t PAGE_MAGIC = 0x53525047u;  // "SRPG"

// Degree bins of a page (Section 3.1 pages, load-balanced for wave64).
// A vertex with in-degree d >= 1 goes to
//   bin b in [0, 5]  if 2^b <= d < 2^(b+1): a group of 2^b lanes, <= 2 edges per lane
//   bin 6            if 64 <= d <= HEAVY: one wavefront per vertex
//   bin 7            if d > HEAVY: split into CHUNK-edge chunks, one wavefront
//                    per chunk, partial results combined by the last chunk
//   bin 8            if d = 0: a pull can never change a min program's value
//                    there, so only PageRank (whose value also depends on the
//                    dangling mass) visits this bin.
constexpr int NBINS = 9;
constexpr int BIN_WAVE = 6;
constexpr int BIN_CHUNK = 7;
constexpr int BIN_ZERO = 8;
constexpr int HEAVY = 2048;
constexpr int CHUNK = 2048;

constexpr int BLOCK = 256;        // threads per workgroup (4 wavefronts)
constexpr int WAVES = BLOCK / 64;

// Tiles of the single-instance sweep: runs of consecutive non-heavy
// vertices with at most TILE_V vertices and TILE_E in-edges, one block
// each (16 edges per thread, so 16 gathers per thread are in flight).
constexpr int TILE_V = 2 * BLOCK;
constexpr int TILE_E = 16 * BLOCK;

// vertices per block for bins 0..6 and chunks per block for bin 7
constexpr int SMALL_ROUNDS = 4;   // vertices per lane group in bins 0..5
constexpr int WAVE_ROUNDS = 2;    // vertices per wavefront in bin 6
__host__ __device__ constexpr int bin_items_per_block(int b) {
  return b < BIN_WAVE ? (BLOCK >> b) * SMALL_ROUNDS
                      : (b == BIN_WAVE ? WAVES * WAVE_ROUNDS : (b == BIN_CHUNK ? WAVES : BLOCK * 4));
}

// A heavy-vertex chunk: edges [e_begin, e_end) of local vertex vl; `first`
// is the index (in the page's chunk list) of the vertex's first chunk and
// `count` its number of chunks.
struct Chunk {
  int32_t vl;
  int32_t e_begin, e_end;
  int32_t first_count;  // first | (count << 20), as uint32: first < 2^20, count < 2^12
};

// A heavy vertex (bin 7): local id and its chunk range, packed like Chunk.
struct Heavy {
  int32_t vl;
  int32_t first_count;
};

// Per-block sweep counters, written with plain stores by every block of a
// sweep and reduced by the close kernel after the sweep has finished.
// Sweep counters: every block of a sweep adds its totals with device-scope
// atomics into one of NSTRIPE stripes (block id modulo NSTRIPE), so no block
// waits on another and no fence is needed; the close kernel reads each
// stripe back and resets it with atomic exchanges. Floating sums travel as
// fixed point (FIX_ONE = 2^54) so they add exactly and in any order.
constexpr int NSTRIPE = 64;
constexpr double FIX_ONE = 18014398509481984.0;  // 2^54
struct alignas(128) Stripe {
  unsigned long long ca;       // changed | attempted << 32
  unsigned long long sm;       // skipped | mispred << 32
  unsigned long long edges;
  unsigned long long l1;       // PageRank: sum |delta|, fixed point
  unsigned long long dd;       // PageRank: dangling-mass change, two's complement fixed point
  unsigned long long dm;       // PageRank: change of the rank sum (mass), two's complement fixed point
  unsigned long long narrow;   // split images: scanned edges read from the narrow section
  unsigned long long hist[4];  // weak predictor states, two 32-bit counts per word
  uint32_t min_changed;        // smallest new value among changed vertices (min programs)
};
static_assert(sizeof(Stripe) == 128, "one stripe per 128-byte line");

// First 256 bytes of every page buffer. Section offsets are in bytes from
// the buffer start, all multiples of 256. Sections are ordered so that each
// use copies a prefix: header, tiles, chunks, heavy list, sources, offsets
// (unweighted programs stop here; a min program that reads no separate
// weights stops at bytes_lead, inside the offsets), weights (single-instance
// sweeps stop here), degree-bin lists (multi-instance sweeps).
constexpr uint32_t PACKED_SRC_MASK = 0x00FFFFFFu;  // source id bits of a packed edge word
struct alignas(256) PageHeader {
  uint32_t magic;
  int32_t v_begin;
  int32_t n_p;
  int32_t n_chunks;
  int64_t m_p;
  uint64_t off_offsets;   // int32[n_p + 1], rebased to 0
  uint64_t off_bins;      // int32 local vertex ids, bins 0..6 and 8 back to back
  uint64_t off_chunks;    // Chunk[n_chunks]
  uint64_t off_heavy;     // Heavy[n_heavy]: the vertices of bin 7, one entry each
  uint64_t off_tiles;     // int32 pairs [v_begin, v_end) of the n_tiles tiles
  uint64_t off_src;       // u32[m_p]: global source id, or source | weight << 24 when packed
  uint64_t off_w;         // u32 weights (weighted graphs that are not packed)
  uint64_t bytes_unweighted;  // prefix a program without weights needs
  uint64_t bytes_weighted;    // prefix with weights (single-instance sweeps)
  uint64_t bytes_total;       // everything, bin lists of the multi-instance sweep included
  uint64_t bytes_lead;        // prefix a min program without weights reads (offsets up to the last
                              // vertex of a tile with in-edges or of a heavy vertex)
  int32_t bin_count[NBINS];      // bin 7: number of chunks
  int32_t bin_start[NBINS];      // start of bin b in the bins section (not bin 7)
  int32_t n_heavy;               // vertices in bin 7
  int32_t max_indeg;
  int32_t n_tiles;
  int32_t w_bytes;               // 4: separate u32 weight section; 0: none (unweighted or packed)
  int32_t tile_e;                // in-edge cap of a tile (TILE_E)
  int32_t packed;                // edge words carry the weight in their top byte
  int32_t n_tiles_edges;         // tiles with at least one in-edge; they come first in the tile list
  // Split-width image (split = 1), streamed to the min programs: each
  // vertex's in-edges from sources below 2^16 ("narrow": a u16 id and, for
  // weighted graphs, a u8 weight) come apart from the others ("wide": the
  // usual edge words, at off_src); a vertex's narrow edges precede its
  // wide ones. The image has no offsets: a tile with in-edges has a base
  // (int2: its first vertex's in-edges before it, and its narrow edges
  // before it), and each of its vertices a u32 of its narrow and wide edge
  // ends relative to the tile's bases (low and high 16 bits; a tile holds at
  // most TILE_E edges). The entry of a heavy vertex is its index in the
  // heavy table (int4: in-edges before it, narrow edges before it, narrow
  // edges, in-degree). The wide edges before a vertex with e in-edges and n
  // narrow edges before it are e - n.
  // Layout: header | tiles | chunks | heavy | tile bases | heavy table |
  // vertex entries | narrow ids | wide words | narrow weights (off_w), the
  // entries up to the last vertex the min programs read; bytes_lead is the
  // whole image.
  int32_t split;
  int32_t wide3;                 // unweighted graphs: the wide in-edges are 3-byte ids back to back
                                 // (little-endian; 8 bytes of padding after the last)
  uint64_t off_vpk;              // u32 per vertex (see above)
  uint64_t off_hsrc;             // u16 narrow source ids
  uint64_t off_tbase;            // int2 per tile with in-edges
  uint64_t off_hside;            // int4 per heavy vertex
};
static_assert(sizeof(PageHeader) == 256, "page header is one 256-byte line");
constexpr uint32_t NARROW_LIMIT = 1u << 16;  // narrow source ids are below this

enum Algo : int32_t { A_BFS = 0, A_SSSP = 1, A_CC = 2, A_PR = 3, A_PPR = 4 };
enum Pvu : int32_t { P_OFF = 0, P_STRONG = 1, P_WEAK = 2 };

// Weak predictor diagram in device-friendly form.
struct Diagram {
  uint32_t num_states, initial, attempt_mask, pad;
  uint8_t succ[8], fail[8];
};

// Per-sweep host-visible record (written by the last block of each sweep
// into a pinned, device-mapped ring).
struct alignas(16) SweepRecord {
  uint64_t seq;
  uint64_t changed;
  uint64_t edges;
  uint64_t attempted;
  uint64_t skipped;
  uint64_t mispred;
  double l1;
  uint32_t min_changed;
  uint32_t threshold;     // strong threshold this sweep used
  uint32_t phase;         // 0 normal, 1 verification
  uint32_t done_after;    // control state after this sweep's end-of-pass step
  uint32_t pass_after;
  uint32_t stop_reason;
  uint64_t hist[8];
  double dangling;        // PageRank dangling mass after the sweep
  double pass_l1_closed;  // L1 of the pass closed by this sweep (if any)
  uint64_t edges_narrow;  // scanned edges read from the narrow section of split images
  uint32_t phase_after;   // phase of the next sweep (after this sweep's end-of-pass step)
  uint32_t pad_;
};
static_assert(sizeof(SweepRecord) % 16 == 0, "record copied in 16-byte words");

// Device-resident control block of one run. The sweeps and the end-of-pass
// step read and update it, so a whole resident solve can be enqueued (or
// captured) without host round trips.
struct Ctl {
  // current pass configuration
  uint32_t threshold;     // strong: skip vertices with value <= threshold
  uint32_t phase;         // 1 = verification pass (prediction off)
  uint32_t done;          // converged or stopped: sweeps become no-ops
  uint32_t pass;          // passes completed
  uint32_t stop_reason;
  uint32_t sweep_seq;
  uint32_t no_improve;
  uint32_t delta;         // PageRank-delta: the residual-propagation phase is on
  // current pass accumulators
  unsigned long long pass_changed;
  uint32_t pass_min_changed;
  uint32_t win_quiet;     // the last sweep changed nothing (later sweeps of its window may exit at once)
  double pass_l1;
  double best_l1;
  double dangling;        // PageRank: D used by the sweeps (sum of the dangling ranks)
  double mass;            // PageRank: sum of all ranks; a sweep scales its update by 1 / mass
  double dangling_next;   // PageRank-delta: residual mass sent by dangling vertices in this pass
  // run constants
  int32_t algo, pvu, max_passes, pad2;
  double tol_l1;
  double floor_cap;
};
static_assert(sizeof(Ctl) % 4 == 0, "the control block is copied as 32-bit words");

}  // namespace sr
