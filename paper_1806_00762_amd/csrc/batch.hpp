// batch.hpp -- multi-instance sweeps: K instances of one vertex program on
// one resident graph share every in-edge read; values are laid out
// [vertex][K] so the gather of one neighbour serves all K instances with one
// contiguous 4K-byte access. Used by sr_batch_run and by the query server.
#pragma once
#include <hip/hip_runtime.h>

#include "common.hpp"

namespace sr {

// instances of one plan (their counters live in LDS during a sweep)
constexpr int MI_MAX_INSTANCES = 1024;
// consecutive heavy vertices per thread of the heavy-vertex kernel
constexpr int MI_HEAVY_RUN = 8;

// Per-instance control (device memory), one per column of a group.
struct MiInst {
  uint32_t active;       // 1 = running this sweep
  uint32_t unit;         // min programs: 1 = BFS (unit weights), 0 = SSSP
  int32_t source;        // SSSP/BFS source or PPR seed
  uint32_t threshold;    // strong predictor threshold (min programs)
  uint32_t sweeps;       // sweeps done since admission
  uint32_t done;         // converged
  uint32_t stop_reason;
  uint32_t no_improve;
  // accumulators of the current sweep
  uint32_t sw_changed;
  uint32_t sw_min_changed;
  unsigned long long sw_edges;
  double sw_l1;
  double sw_ddelta;
  double sw_dmass;
  // PageRank state
  double dangling;
  double mass;           // sum of the column's ranks (updates are scaled by 1 / mass)
  double best_l1;
  double last_l1;
  unsigned long long edges_total;
  uint32_t overflow;     // 16-bit columns: a candidate did not fit (the host completes the column)
  uint32_t pad;
};

// One group: K columns over one graph.
struct MiGroup {
  uint32_t *value;          // [n][K] u32 distances/levels, or f32 ranks
  float *contrib;           // [n][K] PPR only
  const float *inv_outdeg;  // [n] PPR only
  MiInst *inst;             // [K]
  int32_t n;
  int32_t pvu;              // P_OFF or P_STRONG
  int32_t has_w;            // SSSP on weighted pages (weights read only then)
  int32_t packed;           // edge words carry the weight in their top byte
  uint32_t src_mask;        // source id bits of an edge word
};

// One unit of work: a resident page of a group's graph.
struct MiUnit {
  int32_t group;
  int32_t heavy_base;       // heavy vertices of the units before this one
  const char *page;
  unsigned long long *acc;  // [n_chunks][K] heavy-vertex accumulators (at each vertex's first chunk)
  int32_t blk_prefix[NBINS + 1];  // items per bin within this unit
};

// Global control of a batched sweep (device memory).
struct MiCtl {
  uint32_t queue;           // next work item (persistent grid)
  uint32_t pad;
  uint32_t remaining;       // instances still active after the last sweep
  uint32_t sweeps;
};

struct MiArgs {
  const MiGroup *groups;
  const MiUnit *units;
  const int32_t *unit_prefix;  // [nunits + 1] items
  int32_t ngroups, nunits;
  int32_t total_items;
  int32_t total_heavy;      // heavy vertices over all units
  int32_t heavy_blocks;     // blocks of the heavy-vertex kernel
  int32_t grab;             // items taken per queue access
  int32_t rounds;           // vertex rounds per wavefront and item in the small-degree bins (2, 4, 8)
  int32_t narrow;           // SSSP/BFS columns stored as 16 bits (0xFFFF = unreached)
  int32_t wmode;            // edge weights of every group: 0 none (or PPR), 1 packed in the edge word,
                            // 2 separate array; 3 when the groups differ
  int32_t nblocks;
  double damping;
  double tol_l1, floor_cap;
  int32_t max_sweeps;
  int32_t tuning;           // 1: never retire instances (timing runs)
  int32_t lane_lds;         // set at launch: the sweep keeps the lanes' instance state in LDS
  int32_t descending;       // 1: the queue hands out items last to first (heavy chunks and
                            // high in-degree bins of the last unit first)
  MiCtl *ctl;
  uint32_t *group_active;   // [ngroups] active instances per group (0: group skipped)
  uint32_t *host_remaining; // host-mapped copy of ctl->remaining
};

int mi_items_per_block_host(int b, int K, int rounds);
hipError_t launch_mi_sweep(int algo, int K, const MiArgs &a, hipStream_t s);
hipError_t launch_mi_init_column(int algo, int K, uint32_t *value, float *contrib, const float *inv_outdeg,
                                 int32_t n, int32_t col, int32_t source, hipStream_t s, bool narrow = false);
// entry `index` of a 16-bit value array
hipError_t launch_mi_set_u16(uint32_t *value, size_t index, uint32_t v, hipStream_t s);
hipError_t launch_mi_set_inst(MiInst *dst, const MiInst &val, hipStream_t s);
hipError_t launch_mi_set_ctl(MiCtl *dst, const MiCtl &val, hipStream_t s);
// One serving iteration's set-up in one launch: a query admitted into a
// clean column (its source's entry set to 0, the column's record started),
// the per-group active counts and the control block's reset.
struct MiAdmit {
  int32_t group, col, source;  // source: internal vertex id
  uint32_t unit;               // 1 = BFS
};
constexpr int MI_ADMIT_MAX = 1024;
// buf (device): ngroups u32 active counts, then nadmit MiAdmit entries
hipError_t launch_mi_setup(const MiGroup *groups, const uint32_t *buf, int32_t ngroups, int32_t nadmit,
                           uint32_t remaining, MiCtl *ctl, uint32_t *group_active, int32_t K, bool narrow,
                           hipStream_t s);
// Columns to copy out of value[n][K] in one pass: out[j][v] = value[v][col[j]].
constexpr int MI_EXTRACT_MAX = 32;
struct MiExtract {
  int32_t count;
  int32_t col[MI_EXTRACT_MAX];
  uint32_t *out[MI_EXTRACT_MAX];  // device buffers of n words
};
// Copy the listed columns (row rank[v] for vertex v when rank is given:
// internal ids of a reordered graph); with reset, leave `reset_to` in them
// (so the next query on a column only sets its source).
hipError_t launch_mi_extract(int K, uint32_t *value, int32_t n, const MiExtract &x, hipStream_t s,
                             bool reset = false, uint32_t reset_to = 0u, const int32_t *rank = nullptr,
                             bool narrow = false);

}  // namespace sr
