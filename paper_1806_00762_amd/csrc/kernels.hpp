// kernels.hpp -- launch interface of the gfx950 sweep kernels (kernels.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "common.hpp"

namespace sr {

constexpr int MAXW = 16;  // pages per sweep launch
constexpr int NSEC = 2;   // work sections of a page: tiles, heavy-vertex chunks

// Arguments of one window sweep (Section 3.2: the resident pages of the
// window are swept together as one "super subgraph").
struct SweepArgs {
  int32_t nent;            // pages in this launch
  int32_t end_of_pass;     // the last block of this launch closes the pass
  int32_t n;               // vertices of the graph
  int32_t audit;           // evaluate skipped vertices too, count would-be changes
  int32_t pr_seed;         // personalized PageRank seed, -1 = uniform teleport
  int32_t nblocks;         // grid size
  int32_t packed;          // edge words carry the weight in their top byte
  int32_t early;           // BFS under strong prediction: stop at a first in-neighbour on the threshold level
  int32_t split;           // the pages in the slots are split-width images (min programs)
  int32_t wide3;           // ... of an unweighted graph: their wide in-edges are 3-byte ids
  int32_t det;             // PageRank: deterministic sweep (gathers read contrib, pulls write
                           // contrib_next, whose window ranges are copied back after the sweep)
  int32_t delta;           // PageRank-delta run: while the control block's delta phase is on, the
                           // gathers read the terms sent in the last pass (contrib) and the pulls
                           // write this pass's (contrib_next)
  int32_t win_first;       // first sweep of a window step
  int32_t win_skip;        // a sweep after the first of its window exits at once when the sweep
                           // before it changed nothing (its window is at a local fixed point)
  double damping;
  float pr_eps;
  Ctl *ctl;                // device control block
  SweepRecord *ring;       // host-mapped per-sweep records
  uint32_t ring_mask;
  uint32_t *value;         // BFS level / SSSP distance / CC label (u32), or PageRank rank (f32 bits)
  float *contrib;          // PageRank: rank / outdeg, gathered by the pull
  float *contrib_next;     // deterministic PageRank / PageRank-delta: the terms this sweep writes
  float *resid;            // PageRank-delta: residual per vertex (received, not yet applied)
  const float *inv_outdeg; // PageRank: 1 / outdeg (0 for dangling vertices)
  uint8_t *status;         // weak predictor state per vertex
  Stripe *stripes;         // NSTRIPE counter stripes (identity outside a sweep)
  int32_t collect;         // append changed vertices to the pass frontier
  uint32_t fr_cap;         // frontier capacity (entries)
  uint32_t *frontier;      // vertices changed in this pass (host sparse stage)
  uint32_t *fr_count;      // entries appended (may exceed fr_cap: then incomplete)
  Diagram dia;
  int32_t blk_prefix[MAXW * NSEC + 1];   // cumulative blocks over (page, section)
  const char *base[MAXW];                // page buffers on the device
  unsigned long long *partial[MAXW];     // heavy-vertex accumulators (at each vertex's first chunk), per page
};

// Blocks a page needs for section sec (0: one per tile, 1: WAVES chunks each).
// Tiles of zero in-degree vertices only (listed last) matter to PageRank
// alone: the min programs never pull such a vertex.
inline int sec_blocks(const PageHeader &h, int sec, bool all_tiles) {
  return sec == 0 ? (all_tiles ? h.n_tiles : h.n_tiles_edges) : (h.n_chunks + WAVES - 1) / WAVES;
}

// the sweep kernel, then the kernel that closes the sweep; `mid` (optional)
// is recorded between the two
hipError_t launch_sweep(int algo, const SweepArgs &a, hipStream_t s, hipEvent_t mid = nullptr);
hipError_t launch_end_pass(Ctl *ctl, SweepRecord *ring, uint32_t ring_mask, hipStream_t s);
// vertices the next pass would attempt (strong prediction): list (up to cap)
// and their number in *count (which the caller zeroes); has_in: one bit per
// vertex with an in-edge
hipError_t launch_open_list(const uint32_t *value, const uint32_t *has_in, int32_t n, const Ctl *ctl,
                            uint32_t *list, uint32_t cap, uint32_t *count, hipStream_t s);
// how many vertices below v_limit the next pass would attempt if the pass
// ended now (a guess for the copy schedule; *count zeroed by the caller)
hipError_t launch_open_guess(const uint32_t *value, const uint32_t *has_in, int32_t v_limit, const Ctl *ctl,
                             uint32_t *count, hipStream_t s);
hipError_t launch_init_min(int algo, uint32_t *value, int32_t n, int32_t source, hipStream_t s);
hipError_t launch_init_pr(float *rank, float *contrib, const float *inv_outdeg, int32_t n,
                          int32_t seed, hipStream_t s);
// gather-rate probe over m words (ids masked, clamped below n); adds the sum
// of the gathered values to *sink
hipError_t launch_gather_probe(const uint32_t *src, int64_t m, uint32_t mask, const uint32_t *val, int32_t n,
                               unsigned long long *sink, hipStream_t s);
// PageRank: sum of the ranks and of the dangling ranks into ctl->mass, ctl->dangling
hipError_t launch_pr_sums(const float *rank, const float *inv_outdeg, int32_t n, Ctl *ctl, hipStream_t s);
hipError_t launch_fill_u8(uint8_t *p, uint8_t v, size_t count, hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, size_t count, hipStream_t s);
hipError_t launch_init_stripes(Stripe *s, hipStream_t st);
hipError_t launch_init_ctl(Ctl *ctl, const Ctl &init, hipStream_t s);
// Device address of the allocation-free solve's static scratch array on
// `device` (which must be current): looked up once per device, then cached.
constexpr size_t NOALLOC_SCRATCH_BYTES = 16384;
constexpr size_t NOALLOC_CTL_BYTES = 512;  // the control block's section; the stripes follow
hipError_t noalloc_scratch(int device, void **out);
// PageRank-delta run start: rank 0, residual (1 - d) t, no terms sent yet
hipError_t launch_init_prd(float *rank, float *resid, float *contrib, float *contrib_next, int32_t n,
                           int32_t seed, double damping, hipStream_t s);
// rank-form terms contrib = rank / outdeg, when a PageRank-delta run leaves its delta phase
hipError_t launch_rank_terms(const float *rank, float *contrib, const float *inv_outdeg, int32_t n, hipStream_t s);
// set the phase of the next pass (1 = verification) unless the run is done
hipError_t launch_set_phase(Ctl *ctl, uint32_t phase, hipStream_t s);

}  // namespace sr
