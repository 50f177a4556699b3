// engine.hpp -- host-side objects behind the C ABI handles.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/seraph.h"
#include "common.hpp"
#include "kernels.hpp"

namespace sr {

// Pinned host page buffer (Section 3.1 CSC page) plus a copy of its header.
struct Page {
  char *host = nullptr;     // pinned (device context) or aligned malloc (host-only)
  uint64_t bytes = 0;
  PageHeader hdr{};
  // split-width image for streamed min programs (built on first use)
  char *split = nullptr;
  int64_t narrow = -1;      // in-edges from sources below NARROW_LIMIT (-1: not counted yet)
  uint64_t split_bytes = 0; // size of its split-width image (valid once narrow is counted)
  uint64_t split_est = 0;   // page 0 only: sampled estimate of all images' size (0: none yet)
  PageHeader shdr{};
};

// Per-run device state; kept after a run so values can be read back and a
// later run can resume from them.
struct RunState {
  int algo = -1;
  int32_t n = 0;
  uint32_t *value = nullptr;
  float *contrib = nullptr;
  float *contrib_next = nullptr;  // deterministic PageRank / PageRank-delta (allocated on first use)
  float *resid = nullptr;         // PageRank-delta residuals (allocated on first use)
  float *inv_outdeg = nullptr;
  uint8_t *status = nullptr;
  Ctl *ctl = nullptr;
  Stripe *stripes = nullptr;  // NSTRIPE sweep counter stripes
  uint32_t *frontier = nullptr;  // vertices changed in a pass (host sparse stage)
  uint32_t *fr_count = nullptr;
  uint32_t fr_cap = 0;
  uint32_t *has_in = nullptr;    // one bit per vertex with an in-edge (the host stage's open list)
  bool valid = false;
};

// Device residency of the pages: either all pages resident, or num_slots
// slot buffers the pages stream through.
struct Residency {
  bool resident = false;
  bool weights = false;            // page prefix with weights copied
  bool bins = false;               // page prefix with the bin lists copied
  int32_t nslots = 0;
  uint64_t slot_bytes = 0;
  std::vector<char *> buf;         // resident: one per page; streaming: one per slot
  std::vector<unsigned long long *> partial;  // heavy-vertex accumulators, same indexing as buf
  std::vector<uint64_t> partial_words;        // 64-bit words of each accumulator buffer
  std::vector<int32_t> slot_page;  // streaming: page currently in slot (-1 none)
  uint32_t max_chunks = 0;
};

}  // namespace sr

struct sr_ctx {
  int device = -1;
  bool host_only = true;
  uint64_t budget = 0;
  uint64_t used = 0;
  mutable std::string err;
  hipStream_t own_compute = nullptr, own_copy = nullptr;
  hipStream_t compute = nullptr, copy = nullptr;
  // one entry per live device allocation: its charged size and, when it
  // came from the caller's allocator, how to give it back
  struct Alloc {
    uint64_t bytes = 0;
    sr_release_fn release = nullptr;  // null: hipMalloc'd
    void *user = nullptr;
  };
  std::unordered_map<void *, Alloc> allocs;
  // caller-provided device allocator (sr_ctx_set_allocator), null = hipMalloc
  sr_alloc_fn hook_alloc = nullptr;
  sr_release_fn hook_release = nullptr;
  void *hook_user = nullptr;
  // host-mapped per-sweep record ring
  sr::SweepRecord *ring_host = nullptr;
  sr::SweepRecord *ring_dev = nullptr;
  uint32_t ring_mask = 0;
  // device address of the allocation-free solve's static scratch array
  // (null on a host-only context, or if the lookup failed)
  void *scratch_dev = nullptr;
  std::mutex mu;

  sr_status fail(sr_status st, const std::string &msg) const {
    err = msg;
    return st;
  }
  sr_status hip_fail(hipError_t e, const char *what) const {
    err = std::string(what) + ": " + hipGetErrorString(e);
    return SR_EDEVICE;
  }
  // budgeted device allocation
  sr_status dalloc(void **p, uint64_t bytes, const char *what);
  void dfree(void *p);
};

struct sr_graph {
  sr_ctx *ctx = nullptr;
  int32_t n = 0;
  int64_t m = 0;
  bool weighted = false, symmetric = false;
  bool packed = false;  // weights < 256 and n <= 2^24: pages store source | weight << 24
  // SR_LOAD_REORDER: internal ids by descending degree; rank maps the
  // caller's ids to internal ones, perm the other way (both empty otherwise)
  bool reordered = false;
  std::vector<int32_t> rank, perm;
  std::vector<int64_t> in_off;
  std::vector<int32_t> in_src;
  std::vector<uint32_t> in_w;
  std::vector<int32_t> outdeg;
  int32_t nparts = 0, nslots = 0;
  bool auto_parts = false;
  bool equal_edges = false;  // pages cut by in-edge count (SR_PART_EQUAL_EDGES)
  std::vector<sr::Page> pages;
  sr::Residency res;
  sr::RunState state;
  int server_refs = 0;  // servers holding the resident pages (no re-residency meanwhile)
  std::vector<sr_sweep_record> sweeps;  // per-sweep trace of the last run
  // out-edge CSR for the host sparse stage (built on first use)
  bool out_built = false;
  std::vector<int64_t> out_off;
  std::vector<int32_t> out_dst;
  std::vector<uint32_t> out_w;
  // per vertex, the pages its out-edges enter (bit page * 64 / P), for
  // SR_RUN_SKIP_CLEAN; built for the partition with out_mask_parts pages
  std::vector<uint64_t> out_mask;
  int32_t out_mask_parts = 0;
  // host sparse stage: pinned mirror of the value array (n words, so both
  // transfers run at the pinned copy rate) and the per-vertex queue flags,
  // which are all zero between calls
  uint32_t *host_val = nullptr;
  int32_t *perm_pinned = nullptr;  // perm in pinned memory: CC's first labels, copied with no staging
  std::vector<uint8_t> push_inq;
};

namespace sr {
// graph_host.cpp
sr_status build_in_csr(sr_graph *g, const int64_t *row_offsets, const int32_t *col_idx,
                       const uint32_t *weights, bool symmetrize);
void relabel_by_degree(int32_t n, const int64_t *ro, const int32_t *ci, const uint32_t *wi, bool symmetrize,
                       std::vector<int32_t> &rank, std::vector<int32_t> &perm, std::vector<int64_t> &ro2,
                       std::vector<int32_t> &ci2, std::vector<uint32_t> &w2);
// equal_edges: boundaries by in-edge count instead of streamed bytes
sr_status make_pages(sr_graph *g, int32_t nparts, bool equal_edges = false);
// split-width images of every page (PageHeader::split), for streamed min
// programs; built once per partition
bool split_eligible(const sr_graph *g);
// counts each page's narrow in-edges (once per partition) and sets the
// sizes its split-width image would have, without building it
void size_split_pages(sr_graph *g);
// total size of the split-width images estimated from every 1024th in-edge
// (a few MB read instead of the whole in-edge array)
uint64_t estimate_split_bytes(const sr_graph *g);
sr_status build_split_pages(sr_graph *g);
// Smallest page count whose largest streamed page (with its chunk scratch)
// fits slot_bytes; -1 if none does.
int32_t auto_parts(const sr_graph *g, uint64_t slot_bytes, bool equal_edges = false);
void free_pages(sr_graph *g);
uint64_t graph_bytes(const sr_graph *g);
int host_threads();
// sparse.cpp
void build_out_csr(sr_graph *g);
void build_out_masks(sr_graph *g);
// OR of the out-page masks of the frontier's vertices
uint64_t frontier_pages(const sr_graph *g, const uint32_t *front, int64_t nf);
// push from a frontier to the fixed point, or until a round's list exceeds
// limit (> 0): then *rest receives that list and the caller resumes on the
// device; returns the edges relaxed
int64_t sparse_push(sr_graph *g, int algo, uint32_t *val, const uint32_t *front, int64_t nf,
                    int32_t *rounds, int64_t limit = 0, std::vector<uint32_t> *rest = nullptr);
// push from a frontier over values the host holds only in part: `known`
// maps vertices to their values; before each round `fetch(need, got)` is
// asked for the values of the round's vertices and out-neighbours missing
// from `known` and may refuse (returns false). Returns false, with nothing
// written to the device, when a fetch is refused, `known` would pass cap
// entries or a round's list exceeds limit (> 0); else true, with *lowered
// listing every vertex whose value decreased (its new value in `known`),
// *rounds and *relaxed set
bool sparse_push_partial(sr_graph *g, int algo, std::unordered_map<uint32_t, uint32_t> &known,
                         const std::vector<uint32_t> &front, int64_t limit, size_t cap,
                         const std::function<bool(const std::vector<uint32_t> &, std::vector<uint32_t> &)> &fetch,
                         std::vector<uint32_t> *lowered, int32_t *rounds, int64_t *relaxed);
// stage.hip: dst[i] = src[idx[i]] for i < count (device buffers)
hipError_t launch_gather_u32(const uint32_t *src, const uint32_t *idx, uint32_t count, uint32_t *dst,
                             hipStream_t s);
// stage.hip: dst[idx[i]] = vals[i] for i < count (device buffers, distinct idx)
hipError_t launch_scatter_u32(uint32_t *dst, const uint32_t *idx, const uint32_t *vals, uint32_t count,
                              hipStream_t s);
// one Jacobi pull over the listed vertices' in-edges; *changed receives the
// vertices whose value decreased; returns the edges read
int64_t sparse_pull(sr_graph *g, int algo, uint32_t *val, const uint32_t *list, int64_t nl,
                    std::vector<uint32_t> *changed);
// engine.cpp
// min_slot: streaming slots hold at least this many bytes (forced split-width images)
sr_status ensure_residency(sr_graph *g, bool weights, bool force_stream, bool bins = false,
                           uint64_t min_slot = 0);
void release_residency(sr_graph *g);
}  // namespace sr
