// engine.cpp -- C ABI of libseraph: contexts with a device-memory budget,
// graph loading and partitioning, and the pass scheduler of Seraph
// (Section 3.2 pipelined subgraph iteration; Section 4 predictive vertex
// updating with the all-pull verification pass of Section 4.3).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <thread>

#include "engine.hpp"

using namespace sr;

namespace {

thread_local std::string g_create_err;

#define HIP_TRY(ctx, expr, what)                   \
  do {                                             \
    hipError_t e_ = (expr);                        \
    if (e_ != hipSuccess) return (ctx)->hip_fail(e_, what); \
  } while (0)

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

constexpr uint32_t RING = 4096;

}  // namespace

// ------------------------------------------------------------ allocation

sr_status sr_ctx::dalloc(void **p, uint64_t bytes, const char *what) {
  *p = nullptr;
  if (host_only) return fail(SR_EDEVICE, "host-only context has no device");
  if (bytes == 0) bytes = 256;
  bytes = (bytes + 255) & ~255ull;
  if (used + bytes > budget)
    return fail(SR_EBUDGET, std::string("device budget exceeded allocating ") + what + " (" +
                                std::to_string(bytes) + " B, used " + std::to_string(used) +
                                " of " + std::to_string(budget) + ")");
  Alloc rec;
  rec.bytes = bytes;
  if (hook_alloc) {
    void *q = hook_alloc((size_t)bytes, hook_user);
    if (!q) return fail(SR_ENOMEM, std::string("caller's allocator returned NULL for ") + what);
    if ((uintptr_t)q & 255u) {
      hook_release(q, hook_user);
      return fail(SR_EDEVICE, std::string("caller's allocator returned memory not aligned to 256 bytes for ") +
                                  what);
    }
    *p = q;
    rec.release = hook_release;
    rec.user = hook_user;
  } else {
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) { *p = nullptr; return hip_fail(e, what); }
  }
  used += bytes;
  allocs[*p] = rec;
  return SR_OK;
}

void sr_ctx::dfree(void *p) {
  if (!p) return;
  auto it = allocs.find(p);
  if (it == allocs.end()) { (void)hipFree(p); return; }
  const Alloc rec = it->second;
  used -= rec.bytes;
  allocs.erase(it);
  if (rec.release) {
    // the caller may hand the memory to other work at once: finish ours first
    (void)hipDeviceSynchronize();
    rec.release(p, rec.user);
  } else {
    (void)hipFree(p);
  }
}

// --------------------------------------------------------------- context

extern "C" sr_status sr_ctx_create(int device, uint64_t budget, sr_ctx **out) {
  if (!out) { g_create_err = "out is NULL"; return SR_EINVAL; }
  sr_ctx *c = new (std::nothrow) sr_ctx();
  if (!c) { g_create_err = "out of host memory"; return SR_ENOMEM; }
  c->device = device;
  c->host_only = device < 0;
  if (!c->host_only) {
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device >= ndev) {
      g_create_err = "no such HIP device";
      delete c;
      return SR_EDEVICE;
    }
    hipError_t e = hipSetDevice(device);
    size_t freeb = 0, totalb = 0;
    if (e == hipSuccess) e = hipMemGetInfo(&freeb, &totalb);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->own_compute, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->own_copy, hipStreamNonBlocking);
    void *ring = nullptr;
    if (e == hipSuccess) e = hipHostMalloc(&ring, sizeof(SweepRecord) * RING, hipHostMallocMapped);
    if (e != hipSuccess) {
      g_create_err = std::string("HIP init failed: ") + hipGetErrorString(e);
      if (c->own_compute) (void)hipStreamDestroy(c->own_compute);
      if (c->own_copy) (void)hipStreamDestroy(c->own_copy);
      delete c;
      return SR_EDEVICE;
    }
    c->ring_host = (SweepRecord *)ring;
    std::memset(c->ring_host, 0xFF, sizeof(SweepRecord) * RING);
    void *dptr = nullptr;
    if (hipHostGetDevicePointer(&dptr, ring, 0) != hipSuccess) dptr = ring;
    c->ring_dev = (SweepRecord *)dptr;
    c->ring_mask = RING - 1;
    // the allocation-free solve's scratch: its device address, looked up once
    // for this device (a failure only disables that entry point)
    void *scr = nullptr;
    if (sr::noalloc_scratch(device, &scr) == hipSuccess) c->scratch_dev = scr;
    c->compute = c->own_compute;
    c->copy = c->own_copy;
    c->budget = budget ? budget : (uint64_t)freeb;
  } else {
    c->budget = budget;
  }
  *out = c;
  return SR_OK;
}

extern "C" void sr_ctx_destroy(sr_ctx *c) {
  if (!c) return;
  if (!c->host_only) {
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    for (auto &kv : c->allocs) {
      if (kv.second.release) kv.second.release(kv.first, kv.second.user);
      else (void)hipFree(kv.first);
    }
    if (c->ring_host) (void)hipHostFree(c->ring_host);
    if (c->own_compute) (void)hipStreamDestroy(c->own_compute);
    if (c->own_copy) (void)hipStreamDestroy(c->own_copy);
  }
  delete c;
}

extern "C" const char *sr_ctx_last_error(const sr_ctx *c) {
  return c ? c->err.c_str() : g_create_err.c_str();
}

extern "C" sr_status sr_ctx_set_streams(sr_ctx *c, void *compute, void *copy) {
  if (!c) return SR_EINVAL;
  if (c->host_only) return c->fail(SR_EDEVICE, "host-only context has no device");
  c->compute = compute ? (hipStream_t)compute : c->own_compute;
  c->copy = copy ? (hipStream_t)copy : c->own_copy;
  return SR_OK;
}

extern "C" sr_status sr_ctx_set_allocator(sr_ctx *c, sr_alloc_fn alloc, sr_release_fn release, void *user) {
  if (!c) return SR_EINVAL;
  if (c->host_only) return c->fail(SR_EDEVICE, "host-only context has no device");
  if (alloc && !release) return c->fail(SR_EINVAL, "an allocator needs its release function");
  c->hook_alloc = alloc;
  c->hook_release = alloc ? release : nullptr;
  c->hook_user = alloc ? user : nullptr;
  return SR_OK;
}

extern "C" sr_status sr_ctx_memory(const sr_ctx *c, uint64_t *used, uint64_t *budget) {
  if (!c || !used || !budget) return SR_EINVAL;
  *used = c->used;
  *budget = c->budget;
  return SR_OK;
}

// ----------------------------------------------------------------- graph

void sr::release_residency(sr_graph *g) {
  auto &r = g->res;
  for (auto p : r.buf) g->ctx->dfree(p);
  for (auto p : r.partial) g->ctx->dfree(p);
  r = Residency();
}

static void release_state(sr_graph *g) {
  auto &s = g->state;
  g->ctx->dfree(s.value);
  g->ctx->dfree(s.contrib);
  g->ctx->dfree(s.contrib_next);
  g->ctx->dfree(s.resid);
  g->ctx->dfree(s.inv_outdeg);
  g->ctx->dfree(s.status);
  g->ctx->dfree(s.ctl);
  g->ctx->dfree(s.stripes);
  g->ctx->dfree(s.frontier);
  g->ctx->dfree(s.fr_count);
  g->ctx->dfree(s.has_in);
  s = RunState();
}

extern "C" sr_status sr_graph_load_csr(sr_ctx *c, int32_t n, int64_t m, const int64_t *ro,
                                       const int32_t *ci, const uint32_t *w, uint32_t flags,
                                       sr_graph **out) {
  if (!c) return SR_EINVAL;
  if (!out || !ro || (m > 0 && !ci)) return c->fail(SR_EINVAL, "null argument");
  if (n < 1 || m < 0) return c->fail(SR_EINVAL, "need n >= 1 and m >= 0");
  if (flags & ~(SR_LOAD_SYMMETRIZE | SR_LOAD_SYMMETRIC | SR_LOAD_REORDER))
    return c->fail(SR_EINVAL, "unknown load flags");
  if ((flags & SR_LOAD_SYMMETRIZE) && (flags & SR_LOAD_SYMMETRIC))
    return c->fail(SR_EINVAL, "SR_LOAD_SYMMETRIZE and SR_LOAD_SYMMETRIC are exclusive");
  if (ro[0] != 0 || ro[n] != m) return c->fail(SR_EINVAL, "row_offsets must start at 0 and end at m");
  for (int32_t u = 0; u < n; ++u)
    if (ro[u + 1] < ro[u]) return c->fail(SR_EINVAL, "row_offsets must be non-decreasing");
  for (int64_t e = 0; e < m; ++e)
    if (ci[e] < 0 || ci[e] >= n) return c->fail(SR_EINVAL, "col_idx out of range at " + std::to_string(e));
  if (m > INT32_MAX) return c->fail(SR_EINVAL, "m must be below 2^31");
  sr_graph *g = new (std::nothrow) sr_graph();
  if (!g) return c->fail(SR_ENOMEM, "out of host memory");
  g->ctx = c;
  g->n = n;
  g->weighted = w != nullptr;
  g->symmetric = (flags & (SR_LOAD_SYMMETRIZE | SR_LOAD_SYMMETRIC)) != 0;
  sr_status st = SR_OK;
  // relabeled copy of the input (SR_LOAD_REORDER); everything below works
  // on internal ids
  std::vector<int64_t> ro2;
  std::vector<int32_t> ci2;
  std::vector<uint32_t> w2;
  try {
    if (flags & SR_LOAD_REORDER) {
      sr::relabel_by_degree(n, ro, ci, w, (flags & SR_LOAD_SYMMETRIZE) != 0, g->rank, g->perm, ro2, ci2, w2);
      g->reordered = true;
      ro = ro2.data();
      ci = ci2.data();
      if (w) w = w2.data();
    }
    st = build_in_csr(g, ro, ci, w, (flags & SR_LOAD_SYMMETRIZE) != 0);
  } catch (const std::bad_alloc &) {
    st = c->fail(SR_ENOMEM, "out of host memory building in-edges");
  }
  if (st == SR_OK && g->weighted) {
    uint32_t mx = 0;
    for (uint32_t x : g->in_w) mx = std::max(mx, x);
    g->packed = mx <= 0xFFu && (int64_t)g->n <= (int64_t)1 << 24;  // lossless packed edge words
  }
  if (st == SR_OK && (flags & SR_LOAD_SYMMETRIC)) {
    // the transpose of a symmetric graph with sorted rows is the graph itself
    bool same = g->m == m && std::equal(g->in_off.begin(), g->in_off.end(), ro) &&
                std::equal(g->in_src.begin(), g->in_src.end(), ci) &&
                (!w || std::equal(g->in_w.begin(), g->in_w.end(), w));
    if (!same) st = c->fail(SR_EINVAL, "SR_LOAD_SYMMETRIC: input is not symmetric (or rows are not sorted)");
  }
  if (st != SR_OK) { delete g; return st; }
  *out = g;
  return SR_OK;
}

static uint64_t state_bytes(int32_t n, int algo) {
  uint64_t b = 4ull * n + 1ull * n + sizeof(Ctl) + sizeof(Stripe) * NSTRIPE + 4096;
  if (algo == A_PR || algo == A_PPR) b += 8ull * n;
  return b;
}

// bytes of the page prefix a use needs on the device
static uint64_t need_bytes(const Page &p, bool weights, bool bins = false) {
  return bins ? p.hdr.bytes_total : (weights ? p.hdr.bytes_weighted : p.hdr.bytes_unweighted);
}

static uint64_t scratch_bytes(const Page &p) {
  uint64_t c = (uint64_t)std::max<int32_t>(p.hdr.n_chunks, 1);
  return ((8 * c) + 255) & ~255ull;
}

extern "C" sr_status sr_graph_partition(sr_graph *g, int32_t nparts, int32_t nslots) {
  return sr_graph_partition_ex(g, nparts, nslots, 0u);
}

extern "C" sr_status sr_graph_partition_ex(sr_graph *g, int32_t nparts, int32_t nslots, uint32_t flags) {
  if (!g) return SR_EINVAL;
  sr_ctx *c = g->ctx;
  if (flags & ~SR_PART_EQUAL_EDGES) return c->fail(SR_EINVAL, "unknown partition flags");
  const bool eq = (flags & SR_PART_EQUAL_EDGES) != 0;
  if (nparts < 0) return c->fail(SR_EINVAL, "num_parts must be >= 0");
  if (nslots == 0) nslots = 4;
  if (nslots < 2 || nslots > MAXW + 1) return c->fail(SR_EINVAL, "num_slots must be in [2, 17]");
  if (g->server_refs > 0) return c->fail(SR_EBUSY, "graph is attached to a server");
  if (g->ctx->host_only == false) { (void)hipSetDevice(c->device); (void)hipDeviceSynchronize(); }
  release_residency(g);
  g->nslots = nslots;
  g->auto_parts = nparts == 0;
  if (nparts == 0) {
    // smallest part count whose largest page (with weights) fits one slot
    // of the budget left after the vertex state of a min program
    uint64_t st = state_bytes(g->n, A_SSSP);
    if (c->budget <= st) return c->fail(SR_EBUDGET, "budget cannot hold the vertex state");
    const uint64_t slot = (c->budget - st) / (uint64_t)nslots - 4096;
    const int32_t P = sr::auto_parts(g, slot, eq);
    if (P < 1) return c->fail(SR_EBUDGET, "no partition fits the budget");
    return sr::make_pages(g, P, eq);
  }
  return sr::make_pages(g, nparts, eq);
}

extern "C" sr_status sr_graph_info_get(const sr_graph *g, sr_graph_info *o) {
  if (!g || !o) return SR_EINVAL;
  std::memset(o, 0, sizeof(*o));
  o->n = g->n;
  o->m = g->m;
  o->weighted = g->weighted;
  o->symmetric = g->symmetric;
  o->num_parts = (int32_t)g->pages.size();
  o->num_slots = g->nslots;
  o->graph_bytes = graph_bytes(g);
  for (auto &p : g->pages) {
    o->page_bytes_total += p.bytes;
    o->max_page_bytes = std::max(o->max_page_bytes, p.bytes);
  }
  o->resident = g->res.resident;
  o->reordered = g->reordered ? 1 : 0;
  return SR_OK;
}

extern "C" sr_status sr_graph_order(const sr_graph *g, int32_t *internal_of, int32_t *caller_of) {
  if (!g) return SR_EINVAL;
  if (!g->reordered) return g->ctx->fail(SR_ESTATE, "graph was loaded without SR_LOAD_REORDER");
  if (internal_of) std::memcpy(internal_of, g->rank.data(), 4ull * g->n);
  if (caller_of) std::memcpy(caller_of, g->perm.data(), 4ull * g->n);
  return SR_OK;
}

extern "C" sr_status sr_graph_page(const sr_graph *g, int32_t page, sr_page_view *o) {
  if (!g || !o) return SR_EINVAL;
  if (page < 0 || page >= (int32_t)g->pages.size()) return g->ctx->fail(SR_EINVAL, "page out of range");
  const Page &p = g->pages[page];
  o->v_begin = p.hdr.v_begin;
  o->v_end = p.hdr.v_begin + p.hdr.n_p;
  o->num_edges = p.hdr.m_p;
  o->offsets = (const int32_t *)(p.host + p.hdr.off_offsets);
  o->src = (const uint32_t *)(p.host + p.hdr.off_src);
  o->weights = p.hdr.w_bytes == 4 ? (const uint32_t *)(p.host + p.hdr.off_w) : nullptr;
  o->src_packed = p.hdr.packed;
  o->bytes = p.bytes;
  o->stream_bytes = p.hdr.bytes_weighted;
  return SR_OK;
}

extern "C" void sr_graph_destroy(sr_graph *g) {
  if (!g || g->server_refs > 0) return;  // destroy the server first
  if (!g->ctx->host_only) {
    (void)hipSetDevice(g->ctx->device);
    (void)hipDeviceSynchronize();
    release_residency(g);
    release_state(g);
    if (g->host_val) (void)hipHostFree(g->host_val);
    if (g->perm_pinned) (void)hipHostFree(g->perm_pinned);
  }
  sr::free_pages(g);
  delete g;
}

extern "C" sr_status sr_pvu_default_diagram(sr_pvu_diagram *d) {
  if (!d) return SR_EINVAL;
  std::memset(d, 0, sizeof(*d));
  d->num_states = 6;
  d->initial_state = 0;
  d->attempt_mask = (1u << 0) | (1u << 1) | (1u << 5);
  const uint8_t succ[8] = {0, 0, 1, 2, 3, 0, 0, 0};
  const uint8_t fail[8] = {5, 4, 1, 2, 3, 3, 0, 0};
  std::memcpy(d->on_success, succ, 8);
  std::memcpy(d->on_fail, fail, 8);
  return SR_OK;
}

// ------------------------------------------------------------------- run

namespace {

struct Launch {
  SweepArgs a;
  int algo;
};

// Algorithmic bytes of one sweep: per visited vertex its offset and the
// gate's value read (weak prediction: status read and write); per scanned
// in-edge the edge word, a separate u32 weight when the page is not packed
// (SSSP), and the gathered value; per changed vertex the value write;
// PageRank also writes rank and contrib and reads 1/outdeg per attempted
// vertex. On split-width pages an edge read from the narrow section costs
// its u16 id (and the u8 weight for SSSP) instead of the u32 word, and on
// the images of unweighted graphs a wide edge its 3-byte id (a visited
// vertex reads its packed tile-relative ends in place of its offset).
uint64_t algo_bytes(int algo, int pvu, bool sep_weights, bool split, bool wide3, const SweepRecord &r) {
  const uint64_t visited = r.attempted + r.skipped;
  const uint64_t eb = (algo == A_SSSP && sep_weights) ? 12 : 8;
  uint64_t b = r.edges * eb + visited * 8;
  if (split) b -= r.edges_narrow * (algo == A_SSSP ? 1 : 2);
  if (split && wide3) b -= r.edges - r.edges_narrow;
  if (pvu == P_WEAK) b += visited * 2;
  if (algo == A_PR || algo == A_PPR) b += r.attempted * 12;
  else b += r.changed * 4;
  return b;
}

// Validate a diagram: states < 8, every transition in range, and from every
// state some attempting state is reachable via on_fail steps.
bool valid_diagram(const sr_pvu_diagram &d) {
  if (d.num_states < 1 || d.num_states > 8 || d.initial_state >= d.num_states) return false;
  for (int i = 0; i < d.num_states; ++i)
    if (d.on_success[i] >= d.num_states || d.on_fail[i] >= d.num_states) return false;
  for (int i = 0; i < d.num_states; ++i) {
    int s = i;
    bool ok = false;
    for (int k = 0; k <= d.num_states; ++k) {
      if ((d.attempt_mask >> s) & 1) { ok = true; break; }
      s = d.on_fail[s];
    }
    if (!ok) return false;
  }
  return true;
}

struct Runner {
  sr_graph *g;
  sr_ctx *c;
  RunState *rs = nullptr;  // device state the sweeps use (null: the graph's own)
  bool timed = true;       // record HIP events around each sweep
  int algo, pvu;
  bool det = false;    // deterministic PageRank sweeps
  bool delta = false;  // PageRank-delta run (residual phase first, then rank-form verification)
  bool delta_on = false;        // ... still in its residual phase
  uint32_t last_phase_after = 0;  // phase after the last closed pass
  sr_run_params prm;
  Diagram dia;
  bool weights;
  bool split = false;  // the slots receive split-width page images
  sr_run_stats st{};
  uint64_t seq_next = 0;  // next expected sweep record
  uint64_t cur_pass_changed = 0;            // vertices changed so far in the open pass
  uint64_t last_pass_changed = ~0ull;       // ... in the last closed pass
  uint32_t last_pass_phase = 0;             // phase of the last closed pass (1 = verification)
  int32_t collect = 0;                      // sweeps append changed vertices to the frontier
  // timing events: a free list, and start/end pairs not yet read
  std::vector<hipEvent_t> ev_all, ev_free;
  struct Pair { hipEvent_t a, b; bool copy; hipEvent_t mid = nullptr; };  // mid: sweep kernel end
  std::vector<Pair> pending;

  ~Runner() {
    for (auto e : ev_all) (void)hipEventDestroy(e);
  }
  hipEvent_t ev() {
    if (!ev_free.empty()) { hipEvent_t e = ev_free.back(); ev_free.pop_back(); return e; }
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    ev_all.push_back(e);
    return e;
  }
  void track(hipEvent_t a, hipEvent_t b, bool copy, hipEvent_t mid = nullptr) {
    if (a && b) pending.push_back({a, b, copy, mid});
    else { if (a) ev_free.push_back(a); if (b) ev_free.push_back(b); if (mid) ev_free.push_back(mid); }
  }
  // read the timings of completed pairs; pairs still in flight stay pending
  void harvest_events() {
    std::vector<Pair> keep;
    for (auto &p : pending) {
      if (hipEventQuery(p.b) != hipSuccess) { keep.push_back(p); continue; }
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) (p.copy ? st.h2d_ms : st.kernel_ms) += ms;
      if (p.mid && hipEventElapsedTime(&ms, p.a, p.mid) == hipSuccess) st.sweep_kernel_ms += ms;
      ev_free.push_back(p.a);
      ev_free.push_back(p.b);
      if (p.mid) ev_free.push_back(p.mid);
    }
    pending.swap(keep);
  }

  // harvest event timings and sweep records up to what the device wrote
  // (limit: read no record numbered limit or above; records written while
  // later kernels are still running may not have fully landed)
  sr_status harvest(bool *done, uint64_t limit = ~0ull) {
    harvest_events();
    for (;;) {
      if (seq_next >= limit) break;
      const SweepRecord &r = c->ring_host[seq_next & c->ring_mask];
      if (r.seq != seq_next) break;
      if (r.attempted + r.skipped > 0 || r.edges > 0) {
        st.sweeps++;
        sr_sweep_record sw;
        std::memset(&sw, 0, sizeof(sw));
        sw.pass = (int32_t)(r.pass_l1_closed >= 0.0 ? r.pass_after - 1 : r.pass_after);
        sw.phase = (int32_t)r.phase;
        sw.changed = (int64_t)r.changed;
        sw.attempted = (int64_t)r.attempted;
        sw.skipped = (int64_t)r.skipped;
        sw.edges = (int64_t)r.edges;
        for (int i = 0; i < 8; ++i) sw.state_hist[i] = (int64_t)r.hist[i];
        sw.l1 = r.l1;
        g->sweeps.push_back(sw);
      }
      st.edges_scanned += (int64_t)r.edges;
      st.vertices_attempted += (int64_t)r.attempted;
      st.vertices_skipped += (int64_t)r.skipped;
      st.mispredicted += (int64_t)r.mispred;
      for (int i = 0; i < 8; ++i) st.state_hist[i] += (int64_t)r.hist[i];
      st.algo_bytes += algo_bytes(algo, pvu, g->weighted && !g->packed, split, split && !g->weighted, r);
      st.edges_narrow += (int64_t)r.edges_narrow;
      cur_pass_changed += r.changed;
      if (r.pass_l1_closed >= 0.0) {
        last_pass_changed = cur_pass_changed;
        last_pass_phase = r.phase;
        last_phase_after = r.phase_after;
        if (delta_on) st.pr_delta_passes++;
        cur_pass_changed = 0;
        st.final_l1 = r.pass_l1_closed;
        if (r.phase == 1) st.verify_passes++;
      }
      st.passes = (int32_t)r.pass_after;
      if (r.done_after) {
        *done = true;
        st.stop_reason = (int32_t)r.stop_reason;
      }
      seq_next++;
    }
    return SR_OK;
  }

  sr_status launch(const SweepArgs &a) {
    st.sweep_launches++;
    if (!timed) {
      hipError_t e = launch_sweep(algo, a, c->compute, nullptr);
      return e == hipSuccess ? SR_OK : c->hip_fail(e, "sweep launch");
    }
    hipEvent_t e0 = ev(), em = ev(), e1 = ev();
    if (e0) (void)hipEventRecord(e0, c->compute);
    hipError_t e = launch_sweep(algo, a, c->compute, em);
    if (e != hipSuccess) return c->hip_fail(e, "sweep launch");
    if (e1) (void)hipEventRecord(e1, c->compute);
    track(e0, e1, false, em);
    return SR_OK;
  }

  // Fill the per-launch fields for pages [list] resident at bufs.
  sr_status make_args(const std::vector<int32_t> &pages, const std::vector<int32_t> &slots,
                      int end_of_pass, SweepArgs &a) {
    const RunState &S = rs ? *rs : g->state;
    std::memset(&a, 0, sizeof(a));
    a.nent = (int32_t)pages.size();
    a.end_of_pass = end_of_pass;
    a.n = g->n;
    a.audit = (prm.flags & SR_RUN_AUDIT_PVU) ? 1 : 0;
    a.early = (algo == A_BFS && !(prm.flags & SR_RUN_NO_EARLY_BREAK)) ? 1 : 0;
    a.pr_seed = algo == A_PPR ? prm.source : -1;
    a.damping = prm.damping;
    a.pr_eps = prm.pr_change_eps;
    a.ctl = S.ctl;
    a.ring = c->ring_dev;
    a.ring_mask = c->ring_mask;
    a.value = S.value;
    a.contrib = S.contrib;
    a.det = det ? 1 : 0;
    a.delta = delta ? 1 : 0;
    a.contrib_next = (det || delta) ? S.contrib_next : nullptr;
    a.resid = delta ? S.resid : nullptr;
    a.inv_outdeg = S.inv_outdeg;
    a.status = S.status;
    a.dia = dia;
    int32_t blk = 0;
    a.blk_prefix[0] = 0;
    for (size_t i = 0; i < pages.size(); ++i) {
      const PageHeader &h = g->pages[pages[i]].hdr;
      for (int sec = 0; sec < NSEC; ++sec) {
        blk += sec_blocks(h, sec, algo == A_PR || algo == A_PPR);
        a.blk_prefix[i * NSEC + sec + 1] = blk;
      }
      a.base[i] = g->res.buf[slots[i]];
      a.partial[i] = g->res.partial[slots[i]];
    }
    a.stripes = S.stripes;
    a.collect = collect;
    a.frontier = S.frontier;
    a.fr_count = S.fr_count;
    a.fr_cap = S.fr_cap;
    a.nblocks = std::max<int32_t>(blk, 1);  // an empty window still closes its sweep
    // the masked decode also serves unweighted graphs whose ids fit 24 bits
    // (it needs fewer registers than the plain one)
    a.packed = (g->weighted ? g->packed : (int64_t)g->n <= ((int64_t)1 << 24)) ? 1 : 0;
    a.split = split ? 1 : 0;
    a.wide3 = split && !g->weighted ? 1 : 0;  // the images of unweighted graphs (see split_layout)
    if (split && !a.packed) return c->fail(SR_EINVAL, "split-width pages need packed edge words");
    return SR_OK;
  }

  sr_status sync_compute() {
    hipError_t e = hipStreamSynchronize(c->compute);
    if (e != hipSuccess) return c->hip_fail(e, "compute stream");
    return SR_OK;
  }
};

}  // namespace

static sr_status ensure_state(sr_graph *g, int algo) {
  sr_ctx *c = g->ctx;
  auto &s = g->state;
  const bool pr = algo == A_PR || algo == A_PPR;
  if (s.n == g->n && s.value && s.ctl && s.stripes && (!pr || s.contrib)) {
    s.algo = algo;
    return SR_OK;
  }
  release_state(g);
  sr_status st;
  if ((st = c->dalloc((void **)&s.value, 4ull * g->n, "vertex values")) != SR_OK) return st;
  if ((st = c->dalloc((void **)&s.status, 1ull * g->n, "predictor states")) != SR_OK) return st;
  if ((st = c->dalloc((void **)&s.ctl, sizeof(Ctl), "control block")) != SR_OK) return st;
  if ((st = c->dalloc((void **)&s.stripes, sizeof(Stripe) * NSTRIPE, "counter stripes")) != SR_OK) return st;
  if (pr) {
    if ((st = c->dalloc((void **)&s.contrib, 4ull * g->n, "pagerank contrib")) != SR_OK) return st;
    if ((st = c->dalloc((void **)&s.inv_outdeg, 4ull * g->n, "pagerank 1/outdeg")) != SR_OK) return st;
    std::vector<float> iod(g->n);
    for (int32_t v = 0; v < g->n; ++v) iod[v] = g->outdeg[v] ? 1.0f / (float)g->outdeg[v] : 0.0f;
    hipError_t e = hipMemcpy(s.inv_outdeg, iod.data(), 4ull * g->n, hipMemcpyHostToDevice);
    if (e != hipSuccess) return c->hip_fail(e, "copy 1/outdeg");
  }
  s.n = g->n;
  s.algo = algo;
  return SR_OK;
}

// Make the pages resident (all of them) or allocate the streaming slots.
sr_status sr::ensure_residency(sr_graph *g, bool weights, bool force_stream, bool bins, uint64_t min_slot) {
  sr_ctx *c = g->ctx;
  auto &r = g->res;
  uint64_t all = 0, mx = min_slot, smx = 0;
  for (auto &p : g->pages) {
    all += need_bytes(p, weights, bins) + scratch_bytes(p);
    mx = std::max(mx, need_bytes(p, weights, bins));
    smx = std::max(smx, scratch_bytes(p));
  }
  const uint64_t freeb = c->budget - c->used + [&] {
    uint64_t mine = 0;
    for (auto p : r.buf) { auto it = c->allocs.find(p); if (it != c->allocs.end()) mine += it->second.bytes; }
    for (auto p : r.partial) { auto it = c->allocs.find(p); if (it != c->allocs.end()) mine += it->second.bytes; }
    return mine;
  }();
  const bool want_resident = !force_stream && all + 4096 <= freeb;
  if (want_resident && r.resident && (r.weights || !weights) && (r.bins || !bins)) return SR_OK;
  if (!want_resident && !r.resident && r.nslots == g->nslots && r.slot_bytes >= mx &&
      (r.weights || !weights) && !r.buf.empty())
    return SR_OK;
  if (bins && !want_resident) return c->fail(SR_EBUDGET, "multi-instance runs need the graph resident");
  release_residency(g);
  sr_status st;
  if (want_resident) {
    r.resident = true;
    r.weights = weights;
    r.bins = bins;
    for (size_t i = 0; i < g->pages.size(); ++i) {
      auto &p = g->pages[i];
      void *b = nullptr, *pa = nullptr;
      uint64_t nb = need_bytes(p, weights, bins);
      uint64_t sc = scratch_bytes(p);
      if ((st = c->dalloc(&b, nb, "resident page")) != SR_OK) { release_residency(g); return st; }
      r.buf.push_back((char *)b);
      if ((st = c->dalloc(&pa, sc, "chunk partials")) != SR_OK) { release_residency(g); return st; }
      r.partial.push_back((unsigned long long *)pa);
      r.partial_words.push_back(sc / 8);
      hipError_t e = hipMemcpyAsync(b, p.host, nb, hipMemcpyHostToDevice, c->copy);
      if (e != hipSuccess) { release_residency(g); return c->hip_fail(e, "resident page copy"); }
      r.slot_page.push_back((int32_t)i);
    }
    hipError_t e = hipStreamSynchronize(c->copy);
    if (e != hipSuccess) { release_residency(g); return c->hip_fail(e, "resident page copy"); }
    return SR_OK;
  }
  // streaming: nslots slots of the largest page
  const int32_t S = g->nslots;
  if ((uint64_t)S * (mx + smx) + 4096 > freeb)
    return c->fail(SR_EBUDGET, "budget cannot hold " + std::to_string(S) + " slots of " +
                                   std::to_string(mx) + " B; partition into more parts");
  r.resident = false;
  r.weights = weights;
  r.nslots = S;
  r.slot_bytes = mx;
  for (int32_t s = 0; s < S; ++s) {
    void *b = nullptr, *pa = nullptr;
    if ((st = c->dalloc(&b, mx, "page slot")) != SR_OK) { release_residency(g); return st; }
    r.buf.push_back((char *)b);
    if ((st = c->dalloc(&pa, smx, "chunk partials")) != SR_OK) { release_residency(g); return st; }
    r.partial.push_back((unsigned long long *)pa);
    r.partial_words.push_back(smx / 8);
    r.slot_page.push_back(-1);
  }
  return SR_OK;
}

extern "C" sr_status sr_run(sr_graph *g, const sr_run_params *params, sr_run_stats *stats) {
  if (!g || !params) return g ? g->ctx->fail(SR_EINVAL, "params is NULL") : SR_EINVAL;
  sr_ctx *c = g->ctx;
  if (c->host_only) return c->fail(SR_EDEVICE, "host-only context cannot run");
  if (g->server_refs > 0) return c->fail(SR_EBUSY, "graph is attached to a server");
  const double t0 = now_ms();
  HIP_TRY(c, hipSetDevice(c->device), "set device");
  Runner R;
  R.g = g;
  R.c = c;
  R.prm = *params;
  sr_run_params &p = R.prm;
  if (p.algo < SR_BFS || p.algo > SR_PPR) return c->fail(SR_EINVAL, "unknown algorithm");
  R.algo = (int)p.algo;
  if (p.damping == 0.0) p.damping = 0.85;
  if (!(p.damping > 0.0 && p.damping < 1.0)) return c->fail(SR_EINVAL, "damping must be in (0,1)");
  if (p.tol_l1 == 0.0) p.tol_l1 = 1e-9;
  if (p.max_passes == 0) p.max_passes = 10000;
  if (p.max_inner_iters == 0) p.max_inner_iters = 4;
  if (p.max_passes < 0 || p.max_inner_iters < 0) return c->fail(SR_EINVAL, "negative limits");
  if (p.flags & ~(SR_RUN_AUDIT_PVU | SR_RUN_FORCE_STREAM | SR_RUN_RESUME | SR_RUN_FIXED_INNER | SR_RUN_HETERO |
                  SR_RUN_SKIP_CLEAN | SR_RUN_NO_EARLY_BREAK | SR_RUN_WIDE_PAGES | SR_RUN_SPLIT_PAGES |
                  SR_RUN_DETERMINISTIC | SR_RUN_PR_DELTA))
    return c->fail(SR_EINVAL, "unknown run flags");
  const bool pr = R.algo == A_PR || R.algo == A_PPR;
  // defaults (Section 4.3 discussion): BFS/CC strong, SSSP/PageRank weak;
  // with the host sparse stage SSSP takes the strong conditions too
  if (p.pvu == SR_PVU_DEFAULT)
    p.pvu = (R.algo == A_BFS || R.algo == A_CC ||
             (R.algo == A_SSSP && (p.flags & (SR_RUN_HETERO | SR_RUN_SKIP_CLEAN))))
                ? SR_PVU_STRONG : SR_PVU_WEAK;
  if (p.pvu < SR_PVU_OFF || p.pvu > SR_PVU_WEAK) return c->fail(SR_EINVAL, "unknown pvu mode");
  if (pr && p.pvu == SR_PVU_STRONG) return c->fail(SR_EINVAL, "PageRank has no strong condition (Table I)");
  R.pvu = (int)p.pvu;
  if ((R.algo == A_BFS || R.algo == A_SSSP || R.algo == A_PPR) && (p.source < 0 || p.source >= g->n))
    return c->fail(SR_EINVAL, "source out of range");
  if (R.algo == A_CC && !g->symmetric)
    return c->fail(SR_EINVAL, "CC needs the undirected graph: load with SR_LOAD_SYMMETRIZE");
  // the caller's source id to the internal one
  if (g->reordered && (R.algo == A_BFS || R.algo == A_SSSP || R.algo == A_PPR)) p.source = g->rank[p.source];
  if (R.algo == A_SSSP && !g->weighted) return c->fail(SR_EINVAL, "SSSP needs weights");
  sr_pvu_diagram d;
  if (p.diagram) d = *p.diagram; else sr_pvu_default_diagram(&d);
  if (!valid_diagram(d)) return c->fail(SR_EINVAL, "invalid predictor diagram");
  std::memset(&R.dia, 0, sizeof(R.dia));
  R.dia.num_states = d.num_states;
  R.dia.initial = d.initial_state;
  R.dia.attempt_mask = d.attempt_mask;
  std::memcpy(R.dia.succ, d.on_success, 8);
  std::memcpy(R.dia.fail, d.on_fail, 8);
  R.weights = R.algo == A_SSSP;
  const bool resume = (p.flags & SR_RUN_RESUME) != 0;
  if (resume && (!g->state.valid || g->state.algo != R.algo))
    return c->fail(SR_ESTATE, "nothing to resume for this algorithm");

  sr_status s;
  if ((p.flags & SR_RUN_WIDE_PAGES) && (p.flags & SR_RUN_SPLIT_PAGES))
    return c->fail(SR_EINVAL, "SR_RUN_WIDE_PAGES and SR_RUN_SPLIT_PAGES exclude each other");
  const bool force_split = (p.flags & SR_RUN_SPLIT_PAGES) != 0;
  if (force_split && (pr || !sr::split_eligible(g)))
    return c->fail(SR_EINVAL, "split-width pages serve streamed BFS/SSSP/CC on graphs with packed edge words");
  if (g->pages.empty())
    if ((s = sr_graph_partition(g, 0, 0)) != SR_OK) return s;
  if ((s = ensure_state(g, R.algo)) != SR_OK) return s;
  // deterministic schedule; PageRank also reads a per-sweep snapshot of the
  // gathered terms (second buffer, allocated once and kept with the state)
  R.det = (p.flags & SR_RUN_DETERMINISTIC) != 0;
  R.delta = (p.flags & SR_RUN_PR_DELTA) != 0;
  if (R.delta) {
    if (!pr) return c->fail(SR_EINVAL, "SR_RUN_PR_DELTA serves PageRank and PPR");
    if (R.det || resume || (p.flags & SR_RUN_AUDIT_PVU))
      return c->fail(SR_EINVAL, "SR_RUN_PR_DELTA excludes SR_RUN_DETERMINISTIC, SR_RUN_RESUME and SR_RUN_AUDIT_PVU");
  }
  if ((R.det || R.delta) && pr && !g->state.contrib_next &&
      (s = c->dalloc((void **)&g->state.contrib_next, 4ull * g->n, "pagerank contrib snapshot")) != SR_OK)
    return s;
  if (R.delta && !g->state.resid &&
      (s = c->dalloc((void **)&g->state.resid, 4ull * g->n, "pagerank-delta residuals")) != SR_OK)
    return s;
  R.delta_on = R.delta;
  // forced split-width images: the slots are sized to hold them too
  auto residency = [&]() -> sr_status {
    uint64_t min_slot = 0;
    if (force_split) {
      sr::size_split_pages(g);
      for (auto &pg : g->pages) min_slot = std::max(min_slot, pg.split_bytes);
    }
    return ensure_residency(g, R.weights, (p.flags & SR_RUN_FORCE_STREAM) != 0, false, min_slot);
  };
  s = residency();
  if (s == SR_EBUDGET && g->auto_parts) {
    // pages sized for a min program do not fit next to this state: recut
    uint64_t st_b = state_bytes(g->n, R.algo);
    if (c->budget > st_b + c->used) {
      for (int32_t P = (int32_t)g->pages.size() * 2; P <= g->n && s == SR_EBUDGET; P *= 2) {
        release_residency(g);
        if ((s = sr::make_pages(g, P, g->equal_edges)) != SR_OK) return s;
        s = residency();
      }
    }
  }
  if (s != SR_OK) return s;
  const int32_t depth = p.copy_depth == 0 ? 1 : p.copy_depth;
  // heterogeneous model (Section 3.1): a host sparse stage finishes the run
  // once a pass changes few vertices; exact when every vertex of that pass
  // was pulled or provably final (strong or no prediction)
  const bool hetero = (p.flags & SR_RUN_HETERO) != 0;
  // page skipping: only streamed passes have copies and sweeps to leave out
  const bool skip = (p.flags & SR_RUN_SKIP_CLEAN) != 0 && !g->res.resident;
  uint32_t sparse_thr = 0, fr_need = 0;
  if (hetero || (p.flags & SR_RUN_SKIP_CLEAN)) {
    if (pr) return c->fail(SR_EINVAL, "the sparse stage and page skipping serve BFS, SSSP and CC");
    if (R.pvu == P_WEAK && (p.flags & SR_RUN_SKIP_CLEAN))
      return c->fail(SR_EINVAL, "page skipping needs strong or no prediction");
  }
  int64_t sparse_ret = 0;  // host frontier size that sends the run back to the device
  if (hetero) {
    if (p.sparse_switch < 0) return c->fail(SR_EINVAL, "sparse_switch must be >= 0");
    if (p.sparse_return < 0) return c->fail(SR_EINVAL, "sparse_return must be >= 0");
    sparse_thr = p.sparse_switch > 0 ? (uint32_t)p.sparse_switch : (uint32_t)std::max<int32_t>(1024, g->n / 512);
    sparse_thr = std::min<uint32_t>(sparse_thr, (uint32_t)g->n);
    sparse_ret = p.sparse_return > 0 ? p.sparse_return : 32ll * sparse_thr;
    fr_need = sparse_thr;
  }
  if (skip) {
    fr_need = std::max<uint32_t>(fr_need, std::min<uint32_t>((uint32_t)g->n, std::max<uint32_t>(1024, g->n / 16)));
    sr::build_out_masks(g);
  }
  if (fr_need > 0) {
    // the frontier takes what the budget has left, up to fr_need entries: a
    // smaller one only means more passes overflow it (then every page is
    // visited, and the sparse stage waits for a pass that fits)
    if (g->state.fr_cap < fr_need) {
      const uint64_t room = c->budget > c->used + 1024 ? c->budget - c->used - 1024 : 0;
      const uint64_t mine = 4ull * g->state.fr_cap;  // freed below
      const uint32_t want = fr_need;
      fr_need = (uint32_t)std::min<uint64_t>(want, (room + mine) / 4);
      if (fr_need < std::min<uint32_t>(want, 256))
        return c->fail(SR_EBUDGET, "budget has no room for the pass frontier");
    }
    if (g->state.fr_cap < fr_need) {
      c->dfree(g->state.frontier);
      g->state.frontier = nullptr;
      g->state.fr_cap = 0;
      if ((s = c->dalloc((void **)&g->state.frontier, 4ull * fr_need, "pass frontier")) != SR_OK) return s;
      g->state.fr_cap = fr_need;
    }
    if (!g->state.fr_count && (s = c->dalloc((void **)&g->state.fr_count, 256, "frontier count")) != SR_OK)
      return s;
  }
  // the host stage's open list (streamed runs under strong prediction)
  // marks the vertices with an in-edge: one bit each, built once per graph;
  // without room in the budget the run goes without that entry to the stage
  if (hetero && R.pvu == P_STRONG && !g->res.resident && g->state.fr_cap > 0 && !g->state.has_in) {
    const uint64_t words = ((uint64_t)g->n + 31) / 32;
    if (c->used + 4 * words + 512 <= c->budget) {
      std::vector<uint32_t> bits((size_t)words, 0u);
      for (int32_t v = 0; v < g->n; ++v)
        if (g->in_off[v + 1] > g->in_off[v]) bits[(size_t)v >> 5] |= 1u << (v & 31);
      if ((s = c->dalloc((void **)&g->state.has_in, 4 * words, "in-edge bitmap")) != SR_OK) return s;
      HIP_TRY(c, hipMemcpy(g->state.has_in, bits.data(), 4 * words, hipMemcpyHostToDevice), "in-edge bitmap");
    }
  }
  if (!g->res.resident && (depth < 1 || depth >= g->res.nslots))
    return c->fail(SR_EINVAL, "copy_depth must be in [1, num_slots)");
  // streamed min programs copy split-width images when every one fits a slot
  // and together they are smaller than the full-width prefixes they replace;
  // when the pinned images cannot be allocated the run streams the
  // full-width pages, unless the images were asked for
  if (force_split && g->res.resident)
    return c->fail(SR_EINVAL, "split-width pages serve streamed runs; this graph is resident");
  if (!pr && !g->res.resident && !(p.flags & SR_RUN_WIDE_PAGES) && sr::split_eligible(g)) {
    uint64_t wide = 0, narrow = 0, mx = 0;
    for (auto &pg : g->pages) {
      const bool lead = !R.weights || pg.hdr.w_bytes == 0;
      wide += lead ? pg.hdr.bytes_lead : need_bytes(pg, R.weights);
    }
    // a sampled estimate first, so graphs whose images would not be clearly
    // smaller are not read whole; the images are built (which sizes them
    // exactly) when the estimate takes them, and used when each fits a slot
    // and together they are smaller
    const bool counted = !g->pages.empty() && g->pages[0].narrow >= 0;
    if (!counted && !g->pages.empty() && g->pages[0].split_est == 0)
      g->pages[0].split_est = sr::estimate_split_bytes(g);
    if (force_split || counted || (double)g->pages[0].split_est < 0.97 * (double)wide) {
      if ((s = sr::build_split_pages(g)) != SR_OK) {
        if (force_split) return s;
        narrow = wide;  // not taken
      } else {
        for (auto &pg : g->pages) {
          narrow += pg.split_bytes;
          mx = std::max(mx, pg.split_bytes);
        }
      }
    } else {
      narrow = wide;  // not taken
    }
    if (force_split && mx > g->res.slot_bytes)
      return c->fail(SR_EBUDGET, "a split-width page image is larger than a slot");
    R.split = mx <= g->res.slot_bytes && (force_split || narrow < wide);
  }

  // initial values, predictor states and control block
  RunState &rs = g->state;
  Ctl init;
  std::memset(&init, 0, sizeof(init));
  init.threshold = 0;  // value 0 is final for every min program (source, global minimum label)
  init.phase = 0;
  init.pass_min_changed = INF;
  init.best_l1 = 1e300;
  init.algo = R.algo;
  init.pvu = R.pvu;
  init.max_passes = p.max_passes;
  init.tol_l1 = p.tol_l1;
  init.floor_cap = 1e-6;
  // a PageRank pass of single plain sweeps is already a verification pass
  // (not for PageRank-delta, whose residual phase comes first)
  if (pr && !R.delta && R.pvu == P_OFF && (p.max_inner_iters == 1 || g->res.resident)) init.phase = 1;
  init.delta = R.delta ? 1u : 0u;
  init.dangling_next = 0.0;
  // PageRank: the rank sum and dangling sum are taken from the ranks on the
  // device once they are set (fresh or resumed)
  init.mass = 1.0;
  hipError_t e = hipSuccess;
  if (!resume) {
    if (R.delta) e = launch_init_prd((float *)rs.value, rs.resid, rs.contrib, rs.contrib_next, g->n,
                                     R.algo == A_PPR ? p.source : -1, p.damping, c->compute);
    else if (pr) e = launch_init_pr((float *)rs.value, rs.contrib, rs.inv_outdeg, g->n,
                                    R.algo == A_PPR ? p.source : -1, c->compute);
    else e = launch_init_min(R.algo, rs.value, g->n, p.source, c->compute);
    // CC labels are the caller's ids, so the smallest one of a component
    // wins; from pinned memory the copy needs no staging and overlaps the
    // first page's
    if (e == hipSuccess && R.algo == A_CC && g->reordered) {
      if (!g->perm_pinned) {
        if (hipHostMalloc((void **)&g->perm_pinned, 4ull * g->n, hipHostMallocDefault) == hipSuccess)
          std::memcpy(g->perm_pinned, g->perm.data(), 4ull * g->n);
        else
          g->perm_pinned = nullptr;  // (the pageable copy below still works, staged)
      }
      const int32_t *src = g->perm_pinned ? g->perm_pinned : g->perm.data();
      e = hipMemcpyAsync(rs.value, src, 4ull * g->n, hipMemcpyHostToDevice, c->compute);
    }
    if (e == hipSuccess) e = launch_fill_u8(rs.status, (uint8_t)d.initial_state, (size_t)g->n, c->compute);
  }
  // on resume the values and predictor states stay; the control block
  // (pass bookkeeping, thresholds back at their safe initial value) and, for
  // PageRank, the rank and dangling sums start afresh from the values
  if (e == hipSuccess) e = launch_init_ctl(rs.ctl, init, c->compute);
  // (PageRank-delta: nothing sent yet, so no dangling mass; the sums are
  // taken when its residual phase ends)
  if (e == hipSuccess && pr && !R.delta)
    e = launch_pr_sums((const float *)rs.value, rs.inv_outdeg, g->n, rs.ctl, c->compute);
  // the snapshot's second buffer starts equal to the gathered terms
  if (e == hipSuccess && pr && R.det)
    e = hipMemcpyAsync(rs.contrib_next, rs.contrib, 4ull * g->n, hipMemcpyDeviceToDevice, c->compute);
  if (e == hipSuccess) e = launch_init_stripes(rs.stripes, c->compute);
  // heavy-vertex accumulators start at the reduction's identity (min: all
  // ones; PageRank: fixed-point zero); the close kernel restores it after
  // every sweep
  for (size_t i = 0; i < g->res.partial.size() && e == hipSuccess; ++i) {
    const uint64_t words = g->res.partial_words[i];
    e = launch_fill_u32((uint32_t *)g->res.partial[i], pr ? 0u : INF, 2 * words, c->compute);
  }
  if (e != hipSuccess) return c->hip_fail(e, "init");
  // fresh record numbering for this run
  for (uint32_t i = 0; i < RING; ++i) c->ring_host[i].seq = ~0ull;
  g->sweeps.clear();
  R.seq_next = 0;
  rs.valid = true;

  // Host sparse stage (Section 3.1). A pass collects the vertices it changes
  // once the pass before changed few enough; when a pass changed at most
  // sparse_thr vertices and all were collected, the host pushes from them to
  // the fixed point. Every edge whose source did not change in that pass is
  // already satisfied (its target was pulled after the source's last change,
  // or is final by Table I), so the push from the frontier is exact.
  // With weak prediction a skipped vertex is not provably final, so the
  // switch first runs a verification pass (prediction off, every vertex
  // pulled once, Section 4.3's all-pull at the dense to sparse switch) and
  // hands over after it; so does a run the host stage gave back.
  bool force_verify = false;
  bool returned = false;  // the host stage gave the run back in the last pass end
  auto begin_pass = [&]() -> sr_status {
    if (hetero && R.pvu == P_WEAK &&
        (force_verify || (R.last_pass_phase == 0 && R.last_pass_changed <= sparse_thr))) {
      hipError_t e2 = launch_set_phase(g->state.ctl, 1u, c->compute);
      if (e2 != hipSuccess) return c->hip_fail(e2, "verification switch");
      force_verify = false;
    }
    R.collect = (skip || (hetero && (R.last_pass_changed <= 32ull * sparse_thr ||
                                     (uint64_t)g->n <= 32ull * sparse_thr))) ? 1 : 0;
    if (R.collect) {
      hipError_t e2 = launch_fill_u32(g->state.fr_count, 0u, 1, c->compute);
      if (e2 != hipSuccess) return c->hip_fail(e2, "frontier reset");
    }
    return SR_OK;
  };
  // the frontier of the pass just closed (false when it overflowed)
  std::vector<uint32_t> fr;
  auto read_frontier = [&](bool *complete) -> sr_status {
    *complete = false;
    uint32_t cnt = 0;
    HIP_TRY(c, hipMemcpyAsync(&cnt, g->state.fr_count, 4, hipMemcpyDeviceToHost, c->compute), "frontier count");
    HIP_TRY(c, hipStreamSynchronize(c->compute), "frontier count");
    if (cnt > g->state.fr_cap) return SR_OK;  // incomplete
    fr.resize(cnt);
    if (cnt) {
      HIP_TRY(c, hipMemcpyAsync(fr.data(), g->state.frontier, 4ull * cnt, hipMemcpyDeviceToHost, c->compute),
              "frontier to host");
      HIP_TRY(c, hipStreamSynchronize(c->compute), "frontier to host");
    }
    *complete = true;
    return SR_OK;
  };
  std::vector<uint32_t> rest;  // host frontier handed back to the device
  // A push that stays small reads only the values it needs: each round's
  // missing values are gathered on the device into the frontier buffer's
  // upper half (ids in its lower half), and at the end the lowered values
  // (and `also`, vertices the caller lowered) are scattered back. *done is
  // false, with the device values untouched, when the push outgrows half the
  // buffer, its list passes sparse_ret, or it needs more round trips (about
  // 40 us each) than copying the value array both ways would cost (8n bytes
  // at ~56 GB/s, about n / 7000 us; at least 2 round trips); the caller then
  // copies the arrays.
  auto push_fetched = [&](std::unordered_map<uint32_t, uint32_t> &known, const std::vector<uint32_t> &front,
                          const std::vector<uint32_t> &also, bool *done, int32_t *rounds,
                          int64_t *relaxed) -> sr_status {
    *done = false;
    const uint32_t half = g->state.fr_cap / 2;
    if (half == 0) return SR_OK;
    uint32_t *d_ids = g->state.frontier, *d_got = g->state.frontier + half;
    sr::build_out_csr(g);
    hipError_t fe = hipSuccess;
    const int64_t max_fetches = std::max<int64_t>(2, (int64_t)g->n / 350000);
    int64_t fetches = 0;
    auto fetch = [&](const std::vector<uint32_t> &need, std::vector<uint32_t> &vals) -> bool {
      if (++fetches > max_fetches) return false;
      fe = hipMemcpyAsync(d_ids, need.data(), 4ull * need.size(), hipMemcpyHostToDevice, c->compute);
      if (fe == hipSuccess) fe = launch_gather_u32(g->state.value, d_ids, (uint32_t)need.size(), d_got, c->compute);
      if (fe == hipSuccess) fe = hipMemcpyAsync(vals.data(), d_got, 4ull * need.size(), hipMemcpyDeviceToHost, c->compute);
      if (fe == hipSuccess) fe = hipStreamSynchronize(c->compute);
      R.st.sparse_copy_bytes += 4ull * need.size();
      return fe == hipSuccess;
    };
    std::vector<uint32_t> lowered;
    int32_t pr = 0;
    int64_t rel = 0;
    const bool ok = sr::sparse_push_partial(g, R.algo, known, front, sparse_ret, half, fetch, &lowered, &pr, &rel);
    if (fe != hipSuccess) return c->hip_fail(fe, "push values from device");
    if (!ok) return SR_OK;
    std::vector<uint32_t> wid(also);
    wid.insert(wid.end(), lowered.begin(), lowered.end());
    std::sort(wid.begin(), wid.end());
    wid.erase(std::unique(wid.begin(), wid.end()), wid.end());
    if (wid.size() > half) return SR_OK;
    if (!wid.empty()) {
      std::vector<uint32_t> wval(wid.size());
      for (size_t i = 0; i < wid.size(); ++i) wval[i] = known[wid[i]];
      HIP_TRY(c, hipMemcpyAsync(d_ids, wid.data(), 4ull * wid.size(), hipMemcpyHostToDevice, c->compute),
              "lowered ids to device");
      HIP_TRY(c, hipMemcpyAsync(d_got, wval.data(), 4ull * wid.size(), hipMemcpyHostToDevice, c->compute),
              "lowered values to device");
      HIP_TRY(c, launch_scatter_u32(g->state.value, d_ids, d_got, (uint32_t)wid.size(), c->compute), "lowered values");
      HIP_TRY(c, hipStreamSynchronize(c->compute), "lowered values");
      R.st.sparse_copy_bytes += 4ull * wid.size();
    }
    *done = true;
    *rounds = pr;
    *relaxed = rel;
    return SR_OK;
  };
  auto sparse_stage = [&](bool have_fr, bool *fin) -> sr_status {
    *fin = false;
    returned = false;
    if (!hetero || !R.collect || !have_fr || R.last_pass_changed > sparse_thr) return SR_OK;
    if (R.pvu == P_WEAK && R.last_pass_phase != 1) return SR_OK;  // not after a verification pass
    const double t1 = now_ms();
    int32_t rounds = 0;
    int64_t relaxed = 0;
    bool pushed = false;
    rest.clear();
    {
      std::unordered_map<uint32_t, uint32_t> known;
      sr_status s2 = push_fetched(known, fr, {}, &pushed, &rounds, &relaxed);
      if (s2 != SR_OK) return s2;
    }
    if (!pushed) {
      if (!g->host_val && g->n > 0) {
        HIP_TRY(c, hipHostMalloc((void **)&g->host_val, 4ull * g->n, hipHostMallocDefault), "pinned value mirror");
      }
      uint32_t *val = g->host_val;
      R.st.sparse_copy_bytes += 4ull * g->n;
      HIP_TRY(c, hipMemcpyAsync(val, g->state.value, 4ull * g->n, hipMemcpyDeviceToHost, c->compute),
              "values to host");
      HIP_TRY(c, hipStreamSynchronize(c->compute), "values to host");
      sr::build_out_csr(g);
      relaxed = sr::sparse_push(g, R.algo, val, fr.data(), (int64_t)fr.size(), &rounds, sparse_ret, &rest);
      R.st.sparse_copy_bytes += 4ull * g->n;
      HIP_TRY(c, hipMemcpyAsync(g->state.value, val, 4ull * g->n, hipMemcpyHostToDevice, c->compute),
              "values to device");
      HIP_TRY(c, hipStreamSynchronize(c->compute), "values to device");
    }
    R.st.sparse_entries++;
    R.st.sparse_rounds += rounds;
    R.st.sparse_frontier = (int64_t)fr.size();
    R.st.sparse_relaxations += relaxed;
    R.st.sparse_ms += now_ms() - t1;
    if (!rest.empty()) {
      // the frontier grew dense again: the device passes take over. Every
      // value is still an upper bound reached along real paths, and every
      // value the host produced is at least the smallest value the last
      // device pass changed, so the Table I threshold stays sound; with weak
      // prediction the next pass is a verification pass.
      R.st.sparse_returns++;
      R.last_pass_changed = (uint64_t)rest.size();
      if (R.pvu == P_WEAK) force_verify = true;
      returned = true;
      return SR_OK;
    }
    R.st.sparse_stage = 1;
    R.st.stop_reason = SR_STOP_CONVERGED;
    *fin = true;
    return SR_OK;
  };
  // The host stage entered from the vertices the next pass would attempt
  // (streamed runs under strong prediction): after a pass whose changed set
  // is too large for the sparse stage above, the device lists the vertices
  // with an in-edge and a value above the Table I threshold; when there are
  // at most sparse_thr of them, the host pulls them over its copy of the
  // in-edges instead of streaming every page again, and pushes from those
  // that changed. Exact: every vertex off the list is final by Table I or
  // has no in-edge, and every value the host lowers stays above the
  // threshold (a vertex on the list is not final, so its true value is
  // above it), so a hand-back to the device keeps Table I sound.
  auto open_stage = [&](bool *fin) -> sr_status {
    *fin = false;
    if (!hetero || R.pvu != P_STRONG || g->res.resident || !g->state.has_in || g->state.fr_cap == 0) return SR_OK;
    const double t1 = now_ms();
    HIP_TRY(c, launch_fill_u32(g->state.fr_count, 0u, 1, c->compute), "open list");
    HIP_TRY(c, launch_open_list(g->state.value, g->state.has_in, g->n, g->state.ctl, g->state.frontier,
                                g->state.fr_cap, g->state.fr_count, c->compute), "open list");
    uint32_t cnt = 0;
    HIP_TRY(c, hipMemcpyAsync(&cnt, g->state.fr_count, 4, hipMemcpyDeviceToHost, c->compute), "open count");
    HIP_TRY(c, hipStreamSynchronize(c->compute), "open count");
    if (cnt > sparse_thr || cnt > g->state.fr_cap) return SR_OK;
    if (!g->host_val && g->n > 0) {
      HIP_TRY(c, hipHostMalloc((void **)&g->host_val, 4ull * g->n, hipHostMallocDefault), "pinned value mirror");
    }
    uint32_t *val = g->host_val;
    std::vector<uint32_t> open((size_t)cnt);
    if (cnt) {
      HIP_TRY(c, hipMemcpyAsync(open.data(), g->state.frontier, 4ull * cnt, hipMemcpyDeviceToHost, c->compute),
              "open list to host");
      HIP_TRY(c, hipStreamSynchronize(c->compute), "open list to host");
    }
    // a short list reads only the values the pull needs (the listed vertices
    // and their in-neighbours, gathered on the device into the frontier's
    // upper half); when the pull changes something the push goes on the same
    // way, fetching each round's missing values and writing back only the
    // lowered ones; a long list, or a push that outgrows the buffer, reads
    // the whole value array
    std::vector<uint32_t> changed;
    int64_t relaxed = 0;
    int32_t rounds = 1;
    bool pulled = false;  // the pull changed nothing
    bool pushed = false;  // a short push reached the fixed point
    {
      std::vector<uint32_t> ids(open.begin(), open.end());
      const uint32_t half = g->state.fr_cap / 2;
      for (uint32_t v : open) {
        for (int64_t e = g->in_off[v]; e < g->in_off[v + 1] && ids.size() <= half; ++e) ids.push_back((uint32_t)g->in_src[e]);
        if (ids.size() > half) break;
      }
      if (ids.size() <= half) {
        std::vector<uint32_t> got(ids.size());
        uint32_t *d_ids = g->state.frontier, *d_got = g->state.frontier + half;
        if (!ids.empty()) {
          HIP_TRY(c, hipMemcpyAsync(d_ids, ids.data(), 4ull * ids.size(), hipMemcpyHostToDevice, c->compute),
                  "open ids to device");
          HIP_TRY(c, launch_gather_u32(g->state.value, d_ids, (uint32_t)ids.size(), d_got, c->compute), "open gather");
          HIP_TRY(c, hipMemcpyAsync(got.data(), d_got, 4ull * ids.size(), hipMemcpyDeviceToHost, c->compute),
                  "open values to host");
          HIP_TRY(c, hipStreamSynchronize(c->compute), "open values to host");
          R.st.sparse_copy_bytes += 4ull * ids.size();
        }
        for (size_t i = 0; i < ids.size(); ++i) val[ids[i]] = got[i];
        relaxed = sr::sparse_pull(g, R.algo, val, open.data(), (int64_t)cnt, &changed);
        pulled = changed.empty();
        if (!pulled) {
          std::unordered_map<uint32_t, uint32_t> known;
          known.reserve(2 * ids.size());
          for (uint32_t v : ids) known[v] = val[v];
          int32_t prounds = 0;
          int64_t prelaxed = 0;
          sr_status s2 = push_fetched(known, changed, changed, &pushed, &prounds, &prelaxed);
          if (s2 != SR_OK) return s2;
          if (pushed) {
            rounds += prounds;
            relaxed += prelaxed;
          }
        }
      }
    }
    rest.clear();
    if (!pulled && !pushed) {
      HIP_TRY(c, hipMemcpyAsync(val, g->state.value, 4ull * g->n, hipMemcpyDeviceToHost, c->compute), "values to host");
      HIP_TRY(c, hipStreamSynchronize(c->compute), "values to host");
      R.st.sparse_copy_bytes += 4ull * g->n;
      relaxed = sr::sparse_pull(g, R.algo, val, open.data(), (int64_t)cnt, &changed);
      if (!changed.empty()) {
        sr::build_out_csr(g);
        int32_t pr_rounds = 0;
        relaxed += sr::sparse_push(g, R.algo, val, changed.data(), (int64_t)changed.size(), &pr_rounds, sparse_ret,
                                   &rest);
        rounds += pr_rounds;
        HIP_TRY(c, hipMemcpyAsync(g->state.value, val, 4ull * g->n, hipMemcpyHostToDevice, c->compute),
                "values to device");
        HIP_TRY(c, hipStreamSynchronize(c->compute), "values to device");
        R.st.sparse_copy_bytes += 4ull * g->n;
      }
    }
    R.st.sparse_entries++;
    R.st.sparse_rounds += rounds;
    R.st.sparse_frontier = (int64_t)cnt;
    R.st.sparse_relaxations += relaxed;
    R.st.sparse_ms += now_ms() - t1;
    if (!rest.empty()) {
      R.st.sparse_returns++;
      R.last_pass_changed = (uint64_t)rest.size();
      returned = true;
      return SR_OK;
    }
    R.st.sparse_stage = 1;
    R.st.stop_reason = SR_STOP_CONVERGED;
    *fin = true;
    return SR_OK;
  };
  // after a pass: the host sparse stage if it applies
  auto pass_end_host = [&](bool *fin) -> sr_status {
    *fin = false;
    bool have = false;
    if (R.collect) {
      sr_status s2 = read_frontier(&have);
      if (s2 != SR_OK) return s2;
    }
    return sparse_stage(have, fin);
  };

  // PageRank-delta: after every pass of its residual phase the terms that
  // pass sent become the ones the next pass gathers; when the phase ends
  // (close_pass turned the verification phase on) the ranks are turned into
  // rank-form terms and the rank and dangling sums are taken afresh
  auto delta_pass_end = [&]() -> sr_status {
    if (!R.delta_on) return SR_OK;
    std::swap(g->state.contrib, g->state.contrib_next);
    if (R.last_phase_after == 1) {
      R.delta_on = false;
      hipError_t e2 = launch_rank_terms((const float *)g->state.value, g->state.contrib, g->state.inv_outdeg,
                                        g->n, c->compute);
      if (e2 == hipSuccess)
        e2 = launch_pr_sums((const float *)g->state.value, g->state.inv_outdeg, g->n, g->state.ctl, c->compute);
      if (e2 != hipSuccess) return c->hip_fail(e2, "rank-form terms");
    }
    return SR_OK;
  };

  bool done = false;
  if (g->res.resident) {
    // Every sweep covers every page and closes a pass; the control block
    // carries thresholds and phases between sweeps, so sweeps are enqueued
    // in batches with one host check per batch.
    std::vector<std::vector<int32_t>> groups;
    for (int32_t i = 0; i < (int32_t)g->pages.size(); i += MAXW) {
      std::vector<int32_t> grp;
      for (int32_t j = i; j < std::min<int32_t>(i + MAXW, (int32_t)g->pages.size()); ++j) grp.push_back(j);
      groups.push_back(grp);
    }
    std::vector<SweepArgs> args(groups.size());
    for (size_t k = 0; k < groups.size(); ++k)
      R.make_args(groups[k], groups[k], k + 1 == groups.size() ? 1 : 0, args[k]);
    const int batch = 4;
    int32_t launched = 0;
    while (!done) {
      if ((s = begin_pass()) != SR_OK) return s;
      // a collecting pass runs alone so its frontier can be handed over, and
      // so does a pass of PageRank-delta's residual phase (its buffers swap)
      const int nb = (R.collect || R.delta_on) ? 1 : batch;
      for (int b = 0; b < nb; ++b) {
        for (auto &a : args) {
          a.collect = R.collect;
          if ((s = R.launch(a)) != SR_OK) return s;
        }
        launched++;
      }
      if ((s = R.sync_compute()) != SR_OK) return s;
      R.harvest(&done);
      if (!done && R.delta_on) {
        if ((s = delta_pass_end()) != SR_OK) return s;
        for (size_t k = 0; k < groups.size(); ++k)
          R.make_args(groups[k], groups[k], k + 1 == groups.size() ? 1 : 0, args[k]);
      }
      if (!done) {
        bool fin = false;
        if ((s = pass_end_host(&fin)) != SR_OK) return s;
        done = fin;
      }
      if (launched > p.max_passes + 8) break;
    }
  } else {
    // Pipelined subgraph iteration (Section 3.2): a window of W = S-D slots is
    // swept while the next D pages are copied into the remaining slots (the
    // paper's layout is D = 1); each window is swept until the page it takes
    // next has landed (re-entry), max_inner_iters, or a sweep without change;
    // then the window slides by one page. Pages go in increasing order every
    // pass (in R-MAT graphs, whose low ids carry most edges, this order
    // propagates furthest per pass); the last steps of a pass already fetch
    // the first pages of the next one, and a page still in a slot is not
    // copied again.
    const int32_t P = (int32_t)g->pages.size();
    const int32_t S = g->res.nslots;
    const int32_t D = depth;
    const int32_t W = S - D;
    std::vector<hipEvent_t> copy_done(S, nullptr);
    hipEvent_t step_done = nullptr;
    std::vector<hipEvent_t> own;
    // (a failed creation leaves a null entry, which the check below reports)
    auto mk = [&]() {
      hipEvent_t ev = nullptr;
      if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) ev = nullptr;
      own.push_back(ev);
      return ev;
    };
    for (int32_t i = 0; i < S; ++i) copy_done[i] = mk();
    step_done = mk();
    // Deterministic schedule: the host keeps the device one sweep ahead of
    // what it has seen finish. The close kernel marks a window whose sweep
    // changed nothing, and a sweep of that window already queued exits at
    // once (leaving an empty record, so records number the launches). Before
    // a step the host also waits for the step LAG back and reads the records
    // written up to it.
    const bool devq = R.det && !(p.flags & SR_RUN_FIXED_INNER);
    constexpr int LAG = 2;
    std::vector<hipEvent_t> lag_ev(LAG + 1, nullptr);
    std::vector<uint64_t> lag_rec(LAG + 1, 0);  // records written once that step has ended
    hipEvent_t sw_ev[3] = {nullptr, nullptr, nullptr};  // after each of the last three sweeps of a step
    uint64_t sw_rec[3] = {0, 0, 0};
    if (devq) {
      for (auto &ev : lag_ev) ev = mk();
      for (auto &ev : sw_ev) ev = mk();
    }
    int64_t step_idx = 0;
    uint64_t rec_launched = 0;  // records the enqueued kernels will have written (devq: one per sweep)
    struct Cleanup { std::vector<hipEvent_t> *v; ~Cleanup() { for (auto e : *v) if (e) (void)hipEventDestroy(e); } } cl{&own};
    for (auto ev : own) if (!ev) return c->fail(SR_EDEVICE, "event creation failed");
    std::vector<int32_t> &slot_page = g->res.slot_page;
    std::fill(slot_page.begin(), slot_page.end(), -1);  // slot contents of older runs are not trusted
    std::vector<int32_t> page_slot(P, -1);
    std::vector<int64_t> last_use(S, -1);   // step counter of the last window that used each slot
    int64_t step_clock = 0;
    auto copy_page = [&](int32_t page, int32_t slot, bool wait_prev) -> sr_status {
      if (wait_prev) HIP_TRY(c, hipStreamWaitEvent(c->copy, step_done, 0), "copy wait");
      hipEvent_t a = R.ev(), b = R.ev();
      // a min program that reads no separate weights stops at the last
      // offset it reads (PageRank also rewrites zero in-degree vertices)
      const PageHeader &ph = g->pages[page].hdr;
      const bool lead = !pr && (!R.weights || ph.w_bytes == 0);
      uint64_t nb = lead ? ph.bytes_lead : need_bytes(g->pages[page], R.weights);
      const char *src = g->pages[page].host;
      if (R.split) { nb = g->pages[page].shdr.bytes_lead; src = g->pages[page].split; }
      if (a) (void)hipEventRecord(a, c->copy);
      HIP_TRY(c, hipMemcpyAsync(g->res.buf[slot], src, nb, hipMemcpyHostToDevice, c->copy), "page copy");
      if (b) (void)hipEventRecord(b, c->copy);
      R.track(a, b, true);
      HIP_TRY(c, hipEventRecord(copy_done[slot], c->copy), "copy event");
      if (slot_page[slot] >= 0) page_slot[slot_page[slot]] = -1;
      slot_page[slot] = page;
      page_slot[page] = slot;
      R.st.h2d_bytes += nb;
      return SR_OK;
    };
    // a slot that holds none of the pages in `keep` (least recently used first)
    auto free_slot = [&](const std::vector<int32_t> &keep) -> int32_t {
      int32_t best = -1;
      for (int32_t sl = 0; sl < S; ++sl) {
        bool used = false;
        for (int32_t q : keep) used |= page_slot[q] == sl;
        if (used) continue;
        if (best < 0 || last_use[sl] < last_use[best]) best = sl;
      }
      return best;
    };
    int32_t pass = 0;
    const bool fixed_inner = (p.flags & SR_RUN_FIXED_INNER) != 0;
    std::vector<int32_t> ord(P);
    for (int32_t i = 0; i < P; ++i) ord[i] = i;
    // A pass of a min program that has changed nothing by its last steps is
    // most likely the final one (under strong or no prediction, or a weak
    // run's verification pass, its end finds no change and stops the run),
    // so the first pages of a next pass are not fetched ahead then; a wrong
    // guess only delays that pass's first copy.
    const bool guess_last = !pr;
    // A pass whose end the host stage will likely take (open_stage) does not
    // fetch the next pass's first pages ahead. The guess is taken once the
    // window starts on the second half of the pass: the device counts the
    // vertices of the pages it has finished that the next pass would attempt
    // if the pass ended now; few enough, and the copies are left out (a
    // wrong guess only delays the next pass's first copy).
    const bool open_guess = hetero && R.pvu == P_STRONG && !skip && g->state.has_in && g->state.fr_cap > 0;
    while (!done) {
      // pass start: every earlier sweep has finished (host synced at the pass end)
      if ((s = begin_pass()) != SR_OK) return s;
      const int32_t NP = (int32_t)ord.size();  // pages of this pass
      bool pass_changed = false, pass_verify = false;
      bool guessed = false, host_end = false;
      if (NP > 0 && page_slot[ord[0]] < 0) {
        if ((s = copy_page(ord[0], free_slot({}), false)) != SR_OK) return s;
      }
      // records harvested so far: did this pass change anything, is it a
      // verification pass
      auto absorb = [&](uint64_t limit) {
        const uint64_t before = R.seq_next;
        R.harvest(&done, limit);
        bool changed = false;
        for (uint64_t q = before; q < R.seq_next; ++q) {
          changed |= c->ring_host[q & c->ring_mask].changed > 0;
          pass_verify = c->ring_host[q & c->ring_mask].phase == 1;
        }
        pass_changed |= changed;
        return changed;
      };
      for (int32_t j = 0; j < NP && !done; ++j) {
        if (devq && step_idx >= LAG) {
          HIP_TRY(c, hipEventSynchronize(lag_ev[(step_idx - LAG) % (LAG + 1)]), "step wait");
          absorb(lag_rec[(step_idx - LAG) % (LAG + 1)]);
          if (done) break;
        }
        // PageRank-delta's residual phase sweeps every page once per pass
        // (each sent term is received once): the window is the newest page
        std::vector<int32_t> win;
        for (int32_t q = R.delta_on ? j : std::max(0, j - W + 1); q <= j; ++q) win.push_back(ord[q]);
        for (int32_t q : win) HIP_TRY(c, hipStreamWaitEvent(c->compute, copy_done[page_slot[q]], 0), "compute wait");
        // keep the next D pages coming (past the pass end: the next pass's
        // first pages); a free slot was last read by an earlier step's sweeps
        std::vector<int32_t> keep = win;
        if (open_guess && !guessed && j + D >= NP) {
          guessed = true;
          const int32_t first = std::max(0, j - W + 1);  // pages before it are finished
          if (2 * first >= NP) {
            uint32_t *cnt_dev = g->state.fr_count + 1;  // (entry 0 counts the pass frontier)
            uint32_t cnt = 0;
            HIP_TRY(c, launch_fill_u32(cnt_dev, 0u, 1, c->compute), "open guess");
            HIP_TRY(c, launch_open_guess(g->state.value, g->state.has_in, g->pages[ord[first]].hdr.v_begin,
                                         g->state.ctl, cnt_dev, c->compute), "open guess");
            HIP_TRY(c, hipMemcpyAsync(&cnt, cnt_dev, 4, hipMemcpyDeviceToHost, c->compute), "open guess");
            HIP_TRY(c, hipStreamSynchronize(c->compute), "open guess");
            host_end = cnt <= sparse_thr;
          }
        }
        for (int32_t q = 1; q <= D; ++q) {
          // skipping decides the next pass's pages at the pass end: no wrap
          if (skip && j + q >= NP) break;
          if (host_end && j + q >= NP) break;
          if (guess_last && pass > 0 && !pass_changed && (R.pvu != P_WEAK || pass_verify) && j + q >= NP) break;
          const int32_t page = ord[(j + q) % NP];
          if (std::find(keep.begin(), keep.end(), page) != keep.end()) continue;
          if (page_slot[page] < 0) {
            const int32_t sl = free_slot(keep);
            if (sl < 0) break;
            if ((s = copy_page(page, sl, j > 0 || pass > 0)) != SR_OK) return s;
          }
          keep.push_back(page);
        }
        // the window slides once the page it takes next has landed
        const int32_t next_slot = page_slot[ord[(j + 1) % NP]];
        const bool copying = next_slot >= 0 && hipEventQuery(copy_done[next_slot]) != hipSuccess;
        std::vector<int32_t> ws;
        for (int32_t q : win) { ws.push_back(page_slot[q]); last_use[page_slot[q]] = step_clock; }
        ++step_clock;
        SweepArgs a;
        if ((s = R.make_args(win, ws, 0, a)) != SR_OK) return s;
        if (devq) {
          // one sweep stays queued beyond the newest one the host has seen
          // finish: before launching sweep k the host waits for sweep k-2 and
          // stops when it changed nothing (sweep k-1, already queued, then
          // exits at once), so a window step launches at most one sweep that
          // does no work and the device never waits for the host
          const int32_t iters = R.delta_on ? 1 : p.max_inner_iters;  // delta: one sweep per page and pass
          a.win_skip = 1;
          for (int32_t it = 0; it < iters; ++it) {
            if (it >= 2) {
              const int k = (it - 2) % 3;
              HIP_TRY(c, hipEventSynchronize(sw_ev[k]), "sweep wait");
              absorb(sw_rec[k]);
              if (done) break;
              if (c->ring_host[(sw_rec[k] - 1) & c->ring_mask].changed == 0) break;
            }
            a.win_first = it == 0 ? 1 : 0;
            if ((s = R.launch(a)) != SR_OK) return s;
            ++rec_launched;
            HIP_TRY(c, hipEventRecord(sw_ev[it % 3], c->compute), "sweep event");
            sw_rec[it % 3] = rec_launched;
          }
        }
        for (int32_t it = 0; !devq && it < p.max_inner_iters; ++it) {
          if ((s = R.launch(a)) != SR_OK) return s;
          if ((s = R.sync_compute()) != SR_OK) return s;
          const bool changed = absorb(~0ull);
          if (done) break;
          if (R.delta_on) break;                    // one sweep per page and pass
          if (fixed_inner) continue;                // fixed re-entry count (ablation schedules)
          if (!changed) break;                      // the window reached its local fixed point
          if (R.det) continue;                      // deterministic: the copy's timing does not decide
          if (!copying) break;                      // nothing in flight to wait for
          if (hipEventQuery(copy_done[next_slot]) == hipSuccess) break;  // next page landed: slide
        }
        HIP_TRY(c, hipEventRecord(step_done, c->compute), "step event");
        if (devq) {
          HIP_TRY(c, hipEventRecord(lag_ev[step_idx % (LAG + 1)], c->compute), "step event");
          lag_rec[step_idx % (LAG + 1)] = rec_launched;
        }
        ++step_idx;
      }
      if (done) break;
      HIP_TRY(c, launch_end_pass(g->state.ctl, c->ring_dev, c->ring_mask, c->compute), "end pass");
      ++rec_launched;
      if ((s = R.sync_compute()) != SR_OK) return s;
      R.harvest(&done);
      if (!done && (s = delta_pass_end()) != SR_OK) return s;
      if (!done) {
        bool fin = false, have = false;
        if (R.collect && (s = read_frontier(&have)) != SR_OK) return s;
        if ((s = sparse_stage(have, &fin)) != SR_OK) return s;
        done = fin;
        if (!done && !returned) {
          if ((s = open_stage(&fin)) != SR_OK) return s;
          done = fin;
        }
        if (!done && skip) {
          // next pass: the pages an edge from a changed vertex enters; all
          // of them when the frontier overflowed
          ord.clear();
          if (have && !returned) {
            const uint64_t m = sr::frontier_pages(g, fr.data(), (int64_t)fr.size());
            for (int32_t i = 0; i < P; ++i)
              if (m >> (P <= 64 ? i : (int)((int64_t)i * 64 / P)) & 1ull) ord.push_back(i);
          } else {
            for (int32_t i = 0; i < P; ++i) ord.push_back(i);
          }
          R.st.pages_skipped += P - (int64_t)ord.size();
        }
      }
      pass++;
      if (pass > p.max_passes + 2) break;
    }
    HIP_TRY(c, hipStreamSynchronize(c->copy), "copy stream");
    R.harvest_events();
  }
  R.st.converged = R.st.stop_reason == SR_STOP_CONVERGED || R.st.stop_reason == SR_STOP_FP32_FLOOR;
  R.st.wall_ms = now_ms() - t0;
  if (stats) *stats = R.st;
  if (R.st.stop_reason == SR_STOP_MAX_PASSES || !done)
    return c->fail(SR_ENOTCONV, "max_passes reached before convergence");
  return SR_OK;
}

static_assert(SR_NOALLOC_SCRATCH_BYTES == NOALLOC_SCRATCH_BYTES, "header and kernels agree on the scratch size");

// Allocation-free variant of sr_run for a graph already resident on the
// device: the same sweep and close kernels, the vertex values and predictor
// states in the caller's device buffers, the control block and counter
// stripes in the static scratch array (its address looked up per device at
// context creation), the heavy-vertex accumulators those of the resident
// pages. No device memory, event or stream is created.
extern "C" sr_status sr_run_noalloc(sr_graph *g, const sr_run_params *params, uint32_t *values_dev,
                                    uint8_t *status_dev, sr_run_stats *stats) {
  if (!g || !params) return g ? g->ctx->fail(SR_EINVAL, "params is NULL") : SR_EINVAL;
  sr_ctx *c = g->ctx;
  if (c->host_only) return c->fail(SR_EDEVICE, "host-only context cannot run");
  if (!c->scratch_dev) return c->fail(SR_EDEVICE, "static scratch address unavailable on this device");
  if (g->server_refs > 0) return c->fail(SR_EBUSY, "graph is attached to a server");
  if (!values_dev) return c->fail(SR_EINVAL, "values_dev is NULL");
  const double t0 = now_ms();
  HIP_TRY(c, hipSetDevice(c->device), "set device");
  Runner R;
  R.g = g;
  R.c = c;
  R.timed = false;
  R.prm = *params;
  sr_run_params &p = R.prm;
  if (p.algo != SR_BFS && p.algo != SR_SSSP && p.algo != SR_CC)
    return c->fail(SR_EINVAL, "the allocation-free run serves BFS, SSSP and CC");
  R.algo = (int)p.algo;
  if (p.max_passes == 0) p.max_passes = 10000;
  if (p.max_passes < 0) return c->fail(SR_EINVAL, "negative limits");
  if (p.flags & ~(SR_RUN_AUDIT_PVU | SR_RUN_NO_EARLY_BREAK | SR_RUN_DETERMINISTIC))
    return c->fail(SR_EINVAL, "the allocation-free run takes SR_RUN_AUDIT_PVU, SR_RUN_NO_EARLY_BREAK and "
                              "SR_RUN_DETERMINISTIC only");
  if (p.pvu == SR_PVU_DEFAULT) p.pvu = (R.algo == A_SSSP) ? SR_PVU_WEAK : SR_PVU_STRONG;
  if (p.pvu < SR_PVU_OFF || p.pvu > SR_PVU_WEAK) return c->fail(SR_EINVAL, "unknown pvu mode");
  R.pvu = (int)p.pvu;
  if (R.pvu == P_WEAK && !status_dev) return c->fail(SR_EINVAL, "weak prediction needs status_dev");
  if (R.algo != A_CC && (p.source < 0 || p.source >= g->n)) return c->fail(SR_EINVAL, "source out of range");
  if (R.algo == A_CC && !g->symmetric)
    return c->fail(SR_EINVAL, "CC needs the undirected graph: load with SR_LOAD_SYMMETRIZE");
  if (R.algo == A_SSSP && !g->weighted) return c->fail(SR_EINVAL, "SSSP needs weights");
  if (g->reordered)
    return c->fail(SR_EINVAL, "the allocation-free run writes values in the caller's ids: load without "
                              "SR_LOAD_REORDER");
  R.weights = R.algo == A_SSSP;
  if (g->pages.empty() || !g->res.resident || (R.weights && !g->res.weights) || g->res.buf.empty())
    return c->fail(SR_ESTATE, "pages are not resident on the device: run sr_run on this graph first");
  sr_pvu_diagram d;
  if (p.diagram) d = *p.diagram; else sr_pvu_default_diagram(&d);
  if (!valid_diagram(d)) return c->fail(SR_EINVAL, "invalid predictor diagram");
  std::memset(&R.dia, 0, sizeof(R.dia));
  R.dia.num_states = d.num_states;
  R.dia.initial = d.initial_state;
  R.dia.attempt_mask = d.attempt_mask;
  std::memcpy(R.dia.succ, d.on_success, 8);
  std::memcpy(R.dia.fail, d.on_fail, 8);
  R.det = (p.flags & SR_RUN_DETERMINISTIC) != 0;

  // the state the kernels use: caller buffers and the static scratch
  RunState st;
  st.algo = R.algo;
  st.n = g->n;
  st.value = values_dev;
  st.status = status_dev;
  st.ctl = reinterpret_cast<Ctl *>(c->scratch_dev);
  st.stripes = reinterpret_cast<Stripe *>(reinterpret_cast<char *>(c->scratch_dev) + NOALLOC_CTL_BYTES);
  R.rs = &st;

  Ctl init;
  std::memset(&init, 0, sizeof(init));
  init.threshold = 0;
  init.phase = 0;
  init.pass_min_changed = INF;
  init.best_l1 = 1e300;
  init.algo = R.algo;
  init.pvu = R.pvu;
  init.max_passes = p.max_passes;
  init.tol_l1 = 1e-9;
  init.floor_cap = 1e-6;
  init.mass = 1.0;
  // every buffer is set by a kernel (no memset or copy nodes), in stream order
  hipError_t e = launch_init_min(R.algo, values_dev, g->n, p.source, c->compute);
  if (e == hipSuccess && status_dev) e = launch_fill_u8(status_dev, (uint8_t)d.initial_state, (size_t)g->n, c->compute);
  if (e == hipSuccess) e = launch_init_ctl(st.ctl, init, c->compute);
  if (e == hipSuccess) e = launch_init_stripes(st.stripes, c->compute);
  for (size_t i = 0; i < g->res.partial.size() && e == hipSuccess; ++i)
    e = launch_fill_u32((uint32_t *)g->res.partial[i], INF, 2 * g->res.partial_words[i], c->compute);
  if (e != hipSuccess) return c->hip_fail(e, "init");
  for (uint32_t i = 0; i < RING; ++i) c->ring_host[i].seq = ~0ull;
  g->sweeps.clear();
  R.seq_next = 0;

  // resident sweeps: each covers every page and closes a pass; batches of
  // sweeps are enqueued with one host check per batch (the control block
  // turns the sweeps after convergence into no-ops)
  std::vector<std::vector<int32_t>> groups;
  for (int32_t i = 0; i < (int32_t)g->pages.size(); i += MAXW) {
    std::vector<int32_t> grp;
    for (int32_t j = i; j < std::min<int32_t>(i + MAXW, (int32_t)g->pages.size()); ++j) grp.push_back(j);
    groups.push_back(grp);
  }
  std::vector<SweepArgs> args(groups.size());
  sr_status s;
  for (size_t k = 0; k < groups.size(); ++k)
    if ((s = R.make_args(groups[k], groups[k], k + 1 == groups.size() ? 1 : 0, args[k])) != SR_OK) return s;
  bool done = false;
  int32_t launched = 0;
  while (!done) {
    for (int b = 0; b < 4; ++b) {
      for (auto &a : args)
        if ((s = R.launch(a)) != SR_OK) return s;
      launched++;
    }
    if ((s = R.sync_compute()) != SR_OK) return s;
    R.harvest(&done);
    if (launched > p.max_passes + 8) break;
  }
  R.st.converged = R.st.stop_reason == SR_STOP_CONVERGED;
  R.st.wall_ms = now_ms() - t0;
  if (stats) *stats = R.st;
  if (R.st.stop_reason == SR_STOP_MAX_PASSES || !done)
    return c->fail(SR_ENOTCONV, "max_passes reached before convergence");
  return SR_OK;
}

extern "C" sr_status sr_probe_gather(sr_ctx *c, const uint32_t *src, int64_t m, uint32_t src_mask,
                                     const uint32_t *values, int32_t n, int32_t repeats, double *ms_per_launch,
                                     uint64_t *checksum) {
  if (!c) return SR_EINVAL;
  if (!src || !values || !ms_per_launch || !checksum || m < 1 || n < 1 || repeats < 1 ||
      (m + TILE_E - 1) / TILE_E > 0x7FFFFFFF)
    return c->fail(SR_EINVAL, "probe: null pointer or bad size");
  if (c->host_only) return c->fail(SR_EDEVICE, "host-only context has no device");
  HIP_TRY(c, hipSetDevice(c->device), "set device");
  unsigned long long *sink = nullptr;
  uint32_t *d_src = nullptr, *d_values = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto done = [&](sr_status st) {
    (void)hipStreamSynchronize(c->compute);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (sink) c->dfree(sink);
    if (d_src) c->dfree(d_src);
    if (d_values) c->dfree(d_values);
    return st;
  };
  sr_status s = c->dalloc((void **)&sink, 8, "probe checksum");
  if (s == SR_OK) s = c->dalloc((void **)&d_src, 4ull * (uint64_t)m, "probe words");
  if (s == SR_OK) s = c->dalloc((void **)&d_values, 4ull * (uint64_t)n, "probe values");
  if (s != SR_OK) return done(s);
  hipError_t e = hipMemcpyAsync(d_src, src, 4ull * (uint64_t)m, hipMemcpyHostToDevice, c->compute);
  if (e == hipSuccess) e = hipMemcpyAsync(d_values, values, 4ull * (uint64_t)n, hipMemcpyHostToDevice, c->compute);
  if (e == hipSuccess) e = launch_fill_u32((uint32_t *)sink, 0u, 2, c->compute);
  if (e == hipSuccess) e = launch_gather_probe(d_src, m, src_mask, d_values, n, sink, c->compute);
  unsigned long long sum = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&sum, sink, 8, hipMemcpyDeviceToHost, c->compute);
  if (e == hipSuccess) e = hipStreamSynchronize(c->compute);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) e = hipEventRecord(e0, c->compute);
  for (int32_t i = 0; i < repeats && e == hipSuccess; ++i)
    e = launch_gather_probe(d_src, m, src_mask, d_values, n, sink, c->compute);
  if (e == hipSuccess) e = hipEventRecord(e1, c->compute);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  if (e != hipSuccess) return done(c->hip_fail(e, "gather probe"));
  *ms_per_launch = (double)ms / repeats;
  *checksum = sum;
  return done(SR_OK);
}

extern "C" sr_status sr_run_sweeps(const sr_graph *g, sr_sweep_record *out, int32_t max, int32_t *count) {
  if (!g || !count || max < 0 || (max > 0 && !out)) return g ? g->ctx->fail(SR_EINVAL, "bad arguments") : SR_EINVAL;
  const int32_t n = (int32_t)g->sweeps.size();
  for (int32_t i = 0; i < std::min(n, max); ++i) out[i] = g->sweeps[i];
  *count = n;
  return SR_OK;
}

extern "C" sr_status sr_read_values(const sr_graph *g, void *dst, uint64_t bytes) {
  if (!g || !dst) return g ? g->ctx->fail(SR_EINVAL, "dst is NULL") : SR_EINVAL;
  sr_ctx *c = g->ctx;
  if (c->host_only) return c->fail(SR_EDEVICE, "host-only context has no values");
  if (!g->state.valid) return c->fail(SR_ESTATE, "no run has produced values");
  if (bytes < 4ull * g->n) return c->fail(SR_EINVAL, "dst_bytes < 4n");
  HIP_TRY(c, hipSetDevice(c->device), "set device");
  if (!g->reordered) {
    HIP_TRY(c, hipMemcpyAsync(dst, g->state.value, 4ull * g->n, hipMemcpyDeviceToHost, c->compute), "read values");
    HIP_TRY(c, hipStreamSynchronize(c->compute), "read values");
    return SR_OK;
  }
  // internal order to the caller's: dst[v] = value[rank[v]]
  std::vector<uint32_t> tmp((size_t)g->n);
  HIP_TRY(c, hipMemcpyAsync(tmp.data(), g->state.value, 4ull * g->n, hipMemcpyDeviceToHost, c->compute), "read values");
  HIP_TRY(c, hipStreamSynchronize(c->compute), "read values");
  uint32_t *out = (uint32_t *)dst;
  const int32_t *rk = g->rank.data();
  const int T = sr::host_threads();
  std::vector<std::thread> th;
  for (int t = 0; t < T; ++t)
    th.emplace_back([&, t] {
      const int64_t lo = (int64_t)g->n * t / T, hi = (int64_t)g->n * (t + 1) / T;
      for (int64_t v = lo; v < hi; ++v) out[v] = tmp[(size_t)rk[v]];
    });
  for (auto &x : th) x.join();
  return SR_OK;
}
