// mi_plan.cpp -- multi-instance plans (groups of K instance columns over
// resident graphs), the schedule autotuner, HIP-graph replay, and the
// sr_batch_run entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>

#include "kernels.hpp"
#include "mi_plan.hpp"

namespace sr {

namespace {
double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

std::mutex g_tune_mu;
// key -> chosen schedule: group width, vertex rounds per item, grid blocks, grab
struct Tuned { int K, rounds, grid, grab; };
std::map<std::string, Tuned> g_tune_cache;

void load_tune_file() {
  static bool loaded = false;
  if (loaded) return;
  loaded = true;
  const char *path = getenv("SR_TUNE_CACHE");
  if (!path) return;
  std::ifstream f(path);
  std::string line;
  // one entry per line: key K rounds grid grab
  while (std::getline(f, line)) {
    std::istringstream is(line);
    std::string key;
    Tuned t{};
    if (is >> key >> t.K >> t.rounds >> t.grid >> t.grab && t.grid > 0 && t.grab > 0 &&
        (t.rounds == 2 || t.rounds == 4 || t.rounds == 8) && (t.K == 8 || t.K == 16 || t.K == 32 || t.K == 64))
      g_tune_cache[key] = t;
  }
}

void save_tune_file() {
  const char *path = getenv("SR_TUNE_CACHE");
  if (!path) return;
  std::ofstream f(path, std::ios::trunc);
  for (auto &kv : g_tune_cache)
    f << kv.first << " " << kv.second.K << " " << kv.second.rounds << " " << kv.second.grid << " "
      << kv.second.grab << "\n";
}
}  // namespace

MiPlan::~MiPlan() {
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  for (auto p : dev) c->dfree(p);
  if (h_remaining) (void)hipHostFree(h_remaining);
}

sr_status MiPlan::alloc(void **p, uint64_t bytes, const char *what) {
  sr_status s = c->dalloc(p, bytes, what);
  if (s == SR_OK) dev.push_back(*p);
  return s;
}

sr_status MiPlan::add_group(sr_graph *g, int pvu, int *out_index) {
  MiGroup gr{};
  gr.n = g->n;
  gr.pvu = pvu;
  gr.has_w = (algo == A_SSSP && g->res.resident && g->res.weights) ? 1 : 0;
  gr.packed = g->packed ? 1 : 0;
  gr.src_mask = g->packed ? PACKED_SRC_MASK : 0xFFFFFFFFu;
  sr_status s;
  if (narrow && algo != A_SSSP) return c->fail(SR_EINVAL, "16-bit columns serve SSSP and BFS");
  // the sweep addresses a group's [n][K] arrays with 32-bit byte offsets
  if ((uint64_t)g->n * (uint64_t)K * 4ull >= (1ull << 32))
    return c->fail(SR_EINVAL, "graph too large for instance groups of this width (n * K * 4 bytes must stay below 4 GiB)");
  // 16-bit columns carry one more row: a sentinel of unreached values that
  // edge lanes past their range gather instead of being masked
  if ((s = alloc((void **)&gr.value, narrow ? 2ull * (g->n + 1) * K : 4ull * g->n * K, "instance values")) != SR_OK)
    return s;
  if (algo == A_PPR) {
    if ((s = alloc((void **)&gr.contrib, 4ull * g->n * K, "instance contrib")) != SR_OK) return s;
    float *iod = nullptr;
    for (auto &kv : this->iod)
      if (kv.first == g) iod = kv.second;
    if (!iod) {
      if ((s = alloc((void **)&iod, 4ull * g->n, "1/outdeg")) != SR_OK) return s;
      std::vector<float> h(g->n);
      for (int32_t v = 0; v < g->n; ++v) h[v] = g->outdeg[v] ? 1.0f / (float)g->outdeg[v] : 0.0f;
      hipError_t e = hipMemcpy(iod, h.data(), 4ull * g->n, hipMemcpyHostToDevice);
      if (e != hipSuccess) return c->hip_fail(e, "copy 1/outdeg");
      this->iod.push_back({g, iod});
    }
    gr.inv_outdeg = iod;
  }
  if ((s = alloc((void **)&gr.inst, sizeof(MiInst) * K, "instance control")) != SR_OK) return s;
  std::vector<MiInst> z(K);
  std::memset(z.data(), 0, sizeof(MiInst) * K);
  hipError_t e = hipMemcpy(gr.inst, z.data(), sizeof(MiInst) * K, hipMemcpyHostToDevice);
  if (e != hipSuccess) return c->hip_fail(e, "instance control init");
  const int32_t *rk = nullptr;
  if (g->reordered) {
    for (auto &kv : rank)
      if (kv.first == g) rk = kv.second;
    if (!rk) {
      int32_t *d = nullptr;
      if ((s = alloc((void **)&d, 4ull * g->n, "vertex order")) != SR_OK) return s;
      hipError_t e2 = hipMemcpy(d, g->rank.data(), 4ull * g->n, hipMemcpyHostToDevice);
      if (e2 != hipSuccess) return c->hip_fail(e2, "copy vertex order");
      rank.push_back({g, d});
      rk = d;
    }
  }
  group_rank.push_back(rk);
  groups.push_back(gr);
  group_graph.push_back(g);
  *out_index = (int)groups.size() - 1;
  return SR_OK;
}

sr_status MiPlan::finalize(double damping, double tol_l1, int32_t max_sweeps) {
  sr_status s;
  units.clear();
  unit_hdr.clear();
  unit_prefix.assign(1, 0);
  int32_t total_heavy = 0;
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    sr_graph *g = group_graph[gi];
    if (!g->res.resident) return c->fail(SR_EBUDGET, "batched graphs must be resident");
    for (size_t p = 0; p < g->pages.size(); ++p) {
      const PageHeader &h = g->pages[p].hdr;
      MiUnit u{};
      u.group = (int32_t)gi;
      u.page = g->res.buf[p];
      uint64_t nch = (uint64_t)std::max<int32_t>(h.n_chunks, 1);
      if ((s = alloc((void **)&u.acc, 8ull * nch * K, "heavy-vertex accumulators")) != SR_OK) return s;
      {
        // the reduction's identity: all ones (min; INF in the low word) or a
        // fixed-point zero (PageRank sums); the heavy kernel restores it
        std::vector<unsigned long long> idv(nch * K, algo == A_PPR ? 0ull : ~0ull);
        hipError_t e = hipMemcpy(u.acc, idv.data(), 8ull * nch * K, hipMemcpyHostToDevice);
        if (e != hipSuccess) return c->hip_fail(e, "accumulator init");
      }
      u.heavy_base = total_heavy;
      total_heavy += h.n_heavy;
      units.push_back(u);
      unit_hdr.push_back(h);
    }
  }
  if (units.empty()) return c->fail(SR_EINVAL, "no work units");
  prefix_tables();
  if ((int)groups.size() * K > MI_MAX_INSTANCES)
    return c->fail(SR_EINVAL, "too many instances in one call (at most " + std::to_string(MI_MAX_INSTANCES) + ")");
  if ((s = alloc((void **)&d_groups, sizeof(MiGroup) * groups.size(), "group table")) != SR_OK) return s;
  if ((s = alloc((void **)&d_units, sizeof(MiUnit) * units.size(), "unit table")) != SR_OK) return s;
  if ((s = alloc((void **)&d_prefix, 4ull * unit_prefix.size(), "unit prefix")) != SR_OK) return s;
  if ((s = alloc((void **)&d_ctl, sizeof(MiCtl), "batch control")) != SR_OK) return s;
  uint32_t *gact = nullptr;
  if ((s = alloc((void **)&gact, 4ull * groups.size(), "group activity")) != SR_OK) return s;
  hipError_t e = hipMemcpy(d_groups, groups.data(), sizeof(MiGroup) * groups.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(d_units, units.data(), sizeof(MiUnit) * units.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(d_prefix, unit_prefix.data(), 4ull * unit_prefix.size(), hipMemcpyHostToDevice);
  MiCtl z{};
  if (e == hipSuccess) e = hipMemcpy(d_ctl, &z, sizeof(z), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(gact, 0, 4ull * groups.size());
  void *hr = nullptr;
  if (e == hipSuccess) e = hipHostMalloc(&hr, 256, hipHostMallocMapped);
  if (e != hipSuccess) return c->hip_fail(e, "batch tables");
  h_remaining = (uint32_t *)hr;
  *h_remaining = 0;
  void *dr = nullptr;
  if (hipHostGetDevicePointer(&dr, hr, 0) != hipSuccess) dr = hr;
  d_remaining = (uint32_t *)dr;
  std::memset(&args, 0, sizeof(args));
  args.groups = d_groups;
  args.units = d_units;
  args.unit_prefix = d_prefix;
  args.ngroups = (int32_t)groups.size();
  args.nunits = (int32_t)units.size();
  args.total_items = unit_prefix.back();
  args.total_heavy = total_heavy;
  // one thread per instance column and run of MI_HEAVY_RUN heavy vertices
  const int64_t runs = ((int64_t)total_heavy + MI_HEAVY_RUN - 1) / MI_HEAVY_RUN;
  args.heavy_blocks = (int32_t)std::max<int64_t>(1, (runs * K + BLOCK - 1) / BLOCK);
  args.grab = 1;
  args.rounds = rounds;
  args.narrow = narrow ? 1 : 0;
  {
    // one weight mode for the whole plan lets the sweep kernel be compiled
    // for it alone (fewer registers than a kernel that chooses per item)
    int wm = -1;
    for (auto &gr : groups) {
      const int m = algo == A_SSSP && gr.has_w ? (gr.packed ? 1 : 2) : 0;
      wm = wm < 0 ? m : (wm == m ? wm : 3);
    }
    args.wmode = wm < 0 ? 0 : wm;
  }
  args.damping = damping;
  args.tol_l1 = tol_l1;
  args.floor_cap = 1e-6;
  args.max_sweeps = max_sweeps;
  args.tuning = 0;
  // last items first: the heavy chunks and high in-degree bins go out first
  // (the longest items start early, and the in-place sweep updates the
  // vertices most others pull from before they are read)
  args.descending = 1;
  args.ctl = d_ctl;
  args.group_active = gact;
  args.host_remaining = d_remaining;
  int dev = 0, cus = 256;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  grid_blocks = std::max(1, std::min(cus * 4, args.total_items));
  args.nblocks = grid_blocks;
  return SR_OK;
}

void MiPlan::prefix_tables() {
  unit_prefix.assign(1, 0);
  for (size_t i = 0; i < units.size(); ++i) {
    const PageHeader &h = unit_hdr[i];
    MiUnit &u = units[i];
    int32_t acc = 0;
    u.blk_prefix[0] = 0;
    for (int b = 0; b < NBINS; ++b) {
      // 16-bit columns run four per lane: the lane geometry of K/4 columns
      const int per = mi_items_per_block_host(b, narrow ? K / 4 : K, rounds);
      const int nb = (b == BIN_ZERO && algo != A_PPR) ? 0 : (h.bin_count[b] + per - 1) / per;
      acc += nb;
      u.blk_prefix[b + 1] = acc;
    }
    unit_prefix.push_back(unit_prefix.back() + acc);
  }
}

sr_status MiPlan::set_rounds(int r) {
  if (r != 2 && r != 4 && r != 8) return c->fail(SR_EINVAL, "rounds must be 2, 4 or 8");
  rounds = r;
  prefix_tables();
  hipError_t e = hipMemcpy(d_units, units.data(), sizeof(MiUnit) * units.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(d_prefix, unit_prefix.data(), 4ull * unit_prefix.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) return c->hip_fail(e, "schedule tables");
  args.rounds = r;
  args.total_items = unit_prefix.back();
  grid_blocks = std::max(1, std::min(grid_blocks, args.total_items));
  args.nblocks = grid_blocks;
  return SR_OK;
}

sr_status MiPlan::clear_values(hipStream_t s) {
  for (auto &gr : groups) {
    // (16-bit columns: two 0xFFFF entries per word)
    hipError_t e = launch_fill_u32(gr.value, INF, narrow ? (size_t)(gr.n + 1) * K / 2 : (size_t)gr.n * K, s);
    if (e != hipSuccess) return c->hip_fail(e, "column reset");
  }
  return SR_OK;
}

sr_status MiPlan::set_column(int gi, int col, int32_t source, bool unit, bool active, hipStream_t s, bool clean) {
  MiGroup &gr = groups[gi];
  sr_graph *g = group_graph[gi];
  if (source >= 0 && g->reordered) source = g->rank[source];
  MiInst in;
  std::memset(&in, 0, sizeof(in));
  in.active = active ? 1u : 0u;
  in.unit = unit ? 1u : 0u;
  in.source = source;
  in.threshold = 0;  // value 0 (the source) is final from the start
  in.sw_min_changed = INF;
  in.best_l1 = 1e300;
  in.last_l1 = -1.0;
  if (algo == A_PPR) {
    in.dangling = (source >= 0 && g->outdeg[source] == 0) ? 1.0 : 0.0;
    in.mass = 1.0;  // the column starts at e_source
  }
  hipError_t e = hipSuccess;
  if (source >= 0 && clean && algo != A_PPR && narrow)
    e = launch_mi_set_u16(gr.value, (size_t)source * K + col, 0u, s);
  else if (source >= 0 && clean && algo != A_PPR)
    e = launch_fill_u32(gr.value + (size_t)source * K + col, 0u, 1, s);
  else if (source >= 0)
    e = launch_mi_init_column(algo, K, gr.value, gr.contrib, gr.inv_outdeg, gr.n, col, source, s, narrow);
  if (e == hipSuccess) e = launch_mi_set_inst(gr.inst + col, in, s);
  if (e != hipSuccess) return c->hip_fail(e, "column init");
  return SR_OK;
}

sr_status MiPlan::set_remaining(uint32_t r, hipStream_t s) {
  // per-group activity and the total, recomputed from the host view
  MiCtl z{};
  z.remaining = r;
  hipError_t e = launch_mi_set_ctl(d_ctl, z, s);
  if (e != hipSuccess) return c->hip_fail(e, "control reset");
  return SR_OK;
}

sr_status MiPlan::launch(hipStream_t s) {
  hipError_t e = launch_mi_sweep(algo, K, args, s);
  if (e != hipSuccess) return c->hip_fail(e, "batched sweep launch");
  return SR_OK;
}

sr_status MiPlan::autotune(hipStream_t s, const std::string &key, int only_rounds) {
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_tune_file();
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end() && it->second.K == K) {
      const Tuned t = it->second;
      sr_status st = set_rounds(t.rounds);
      if (st != SR_OK) return st;
      grid_blocks = std::min(t.grid, std::max(1, args.total_items));
      grab = t.grab;
      args.nblocks = grid_blocks;
      args.grab = grab;
      tuned = false;
      return SR_OK;
    }
  }
  int dev = 0, cus = 256;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  // (16-bit columns run four per lane: 8 rounds of a lane's vertices would
  // hold more registers than the extra loads in flight are worth)
  std::vector<int> roundss = narrow ? std::vector<int>{2, 4} : std::vector<int>{2, 4, 8};
  if (only_rounds) roundss = {only_rounds};
  const int mults[] = {1, 2, 4, 8, 16};
  const int grabs[] = {1, 2, 4, 8};
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return c->fail(SR_EDEVICE, "event creation failed");
  float best = 1e30f;
  int best_grid = grid_blocks, best_grab = 1, best_rounds = rounds;
  args.tuning = 1;
  sr_status st = SR_OK;
  for (int rd : roundss) {
    if ((st = set_rounds(rd)) != SR_OK) break;
    for (int m : mults) {
      for (int gb : grabs) {
        int grid = std::max(1, std::min(cus * m, (args.total_items + gb - 1) / gb));
        args.nblocks = grid;
        args.grab = gb;
        if ((st = launch(s)) != SR_OK) break;  // warm
        (void)hipEventRecord(e0, s);
        for (int r = 0; r < 3; ++r)
          if ((st = launch(s)) != SR_OK) break;
        (void)hipEventRecord(e1, s);
        if (st != SR_OK) break;
        if (hipEventSynchronize(e1) != hipSuccess) { st = c->fail(SR_EDEVICE, "tuning sync"); break; }
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (ms < best) { best = ms; best_grid = grid; best_grab = gb; best_rounds = rd; }
      }
      if (st != SR_OK) break;
    }
    if (st != SR_OK) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  args.tuning = 0;
  if (st != SR_OK) return st;
  if ((st = set_rounds(best_rounds)) != SR_OK) return st;
  grid_blocks = best_grid;
  grab = best_grab;
  args.nblocks = grid_blocks;
  args.grab = grab;
  tuned = true;
  tuned_ms = best / 3.0f;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune_cache[key] = {K, rounds, grid_blocks, grab};
  save_tune_file();
  return SR_OK;
}

sr_status MiPlan::capture(hipStream_t s) {
  if (exec) return SR_OK;
  hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return c->hip_fail(e, "begin capture");
  hipError_t le = launch_mi_sweep(algo, K, args, s);
  e = hipStreamEndCapture(s, &graph);
  if (le != hipSuccess) return c->hip_fail(le, "captured launch");
  if (e != hipSuccess) return c->hip_fail(e, "end capture");
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) return c->hip_fail(e, "instantiate graph");
  return SR_OK;
}

sr_status MiPlan::replay(hipStream_t s, int times) {
  for (int i = 0; i < times; ++i) {
    hipError_t e = hipGraphLaunch(exec, s);
    if (e != hipSuccess) return c->hip_fail(e, "graph launch");
  }
  return SR_OK;
}

}  // namespace sr

using namespace sr;

extern "C" sr_status sr_batch_run(sr_ctx *c, const sr_instance *inst, int32_t count, const sr_run_params *common,
                                  void *const *dsts, sr_run_stats *per, sr_batch_stats *bst) {
  if (!c) return SR_EINVAL;
  if (!inst || count <= 0 || !dsts) return c->fail(SR_EINVAL, "need instances and destinations");
  if (c->host_only) return c->fail(SR_EDEVICE, "host-only context cannot run");
  const double t0 = now_ms();
  hipError_t he = hipSetDevice(c->device);
  if (he != hipSuccess) return c->hip_fail(he, "set device");
  const bool ppr = inst[0].algo == SR_PPR;
  for (int32_t i = 0; i < count; ++i) {
    const sr_instance &x = inst[i];
    if (!x.g || x.g->ctx != c) return c->fail(SR_EINVAL, "instance graph missing or from another context");
    if (ppr != (x.algo == SR_PPR)) return c->fail(SR_EINVAL, "mix PPR with SSSP/BFS in separate calls");
    if (x.algo != SR_PPR && x.algo != SR_SSSP && x.algo != SR_BFS)
      return c->fail(SR_EINVAL, "batched algorithms are PPR, SSSP and BFS");
    if (x.source < 0 || x.source >= x.g->n) return c->fail(SR_EINVAL, "source out of range");
    if (x.algo == SR_SSSP && !x.g->weighted) return c->fail(SR_EINVAL, "SSSP needs weights");
    if (dsts[i] == nullptr) return c->fail(SR_EINVAL, "null destination");
  }
  double damping = common && common->damping > 0 ? common->damping : 0.85;
  double tol = common && common->tol_l1 > 0 ? common->tol_l1 : 1e-9;
  int32_t max_sweeps = common && common->max_passes > 0 ? common->max_passes : 10000;
  int pvu = P_STRONG;
  if (common && common->pvu == SR_PVU_OFF) pvu = P_OFF;
  if (common && common->pvu == SR_PVU_WEAK) return c->fail(SR_EINVAL, "batched runs use OFF or STRONG prediction");
  if (ppr) pvu = P_OFF;
  // group instances by graph (first appearance order), K per group
  std::vector<sr_graph *> order;
  for (int32_t i = 0; i < count; ++i)
    if (std::find(order.begin(), order.end(), inst[i].g) == order.end()) order.push_back(inst[i].g);
  struct Slot { int group, col; };
  std::vector<Slot> where(count);
  sr_status s;
  for (sr_graph *g : order) {
    bool weights = false;
    for (int32_t i = 0; i < count; ++i) weights |= inst[i].g == g && inst[i].algo == SR_SSSP;
    if (g->server_refs > 0) return c->fail(SR_EBUSY, "graph is attached to a server");
    if (g->pages.empty())
      if ((s = sr_graph_partition(g, 1, 0)) != SR_OK) return s;
    if ((s = ensure_residency(g, weights, false, true)) != SR_OK) return s;
    if (!g->res.resident) return c->fail(SR_EBUDGET, "a batched graph does not fit the budget resident");
  }
  hipStream_t st = c->compute;
  // a plan of groups K columns wide over the graphs, every instance set
  auto build = [&](int K, std::unique_ptr<MiPlan> &out) -> sr_status {
    out.reset(new MiPlan(c, ppr ? A_PPR : A_SSSP, K));
    MiPlan &pl = *out;
    sr_status q;
    for (sr_graph *g : order) {
      int gi = -1, col = K;
      for (int32_t i = 0; i < count; ++i) {
        if (inst[i].g != g) continue;
        if (col == K) {
          if ((q = pl.add_group(g, pvu, &gi)) != SR_OK) return q;
          col = 0;
        }
        where[i] = {gi, col++};
      }
    }
    return pl.finalize(damping, tol, max_sweeps);
  };
  auto init_all = [&](MiPlan &pl) -> sr_status {
    std::vector<uint32_t> gact(pl.groups.size(), 0);
    for (size_t gi = 0; gi < pl.groups.size(); ++gi)
      for (int col = 0; col < pl.K; ++col) {
        // unused columns of a partial group stay inactive
        sr_status q = pl.set_column((int)gi, col, -1, false, false, st);
        if (q != SR_OK) return q;
      }
    for (int32_t i = 0; i < count; ++i) {
      sr_status q = pl.set_column(where[i].group, where[i].col, inst[i].source, inst[i].algo == SR_BFS, true, st);
      if (q != SR_OK) return q;
      gact[where[i].group]++;
    }
    hipError_t e = hipMemcpyAsync(pl.args.group_active, gact.data(), 4 * gact.size(), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return c->hip_fail(e, "group activity");
    sr_status q = pl.set_remaining((uint32_t)count, st);
    if (q != SR_OK) return q;
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return c->hip_fail(e, "batch init");
    return SR_OK;
  };
  // The schedule: group width K (instance columns sharing each gathered row),
  // vertex rounds per work item, grid size and grab, tuned by timing one
  // sweep over every instance and cached under the workload's signature:
  // the algorithm and, per graph, its scale bucket (ceil log2 n), edge
  // factor (m / n rounded) and instance count.
  std::string key;
  {
    std::vector<std::string> parts;
    for (sr_graph *g : order) {
      int per = 0;
      for (int32_t i = 0; i < count; ++i) per += inst[i].g == g;
      int sc = 0;
      while ((1ll << sc) < (long long)g->n) ++sc;
      const long long ef = g->n ? ((long long)g->m + g->n / 2) / g->n : 0;
      parts.push_back("s" + std::to_string(sc) + "e" + std::to_string(ef) + "x" + std::to_string(per));
    }
    std::sort(parts.begin(), parts.end());
    key = ppr ? "ppr" : "min";
    for (auto &x : parts) key += "_" + x;
  }
  std::vector<int> widths = ppr ? std::vector<int>{8, 16} : std::vector<int>{8, 16, 32};
  // SR_BATCH_SCHEDULE="K,rounds" fixes both (grid and grab still tuned)
  int force_rounds = 0;
  if (const char *fs = getenv("SR_BATCH_SCHEDULE")) {
    int fk = 0, fr = 0;
    if (std::sscanf(fs, "%d,%d", &fk, &fr) != 2 || std::find(widths.begin(), widths.end(), fk) == widths.end() ||
        (fr != 2 && fr != 4 && fr != 8))
      return c->fail(SR_EINVAL, "SR_BATCH_SCHEDULE must be \"K,rounds\" with a valid width and rounds 2, 4 or 8");
    widths = {fk};
    force_rounds = fr;
    key += "_forced" + std::to_string(fk) + "r" + std::to_string(fr);
  }
  if (!force_rounds) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_tune_file();
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end() && std::find(widths.begin(), widths.end(), it->second.K) != widths.end())
      widths = {it->second.K};
  }
  std::unique_ptr<MiPlan> best;
  int candidates = 0;
  for (int K : widths) {
    std::unique_ptr<MiPlan> pl;
    if ((s = build(K, pl)) != SR_OK) {
      // a wider plan that does not fit the budget is skipped
      if (s == SR_EBUDGET && best) continue;
      return s;
    }
    if ((s = init_all(*pl)) != SR_OK) return s;
    if ((s = pl->autotune(st, key, force_rounds)) != SR_OK) return s;
    candidates++;
    if (!best || (pl->tuned && best->tuned && pl->tuned_ms < best->tuned_ms)) best = std::move(pl);
  }
  MiPlan &plan = *best;
  const int K = plan.K;
  // the instance slots of the chosen plan (building the others overwrote them)
  {
    int gi = -1;
    for (sr_graph *g : order) {
      int col = K;
      for (int32_t i = 0; i < count; ++i) {
        if (inst[i].g != g) continue;
        if (col == K) { ++gi; col = 0; }
        where[i] = {gi, col++};
      }
    }
  }
  if (candidates > 1 || plan.tuned) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = {plan.K, plan.rounds, plan.grid_blocks, plan.grab};
    save_tune_file();
  }
  if ((s = init_all(plan)) != SR_OK) return s;
  if ((s = plan.capture(st)) != SR_OK) return s;
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  (void)hipEventRecord(e0, st);
  int replays = 0;
  const int chunk = 8;
  while (true) {
    if ((s = plan.replay(st, chunk)) != SR_OK) break;
    replays += chunk;
    he = hipStreamSynchronize(st);
    if (he != hipSuccess) { s = c->hip_fail(he, "batch replay"); break; }
    if (*(volatile uint32_t *)plan.h_remaining == 0) break;
    if (replays > max_sweeps + 2 * chunk) break;
  }
  (void)hipEventRecord(e1, st);
  (void)hipEventSynchronize(e1);
  float kms = 0;
  (void)hipEventElapsedTime(&kms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (s != SR_OK) return s;
  // results and per-instance records
  std::vector<std::vector<MiInst>> ih(plan.groups.size(), std::vector<MiInst>(K));
  for (size_t gi = 0; gi < plan.groups.size(); ++gi) {
    he = hipMemcpy(ih[gi].data(), plan.groups[gi].inst, sizeof(MiInst) * K, hipMemcpyDeviceToHost);
    if (he != hipSuccess) return c->hip_fail(he, "read instance control");
  }
  int32_t maxn = 0;
  for (auto *g : order) maxn = std::max(maxn, g->n);
  // one extraction pass per group (its K columns share each row)
  uint32_t *tmp = nullptr;
  if ((s = plan.alloc((void **)&tmp, 4ull * maxn * K, "extract buffer")) != SR_OK) return s;
  std::vector<int32_t> extracted_group(count, -1);
  bool all_conv = true;
  uint64_t algo_bytes = 0;
  int32_t dev_sweeps = 0;
  std::vector<int32_t> group_sweeps(plan.groups.size(), 0);
  for (int32_t i = 0; i < count; ++i) {
    const int gi = where[i].group;
    const MiGroup &gr = plan.groups[gi];
    if (extracted_group[i] < 0) {
      // every instance of this group: one pass, then all its copies
      MiExtract x{};
      for (int32_t j = i; j < count; ++j)
        if (where[j].group == gi) {
          x.col[x.count] = where[j].col;
          x.out[x.count] = tmp + (size_t)where[j].col * maxn;
          x.count++;
          extracted_group[j] = gi;
        }
      he = launch_mi_extract(K, gr.value, gr.n, x, st, false, 0u, plan.group_rank[gi], plan.narrow);
      for (int32_t j = i; j < count && he == hipSuccess; ++j)
        if (where[j].group == gi)
          he = hipMemcpyAsync(dsts[j], tmp + (size_t)where[j].col * maxn, 4ull * gr.n, hipMemcpyDeviceToHost, st);
      if (he == hipSuccess) he = hipStreamSynchronize(st);
      if (he != hipSuccess) return c->hip_fail(he, "batch results");
    }
    const MiInst &r = ih[where[i].group][where[i].col];
    all_conv &= r.done && (r.stop_reason == 1 || r.stop_reason == 2);
    dev_sweeps = std::max<int32_t>(dev_sweeps, (int32_t)r.sweeps);
    group_sweeps[where[i].group] = std::max<int32_t>(group_sweeps[where[i].group], (int32_t)r.sweeps);
    algo_bytes += r.edges_total * 4ull;  // one gathered value per scanned edge and instance
    if (per) {
      sr_run_stats &p = per[i];
      std::memset(&p, 0, sizeof(p));
      p.passes = (int32_t)r.sweeps;
      p.sweeps = (int32_t)r.sweeps;
      p.converged = r.done && (r.stop_reason == 1 || r.stop_reason == 2);
      p.stop_reason = (int32_t)r.stop_reason;
      p.edges_scanned = (int64_t)r.edges_total;
      p.final_l1 = r.last_l1;
      p.wall_ms = now_ms() - t0;
    }
  }
  // shared per-sweep streams: in-edge ids (and weights), offsets, bins,
  // read once per sweep per group while the group has a live instance
  for (size_t gi = 0; gi < plan.groups.size(); ++gi) {
    sr_graph *g = plan.group_graph[gi];
    const bool sep_w = plan.algo == A_SSSP && g->weighted && !g->packed;
    uint64_t per_sweep = (uint64_t)g->m * (sep_w ? 8 : 4) + 12ull * g->n;
    algo_bytes += per_sweep * (uint64_t)group_sweeps[gi];
  }
  if (bst) {
    std::memset(bst, 0, sizeof(*bst));
    bst->sweeps = dev_sweeps;
    bst->groups = (int32_t)plan.groups.size();
    bst->group_width = K;
    bst->grid_blocks = plan.grid_blocks;
    bst->grab = plan.grab;
    bst->tuned = plan.tuned ? 1 : 0;
    bst->rounds = plan.rounds;
    bst->width_candidates = candidates;
    bst->kernel_ms = kms;
    bst->wall_ms = now_ms() - t0;
    bst->algo_bytes = algo_bytes;
  }
  if (!all_conv) return c->fail(SR_ENOTCONV, "some instances hit the sweep cap");
  return SR_OK;
}
