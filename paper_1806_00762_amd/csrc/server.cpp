// server.cpp -- continuous-batching SSSP/BFS query server over resident
// graphs. Each graph owns one multi-instance group of K slot columns; a
// progress thread admits queued queries into free slots as soon as slots
// (and a result buffer) free up, runs one multi-instance sweep over every
// graph with live slots per iteration, and retires slots whose sweep changed
// nothing (the Table I strong conditions keep the skips exact), moving the
// column into a device result buffer that sr_server_poll copies to the
// caller. Queries admitted later simply start in their own column while
// older ones continue: no query waits for a batch boundary.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdio>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "mi_plan.hpp"

using namespace sr;

namespace {
double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

enum QState { Q_QUEUED = 0, Q_RUNNING = 1, Q_DONE = 2, Q_READING = 3 };

struct Query {
  int32_t graph;
  int32_t algo;
  int32_t source;
  double t_submit = 0, t_done = 0;
  int state = Q_QUEUED;
  int slot = -1;
  uint32_t *result = nullptr;  // device result buffer once done
};
}  // namespace

struct sr_server {
  sr_ctx *c = nullptr;
  std::vector<sr_graph *> graphs;
  MiPlan *plan = nullptr;
  int K = 8;
  std::vector<int> usable;                       // concurrent slots per graph
  std::vector<std::vector<uint64_t>> slot_ticket;  // per graph, per column (0 = free)
  std::vector<std::vector<uint32_t *>> free_results;  // device result buffers per graph
  std::unordered_map<uint64_t, Query> q;
  std::deque<uint64_t> queue;
  uint64_t next_ticket = 1;
  std::mutex mu;
  std::condition_variable cv;
  std::thread th;
  bool stop = false;
  hipStream_t stream = nullptr, poll_stream = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;  // around each sweep replay
  // an iteration's set-up (per-graph active counts, then the admissions),
  // staged in pinned memory and applied on the device by one launch
  uint32_t *h_setup = nullptr, *d_setup = nullptr;
  MiInst *h_inst = nullptr;  // pinned copy of every column's record, read after each sweep
  std::atomic<uint64_t> submitted{0}, completed{0}, sweeps{0}, fallbacks{0};
  double busy_ms = 0;
  double kernel_ms = 0;     // device time of the sweep replays
  uint64_t algo_bytes = 0;  // algorithmic bytes of the sweeps (see sr_server_stats)
  sr_status thread_error = SR_OK;
  std::string thread_msg;

  void progress();
  // exact completion on the host of a retired 16-bit column that overflowed
  sr_status complete_on_host(int gi, int32_t algo, uint32_t *result);
};

// A column stored as 16 bits holds exact values for every vertex whose
// distance (or level) is below the stored cap (2^15 - 1) and leaves the
// others unreached: a shortest path to a vertex that fits passes only
// through vertices that fit (weights are at least 1), and every stored value
// is the length of a real path. Pushing relaxations on the host from every reached vertex therefore
// reaches the exact least fixed point (the label-correcting push of the
// sparse stage). Rare: it needs a distance of at least 32767.
sr_status sr_server::complete_on_host(int gi, int32_t algo, uint32_t *result) {
  sr_graph *g = graphs[gi];
  const int32_t n = g->n;
  std::vector<uint32_t> caller((size_t)n), val((size_t)n);
  hipError_t e = hipMemcpyAsync(caller.data(), result, 4ull * n, hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return c->hip_fail(e, "overflow completion");
  for (int32_t v = 0; v < n; ++v) val[g->reordered ? g->rank[v] : v] = caller[v];
  std::vector<uint32_t> front;
  for (int32_t v = 0; v < n; ++v)
    if (val[v] != INF) front.push_back((uint32_t)v);
  build_out_csr(g);
  int32_t rounds = 0;
  sparse_push(g, algo == SR_BFS ? A_BFS : A_SSSP, val.data(), front.data(), (int64_t)front.size(), &rounds);
  for (int32_t v = 0; v < n; ++v) caller[v] = val[g->reordered ? g->rank[v] : v];
  e = hipMemcpyAsync(result, caller.data(), 4ull * n, hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return c->hip_fail(e, "overflow completion");
  fallbacks++;
  return SR_OK;
}

void sr_server::progress() {
  (void)hipSetDevice(c->device);
  const int G = (int)graphs.size();
  MiInst *ih = h_inst;
  MiAdmit *adm = reinterpret_cast<MiAdmit *>(h_setup + G);
  while (true) {
    bool any_active = false;
    int32_t nadm = 0;
    {
      std::unique_lock<std::mutex> lk(mu);
      // admission: FIFO, skipping queries whose graph has no free slot
      for (auto it = queue.begin(); it != queue.end();) {
        Query &qq = q[*it];
        int gi = qq.graph;
        int col = -1;
        int busy = 0;
        for (int k = 0; k < K; ++k) busy += slot_ticket[gi][k] != 0;
        if (busy < usable[gi] && !free_results[gi].empty())
          for (int k = 0; k < K; ++k)
            if (slot_ticket[gi][k] == 0) { col = k; break; }
        if (col < 0 || nadm >= MI_ADMIT_MAX) { ++it; continue; }
        qq.slot = col;
        qq.state = Q_RUNNING;
        qq.result = free_results[gi].back();
        free_results[gi].pop_back();
        slot_ticket[gi][col] = *it;
        // retired columns are left at INF, so admission writes the source only
        const sr_graph *gg = graphs[gi];
        adm[nadm].group = gi;
        adm[nadm].col = col;
        adm[nadm].source = gg->reordered ? gg->rank[qq.source] : qq.source;
        adm[nadm].unit = qq.algo == SR_BFS ? 1u : 0u;
        nadm++;
        it = queue.erase(it);
      }
      for (int gi = 0; gi < G; ++gi)
        for (int k = 0; k < K; ++k) any_active |= slot_ticket[gi][k] != 0;
      if (!any_active) {
        if (stop) break;
        cv.wait_for(lk, std::chrono::milliseconds(1));
        continue;
      }
    }
    const double t0 = now_ms();
    // device view of live slots: per-group counts and the total
    std::vector<uint32_t> gact(G, 0);
    uint32_t total = 0;
    {
      std::lock_guard<std::mutex> lk(mu);
      for (int gi = 0; gi < G; ++gi)
        for (int k = 0; k < K; ++k) {
          uint64_t t = slot_ticket[gi][k];
          if (t && q[t].state == Q_RUNNING) { gact[gi]++; total++; }
        }
    }
    for (int gi = 0; gi < G; ++gi) h_setup[gi] = gact[gi];
    hipError_t e = hipMemcpyAsync(d_setup, h_setup, 4ull * G + sizeof(MiAdmit) * (size_t)nadm, hipMemcpyHostToDevice,
                                  stream);
    if (e == hipSuccess)
      e = launch_mi_setup(plan->args.groups, d_setup, G, nadm, total, plan->args.ctl, plan->args.group_active, K,
                          plan->narrow, stream);
    if (e == hipSuccess) e = hipEventRecord(ev0, stream);
    if (e == hipSuccess && plan->launch(stream) != SR_OK) e = hipErrorUnknown;
    if (e == hipSuccess) e = hipEventRecord(ev1, stream);
    // the instance records into pinned memory right behind the sweep: one wait for both
    for (int gi = 0; gi < G && e == hipSuccess; ++gi)
      e = hipMemcpyAsync(&ih[(size_t)gi * K], plan->groups[gi].inst, sizeof(MiInst) * K, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    float sweep_ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&sweep_ms, ev0, ev1);
    if (e != hipSuccess) {
      std::lock_guard<std::mutex> lk(mu);
      thread_error = SR_EDEVICE;
      thread_msg = std::string("server sweep: ") + hipGetErrorString(e);
      break;
    }
    sweeps++;
    // algorithmic bytes: each live graph's edge words (and weights), offsets,
    // bin lists and own-value rows once per sweep; the gathered values are
    // counted per instance when it retires
    uint64_t shared_bytes = 0;
    for (int gi = 0; gi < G; ++gi)
      if (gact[gi]) {
        const sr_graph *g = graphs[gi];
        const bool sep_w = g->weighted && !g->packed;
        shared_bytes += (uint64_t)g->m * (sep_w ? 8 : 4) + 12ull * g->n;
      }
    // retire converged slots into their result buffers
    std::vector<std::pair<uint64_t, int>> finished;
    {
      std::lock_guard<std::mutex> lk(mu);
      for (int gi = 0; gi < G; ++gi)
        for (int k = 0; k < K; ++k) {
          uint64_t t = slot_ticket[gi][k];
          if (!t) continue;
          const MiInst &r = ih[(size_t)gi * K + k];
          if (r.done) finished.push_back({t, gi * K + k});
        }
      kernel_ms += sweep_ms;
      algo_bytes += shared_bytes;
      for (auto &f : finished) algo_bytes += ih[(size_t)f.second].edges_total * (plan->narrow ? 2ull : 4ull);
    }
    // one extraction pass per graph for all of its retiring columns (at most
    // MI_EXTRACT_MAX columns per pass)
    for (int gi = 0; gi < G && e == hipSuccess; ++gi) {
      std::vector<std::pair<int32_t, uint32_t *>> cols;
      {
        std::lock_guard<std::mutex> lk(mu);
        for (auto &f : finished)
          if (f.second / K == gi) cols.push_back({f.second % K, q[f.first].result});
      }
      for (size_t b = 0; b < cols.size() && e == hipSuccess; b += MI_EXTRACT_MAX) {
        MiExtract x{};
        for (size_t j = b; j < cols.size() && x.count < MI_EXTRACT_MAX; ++j) {
          x.col[x.count] = cols[j].first;
          x.out[x.count] = cols[j].second;
          x.count++;
        }
        e = launch_mi_extract(K, plan->groups[gi].value, plan->groups[gi].n, x, stream, true, INF,
                              plan->group_rank[gi], plan->narrow);
      }
    }
    if (!finished.empty() && e == hipSuccess) e = hipStreamSynchronize(stream);
    // 16-bit columns whose values did not all fit: completed exactly on the host
    for (auto &f : finished) {
      if (e != hipSuccess || !ih[(size_t)f.second].overflow) continue;
      int32_t algo;
      uint32_t *res;
      {
        std::lock_guard<std::mutex> lk(mu);
        algo = q[f.first].algo;
        res = q[f.first].result;
      }
      if (complete_on_host(f.second / K, algo, res) != SR_OK) e = hipErrorUnknown;
    }
    const double t1 = now_ms();
    {
      std::lock_guard<std::mutex> lk(mu);
      busy_ms += t1 - t0;
      for (auto &f : finished) {
        int gi = f.second / K, k = f.second % K;
        Query &qq = q[f.first];
        qq.state = Q_DONE;
        qq.t_done = t1;
        slot_ticket[gi][k] = 0;
        completed++;
      }
      if (e != hipSuccess) {
        thread_error = SR_EDEVICE;
        thread_msg = std::string("server retire: ") + hipGetErrorString(e);
        break;
      }
    }
  }
}

extern "C" sr_status sr_server_create(sr_ctx *c, sr_graph *const *graphs, int32_t ngraphs, uint64_t state_budget,
                                      int32_t max_slots, sr_server **out) {
  if (!c) return SR_EINVAL;
  if (!graphs || ngraphs < 1 || ngraphs > 8 || !out) return c->fail(SR_EINVAL, "need 1..8 graphs and out");
  if (max_slots != 8 && max_slots != 16 && max_slots != 32 && max_slots != 64)
    return c->fail(SR_EINVAL, "max_slots_per_graph must be 8, 16, 32 or 64");
  if (c->host_only) return c->fail(SR_EDEVICE, "host-only context cannot serve");
  hipError_t he = hipSetDevice(c->device);
  if (he != hipSuccess) return c->hip_fail(he, "set device");
  for (int i = 0; i < ngraphs; ++i)
    if (!graphs[i] || graphs[i]->ctx != c) return c->fail(SR_EINVAL, "graph missing or from another context");
  sr_server *s = new sr_server();
  s->c = c;
  s->K = max_slots;
  s->graphs.assign(graphs, graphs + ngraphs);
  auto fail = [&](sr_status st) {
    if (s->h_setup) (void)hipHostFree(s->h_setup);
    if (s->h_inst) (void)hipHostFree(s->h_inst);
    delete s->plan;
    delete s;
    return st;
  };
  sr_status st;
  for (auto *g : s->graphs) {
    if (g->pages.empty())
      if ((st = sr_graph_partition(g, 1, 0)) != SR_OK) return fail(st);
    if ((st = ensure_residency(g, g->weighted, false, true)) != SR_OK) return fail(st);
    if (!g->res.resident) return fail(c->fail(SR_EBUDGET, "served graphs must fit the budget resident"));
    if (g->server_refs > 0) return fail(c->fail(SR_EBUSY, "graph is attached to another server"));
  }
  // per graph: K slot columns (4 B per vertex each) plus result buffers;
  // the state budget decides how many queries each graph runs at once
  uint64_t col_bytes = 0, per_result = 0;
  // slot columns hold 16-bit values (exact: a column whose values do not all
  // fit is completed on the host when it retires)
  for (auto *g : s->graphs) { col_bytes += 2ull * g->n * s->K; per_result += 4ull * g->n; }
  if (state_budget && col_bytes + per_result > state_budget)
    return fail(c->fail(SR_EBUDGET, "state budget cannot hold the slot columns and one result per graph"));
  uint64_t left = state_budget ? state_budget - col_bytes : ~0ull;
  int R = (int)std::min<uint64_t>(s->K, left / std::max<uint64_t>(per_result, 1));
  s->plan = new MiPlan(c, A_SSSP, s->K);
  s->plan->narrow = true;
  for (auto *g : s->graphs) {
    int gi;
    if ((st = s->plan->add_group(g, P_STRONG, &gi)) != SR_OK) return fail(st);
  }
  if ((st = s->plan->finalize(0.85, 1e-9, 1 << 30)) != SR_OK) return fail(st);
  if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&s->poll_stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreate(&s->ev0) != hipSuccess || hipEventCreate(&s->ev1) != hipSuccess)
    return fail(c->fail(SR_EDEVICE, "stream creation failed"));
  {
    const size_t setup_bytes = 4ull * ngraphs + sizeof(MiAdmit) * MI_ADMIT_MAX;
    if (hipHostMalloc((void **)&s->h_setup, setup_bytes, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&s->h_inst, sizeof(MiInst) * (size_t)ngraphs * s->K, hipHostMallocDefault) != hipSuccess)
      return fail(c->fail(SR_ENOMEM, "pinned set-up buffers"));
    if ((st = s->plan->alloc((void **)&s->d_setup, setup_bytes, "set-up buffer")) != SR_OK) return fail(st);
  }
  s->usable.assign(ngraphs, R);
  s->slot_ticket.assign(ngraphs, std::vector<uint64_t>(s->K, 0));
  s->free_results.resize(ngraphs);
  for (int gi = 0; gi < ngraphs; ++gi) {
    for (int r = 0; r < R; ++r) {
      uint32_t *b = nullptr;
      if ((st = s->plan->alloc((void **)&b, 4ull * s->graphs[gi]->n, "result buffer")) != SR_OK) return fail(st);
      s->free_results[gi].push_back(b);
    }
    for (int k = 0; k < s->K; ++k)
      if ((st = s->plan->set_column(gi, k, -1, false, false, s->stream)) != SR_OK) return fail(st);
  }
  // the schedule autotuner times the multi-source sweep with every column live
  // (a solve from vertex 0 in each)
  {
    if ((st = s->plan->clear_values(s->stream)) != SR_OK) return fail(st);
    for (int gi = 0; gi < ngraphs; ++gi)
      for (int k = 0; k < s->K; ++k)
        if ((st = s->plan->set_column(gi, k, 0, false, true, s->stream)) != SR_OK) return fail(st);
    std::vector<uint32_t> gact(ngraphs, (uint32_t)s->K);
    if (hipMemcpyAsync(s->plan->args.group_active, gact.data(), 4ull * ngraphs, hipMemcpyHostToDevice, s->stream) != hipSuccess)
      return fail(c->fail(SR_EDEVICE, "server init"));
    if ((st = s->plan->set_remaining((uint32_t)(ngraphs * s->K), s->stream)) != SR_OK) return fail(st);
    char key[128];
    uint64_t m = 0;
    for (auto *g : s->graphs) m += (uint64_t)g->m;
    std::snprintf(key, sizeof(key), "serve_K%d_g%d_items%d_m%llu", s->K, ngraphs, s->plan->args.total_items / 64,
                  (unsigned long long)(m >> 20));
    if ((st = s->plan->autotune(s->stream, key)) != SR_OK) return fail(st);
    for (int gi = 0; gi < ngraphs; ++gi)
      for (int k = 0; k < s->K; ++k)
        if ((st = s->plan->set_column(gi, k, -1, false, false, s->stream)) != SR_OK) return fail(st);
    if ((st = s->plan->clear_values(s->stream)) != SR_OK) return fail(st);
    if (hipStreamSynchronize(s->stream) != hipSuccess) return fail(c->fail(SR_EDEVICE, "server init"));
  }
  for (auto *g : s->graphs) g->server_refs++;
  s->th = std::thread([s] { s->progress(); });
  *out = s;
  return SR_OK;
}

extern "C" sr_status sr_server_submit(sr_server *s, int32_t graph, sr_algo algo, int32_t source, uint64_t *ticket) {
  if (!s || !ticket) return SR_EINVAL;
  if (graph < 0 || graph >= (int32_t)s->graphs.size()) return SR_EINVAL;
  if (algo != SR_SSSP && algo != SR_BFS) return SR_EINVAL;
  sr_graph *g = s->graphs[graph];
  if (source < 0 || source >= g->n) return SR_EINVAL;
  if (algo == SR_SSSP && !g->weighted) return SR_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) return SR_ESTATE;
  if (s->thread_error != SR_OK) return s->thread_error;
  if (s->queue.size() >= (1u << 20)) return SR_EBUSY;
  uint64_t t = s->next_ticket++;
  Query qq;
  qq.graph = graph;
  qq.algo = algo;
  qq.source = source;
  qq.t_submit = now_ms();
  s->q[t] = qq;
  s->queue.push_back(t);
  s->submitted++;
  *ticket = t;
  s->cv.notify_one();
  return SR_OK;
}

extern "C" sr_status sr_server_poll(sr_server *s, uint64_t ticket, void *dst, uint64_t bytes, int *done,
                                    double *latency_ms) {
  if (!s || !done) return SR_EINVAL;
  uint32_t *res = nullptr;
  int32_t n = 0, gi = 0;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->q.find(ticket);
    if (it == s->q.end()) return SR_EINVAL;
    if (s->thread_error != SR_OK && it->second.state != Q_DONE) return s->thread_error;
    if (it->second.state != Q_DONE) { *done = 0; return SR_OK; }
    gi = it->second.graph;
    n = s->graphs[gi]->n;
    if (dst && bytes < 4ull * n) return SR_EINVAL;
    it->second.state = Q_READING;
    res = it->second.result;
    if (latency_ms) *latency_ms = it->second.t_done - it->second.t_submit;
  }
  hipError_t e = hipSuccess;
  if (dst) {
    (void)hipSetDevice(s->c->device);
    e = hipMemcpyAsync(dst, res, 4ull * n, hipMemcpyDeviceToHost, s->poll_stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->poll_stream);
  }
  std::lock_guard<std::mutex> lk(s->mu);
  s->free_results[gi].push_back(res);
  s->q.erase(ticket);
  s->cv.notify_one();
  if (e != hipSuccess) return SR_EDEVICE;
  *done = 1;
  return SR_OK;
}

extern "C" sr_status sr_server_stats_get(sr_server *s, sr_server_stats *o) {
  if (!s || !o) return SR_EINVAL;
  std::memset(o, 0, sizeof(*o));
  o->submitted = s->submitted;
  o->completed = s->completed;
  o->sweeps = s->sweeps;
  std::lock_guard<std::mutex> lk(s->mu);
  for (size_t i = 0; i < s->usable.size() && i < 8; ++i) o->slots_per_graph[i] = s->usable[i];
  o->busy_ms = s->busy_ms;
  o->narrow_fallbacks = s->fallbacks;
  o->kernel_ms = s->kernel_ms;
  o->algo_bytes = s->algo_bytes;
  return SR_OK;
}

extern "C" sr_status sr_server_destroy(sr_server *s) {
  if (!s) return SR_EINVAL;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->queue.clear();  // not yet admitted: dropped
    s->cv.notify_all();
  }
  if (s->th.joinable()) s->th.join();
  (void)hipSetDevice(s->c->device);
  (void)hipDeviceSynchronize();
  sr_status st = s->thread_error;
  if (s->stream) (void)hipStreamDestroy(s->stream);
  if (s->poll_stream) (void)hipStreamDestroy(s->poll_stream);
  if (s->ev0) (void)hipEventDestroy(s->ev0);
  if (s->ev1) (void)hipEventDestroy(s->ev1);
  if (s->h_setup) (void)hipHostFree(s->h_setup);
  if (s->h_inst) (void)hipHostFree(s->h_inst);
  delete s->plan;
  for (auto *g : s->graphs) g->server_refs--;
  delete s;
  return st;
}
