// mi_plan.hpp -- host side of the multi-instance sweep: groups of K
// instance columns over resident graphs, their work units, the persistent
// launch configuration and its HIP graph.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "batch.hpp"
#include "engine.hpp"

namespace sr {

struct MiPlan {
  sr_ctx *c = nullptr;
  int algo = A_PPR;   // A_PPR or A_SSSP (SSSP columns may run BFS)
  int K = 8;
  std::vector<MiGroup> groups;       // host mirror (device pointers inside)
  std::vector<sr_graph *> group_graph;
  std::vector<MiUnit> units;
  std::vector<int32_t> unit_prefix;
  MiGroup *d_groups = nullptr;
  MiUnit *d_units = nullptr;
  int32_t *d_prefix = nullptr;
  MiCtl *d_ctl = nullptr;
  uint32_t *h_remaining = nullptr;   // pinned, device-mapped
  uint32_t *d_remaining = nullptr;
  std::vector<void *> dev;           // device allocations owned by the plan
  std::vector<std::pair<sr_graph *, float *>> iod;  // 1/outdeg per graph (PPR)
  std::vector<std::pair<sr_graph *, int32_t *>> rank;  // caller -> internal ids (reordered graphs)
  std::vector<const int32_t *> group_rank;            // per group: device rank map or null
  MiArgs args{};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int grid_blocks = 0, grab = 1;
  int rounds = 4;                    // vertex rounds per wavefront and item (small-degree bins)
  bool narrow = false;               // SSSP/BFS values stored as 16 bits (set before add_group)
  bool tuned = false;
  float tuned_ms = 0.f;              // time of one sweep with the chosen schedule (when tuned)
  std::vector<PageHeader> unit_hdr;  // host copy of each unit's page header (bin counts)

  explicit MiPlan(sr_ctx *ctx, int algo_, int K_) : c(ctx), algo(algo_), K(K_) {}
  ~MiPlan();
  sr_status alloc(void **p, uint64_t bytes, const char *what);
  // a group of K columns over graph g (pages made resident by the caller)
  sr_status add_group(sr_graph *g, int pvu, int *out_index);
  // build units/prefix for all groups and upload the tables
  sr_status finalize(double damping, double tol_l1, int32_t max_sweeps);
  // (re)initialise column `col` of group `gi` and its control record; the
  // source is the caller's id (mapped for reordered graphs)
  // clean: the column already holds the initial value everywhere (SSSP/BFS
  // INF), so only the source entry is written
  sr_status set_column(int gi, int col, int32_t source, bool unit, bool active, hipStream_t s, bool clean = false);
  // every column of every group back to INF (SSSP/BFS plans)
  sr_status clear_values(hipStream_t s);
  sr_status set_remaining(uint32_t r, hipStream_t s);
  // work items per unit and bin for the current rounds (host tables)
  void prefix_tables();
  // work items per unit and bin for `rounds`, uploaded (the tables keep their size)
  sr_status set_rounds(int r);
  // pick rounds, grid size and grab by timing candidate sweeps (or take them
  // from the cache under `key`); restores nothing (callers re-initialise
  // their columns afterwards)
  // (only_rounds != 0: that rounds value alone)
  sr_status autotune(hipStream_t s, const std::string &key, int only_rounds = 0);
  sr_status launch(hipStream_t s);
  sr_status capture(hipStream_t s);
  sr_status replay(hipStream_t s, int times);
  uint64_t total_items() const { return unit_prefix.empty() ? 0 : (uint64_t)unit_prefix.back(); }
};

}  // namespace sr
