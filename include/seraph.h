/*
 * seraph.h -- C ABI of libseraph, an MI355X (gfx950) engine for Seraph's
 * method: repeated in-GPU pull iteration of resident in-edge subgraphs with
 * predictive vertex updating, while the next subgraph streams from pinned
 * host memory (Li, "Scaling Up Large-Scale Graph Processing for
 * GPU-Accelerated Heterogeneous Systems", arXiv 1806.00762).
 *
 * Conventions (all entry points):
 *   - Every function that can fail returns sr_status: 0 = SR_OK, < 0 = error.
 *     No C++ exception crosses the ABI. On error, out-parameters are left
 *     untouched and sr_ctx_last_error() holds a message for the context.
 *   - Pointers marked "host" must point to host memory; "device" to memory
 *     on the context's GPU. The caller owns every buffer it passes; the
 *     library copies what it keeps before returning (except where stated).
 *   - Handles are not thread-safe, except sr_server_submit / sr_server_poll,
 *     which may be called from any thread while the server runs.
 *   - Vertex ids are int32 in [0, n). Unreached vertices and unset values
 *     read back as SR_INF (BFS, SSSP) -- see sr_read_values.
 *   - All device memory the library allocates for a context is charged to
 *     the context's device budget; an allocation that would exceed it fails
 *     with SR_EBUDGET before any device call is made.
 */
#ifndef SERAPH_H
#define SERAPH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SR_ABI_VERSION 1
#define SR_INF 0xFFFFFFFFu

typedef enum {
  SR_OK = 0,
  SR_EINVAL = -1,    /* bad argument (null handle, id out of range, bad flags) */
  SR_ENOMEM = -2,    /* host allocation failed */
  SR_EBUDGET = -3,   /* device budget cannot hold what the call needs */
  SR_EDEVICE = -4,   /* HIP runtime error, or no device on a host-only context */
  SR_ENOTCONV = -5,  /* max_passes reached before convergence (values readable) */
  SR_ESTATE = -6,    /* call not valid in the handle's current state */
  SR_EBUSY = -7      /* server queue full / resource in use */
} sr_status;

/* Vertex programs. BFS, CC and SSSP are the evaluated algorithms (Section 5.1);
 * PageRank is named in Section 4.3 and defined here as
 *   x[v] = (1-d) t[v] + d (sum_{u->v} x[u]/outdeg(u) + D t[v]),
 *   D = sum of x over vertices without out-edges,
 * with t uniform (SR_PAGERANK) or the unit vector of `source` (SR_PPR). */
typedef enum { SR_BFS = 0, SR_SSSP = 1, SR_CC = 2, SR_PAGERANK = 3, SR_PPR = 4 } sr_algo;

/* Predictive vertex updating (Section 4). STRONG uses the Table I
 * thresholds (BFS, SSSP, CC only); WEAK uses the state-transition diagram of
 * Section 4.3 / Fig. 6; DEFAULT picks STRONG for BFS and CC and WEAK for SSSP
 * and PageRank, as the paper evaluates them (Section 4.3 Discussion, 5.1),
 * except STRONG for SSSP under SR_RUN_HETERO or SR_RUN_SKIP_CLEAN. */
typedef enum { SR_PVU_OFF = 0, SR_PVU_STRONG = 1, SR_PVU_WEAK = 2, SR_PVU_DEFAULT = 3 } sr_pvu_mode;

/* sr_graph_load_csr flags */
#define SR_LOAD_SYMMETRIZE 0x1u  /* build in-edges of the undirected graph (needed for CC) */
#define SR_LOAD_SYMMETRIC 0x2u   /* the input is already symmetric with sorted rows: in-edges =
                                    out-edges; verified (SR_EINVAL if not), marks the graph undirected */
#define SR_LOAD_REORDER 0x4u     /* renumber vertices internally by descending in-degree (total
                                    degree when symmetrized), ties by id: hubs share the first pages
                                    and cache lines. Sources, results and CC labels stay in the
                                    caller's ids (CC labels: smallest caller id of the component);
                                    page views show internal ids (sr_graph_order maps them). */

/* sr_run_params.flags */
#define SR_RUN_AUDIT_PVU 0x1u     /* also evaluate skipped vertices; count would-be changes
                                     (mispredictions) without applying them */
#define SR_RUN_FORCE_STREAM 0x2u  /* stream pages through slots even if the graph fits */
#define SR_RUN_RESUME 0x4u        /* continue from the values/state left by the last run */
#define SR_RUN_FIXED_INNER 0x8u   /* every window step runs exactly max_inner_iters sweeps; with
                                     num_slots = 2 this is CLIP's loaded-data re-entry (Section 3.2),
                                     with max_inner_iters = 1 the single-pass baseline of Section 5.4 */
#define SR_RUN_HETERO 0x10u       /* heterogeneous model of Section 3.1 (BFS/SSSP/CC): once a pass
                                     changes at most sparse_switch vertices, the host continues with
                                     push relaxations from that pass's frontier (the sparse stage).
                                     With weak prediction the switch first runs one verification
                                     pass (prediction off: the all-pull of Section 4.3) and hands
                                     over that pass's frontier. When the host's frontier grows past
                                     sparse_return vertices, the run returns to the device passes
                                     (the switch taken back to dense); otherwise the host reaches
                                     the fixed point and ends the run. Streamed runs under strong
                                     prediction also enter the host stage from the other side: after
                                     a pass whose changed set is too large, the device lists the
                                     vertices the next pass would attempt (an in-edge and a value
                                     above the Table I threshold); when at most sparse_switch, the
                                     host pulls them from its copy of the in-edges and pushes from
                                     those that changed, instead of streaming every page again */
#define SR_RUN_SKIP_CLEAN 0x20u   /* streamed min programs (strong or no prediction): a pass copies
                                     and sweeps only the pages with an in-edge from a vertex that
                                     changed in the previous pass (the others are at their local
                                     fixed point); falls back to every page when that pass changed
                                     more vertices than the frontier holds (n / 16 entries, fewer if
                                     the device budget has less room) */
#define SR_RUN_NO_EARLY_BREAK 0x40u /* BFS with strong prediction reads a vertex's first in-edge
                                     first and, when that neighbour is on the threshold level k of
                                     Table I, sets level k + 1 without reading the other in-edges
                                     (the dense-pull early break of Section 5.5, RQ4); this flag
                                     turns it off (results are identical either way) */
#define SR_RUN_WIDE_PAGES 0x80u   /* streamed BFS/SSSP/CC copy split-width page images by default:
                                     in-edges from source ids below 2^16 stored as u16 ids (u8
                                     weights) ahead of the others, so fewer bytes cross the host
                                     link per page (Section 3.1's streamed pages; built once, in
                                     pinned memory, on the first such run, and used when each image
                                     fits a slot and all of them are smaller than the full-width
                                     pages; when the pinned images cannot be allocated the run
                                     copies the full-width pages); this flag copies the full-width
                                     pages instead (results are identical either way) */
#define SR_RUN_SPLIT_PAGES 0x100u /* copy the split-width images even when they are not smaller
                                     (SR_EINVAL for PageRank, resident graphs, graphs whose edge
                                     words are not packed, or together with SR_RUN_WIDE_PAGES;
                                     SR_EBUDGET when an image exceeds a slot) */
#define SR_RUN_DETERMINISTIC 0x200u /* PageRank / PPR: bit-reproducible results. Each sweep reads a
                                     snapshot of the gathered terms (rank / out-degree as they were
                                     when the sweep started: Jacobi within a sweep, Gauss-Seidel
                                     between the sweeps of a window) and sums every vertex's in-edge
                                     terms in 2^-54 fixed point, which adds exactly in any order;
                                     a streamed window is re-swept up to max_inner_iters times or
                                     until a sweep changes nothing, never "until the next page has
                                     landed" (a timing-dependent rule). Costs 4 bytes per vertex of
                                     device memory (the snapshot's second buffer) and one copy of
                                     the window's terms per sweep. Min programs (BFS, SSSP, CC)
                                     reach their unique fixed point in any order, so this flag only
                                     fixes their schedule. */

#define SR_RUN_PR_DELTA 0x400u   /* PageRank / PPR as PageRank-delta, the data-driven form of Section
                                     4.3: every vertex keeps a residual (received rank mass not yet
                                     applied), starting at (1 - d) t with ranks at 0. In each pass a
                                     vertex adds the terms d r_u / outdeg(u) its in-neighbours sent in
                                     the previous pass (and d t_v times the mass sent by vertices
                                     without out-edges); when the residual exceeds pr_change_eps it
                                     applies it to its rank and sends it (a valid update in Fig. 6),
                                     otherwise it keeps it. Passes are Jacobi (each page swept once
                                     per pass; the sent terms live in a second buffer, 4 B per
                                     vertex, plus 4 B per vertex of residuals). With weak prediction
                                     a dormant vertex drops the terms of the passes it skips. When a
                                     pass's applied mass falls below tol_l1 (or stalls below 1e-6),
                                     the run turns its ranks into rank-form terms and ends with the
                                     plain verification passes of PageRank, which recover every
                                     dropped or unsent residual. OFF or WEAK prediction; excludes
                                     SR_RUN_DETERMINISTIC, SR_RUN_RESUME and SR_RUN_AUDIT_PVU */

/* stop reasons reported in sr_run_stats.stop_reason */
#define SR_STOP_CONVERGED 1   /* min programs: a full pass changed nothing (with weak prediction,
                                 a verification pass without prediction), or the host sparse stage
                                 reached the fixed point; PageRank: the L1 change of a pass without
                                 prediction fell below tol_l1 */
#define SR_STOP_FP32_FLOOR 2  /* PageRank: L1 stalled below 1e-6 for 3 full passes */
#define SR_STOP_MAX_PASSES 3

typedef struct sr_ctx sr_ctx;
typedef struct sr_graph sr_graph;
typedef struct sr_server sr_server;

/* ---------------------------------------------------------------- context */

/* Create a context on HIP device `device` with a device-memory budget in
 * bytes (0 = the device's free memory). The budget models the paper's
 * setting (Section 1, Section 3.1): the graph lives in host memory, while
 * GPU memory holds the vertex data and only as many subgraph pages as fit,
 * so a budget below the graph size makes every pass stream its pages.
 * Every device byte the library allocates for the context (vertex state,
 * page slots, work lists, scratch) is charged to it. device = -1 creates a
 * host-only context: graphs can be loaded, partitioned and inspected, but
 * sr_run and every other device call return SR_EDEVICE. *out receives the
 * handle; the caller destroys it with sr_ctx_destroy. */
sr_status sr_ctx_create(int device, uint64_t device_budget_bytes, sr_ctx **out);
void sr_ctx_destroy(sr_ctx *ctx);
/* Message of the last error on this context ("" if none). Valid until the
 * next call on the context. ctx may be NULL (then: last sr_ctx_create error). */
const char *sr_ctx_last_error(const sr_ctx *ctx);
/* Use caller-owned hipStream_t handles (e.g. torch.cuda streams) for compute
 * and for host-to-device page copies. NULL restores the library's own
 * streams. The streams must outlive their use by the context. */
sr_status sr_ctx_set_streams(sr_ctx *ctx, void *compute_stream, void *copy_stream);
/* Device memory from the caller, e.g. PyTorch's caching allocator. When set,
 * every device allocation the library makes for this context afterwards
 * calls alloc(bytes, user), which returns device memory of the context's
 * GPU aligned to 256 bytes (NULL = out of memory, reported as SR_ENOMEM),
 * and hands it back with release(ptr, user) once the library is done with
 * it (after the device work that used it has finished). Allocations stay
 * charged to the device budget. Memory obtained before the call is still
 * released the way it was obtained. alloc = NULL restores hipMalloc (release
 * and user are then ignored). Both functions must stay callable until the
 * context is destroyed; they are called from the thread that makes the
 * library call that needs the memory. SR_EINVAL: alloc without release;
 * SR_EDEVICE: a host-only context. */
typedef void *(*sr_alloc_fn)(size_t bytes, void *user);
typedef void (*sr_release_fn)(void *ptr, void *user);
sr_status sr_ctx_set_allocator(sr_ctx *ctx, sr_alloc_fn alloc, sr_release_fn release, void *user);
/* Device bytes currently charged to the budget, and the budget itself. */
sr_status sr_ctx_memory(const sr_ctx *ctx, uint64_t *used_bytes, uint64_t *budget_bytes);

/* ------------------------------------------------------------------ graph */

/* Load G = (V, E, w) given as an OUT-edge CSR on the host: the heads of the
 * arcs leaving u are col_idx[row_offsets[u] .. row_offsets[u+1]-1], weights
 * (may be NULL = unweighted) aligned with col_idx. n >= 1, m >= 0,
 * row_offsets[0] = 0, row_offsets[n] = m, non-decreasing, col_idx in [0,n).
 * The library keeps the graph the way the paper does (Section 3.1, Subgraph
 * Organization): as in-edges (CSC, i.e. the CSR of the transpose), later cut
 * into pages of consecutive destination vertices. With SR_LOAD_SYMMETRIZE
 * the in-edges of the undirected graph (arcs in both directions, duplicates
 * removed) are kept instead. Out-degrees of the input are kept for PageRank.
 * Inputs are copied; the caller may free them on return. */
sr_status sr_graph_load_csr(sr_ctx *ctx, int32_t n, int64_t m, const int64_t *row_offsets,
                            const int32_t *col_idx, const uint32_t *weights, uint32_t flags,
                            sr_graph **out);

/* Cut the in-edge CSR into pages (Section 3.1: CSC pages of consecutive
 * destination vertices with their incoming edges, no destination array).
 * Pages carry about equal streamed bytes (4 per vertex offset plus 4 per
 * edge word, 8 with separate weights); a vertex is never split across
 * pages, so a page may exceed the share by one vertex. num_parts = 0 picks
 * the smallest count whose largest page fits a slot of the context's
 * budget; num_slots (2..17, 0 = 4) is the number of page slots of the
 * pipelined window (Section 3.2: num_slots - copy_depth pages computed while
 * copy_depth pages are copied). Pages live in pinned host memory owned by
 * the graph. */
sr_status sr_graph_partition(sr_graph *g, int32_t num_parts, int32_t num_slots);
/* sr_graph_partition_ex flags */
#define SR_PART_EQUAL_EDGES 0x1u  /* boundary i is the first vertex whose in-edges start at or after
                                     ceil(i * m / num_parts) (equal in-edge counts rather than equal
                                     streamed bytes; a vertex still never straddles two pages, and
                                     empty ranges are dropped, so fewer pages can result) */
/* sr_graph_partition with flags (0 = the equal-byte split above). */
sr_status sr_graph_partition_ex(sr_graph *g, int32_t num_parts, int32_t num_slots, uint32_t flags);

typedef struct {
  int32_t n;
  int64_t m;                 /* in-edges kept (after symmetrization) */
  int32_t weighted;
  int32_t symmetric;         /* loaded with SR_LOAD_SYMMETRIZE */
  int32_t num_parts;         /* 0 before sr_graph_partition */
  int32_t num_slots;
  uint64_t graph_bytes;      /* in-CSR bytes: 4(n+1) + 4m (+ 4m weights) */
  uint64_t page_bytes_total; /* sum of page buffer bytes (incl. work lists) */
  uint64_t max_page_bytes;
  int32_t resident;          /* pages currently resident on the device */
  int32_t reordered;         /* loaded with SR_LOAD_REORDER */
} sr_graph_info;
/* Fill *out (host) with the graph's sizes and partition. Named with a _get
 * suffix because C does not allow a function and a typedef to share the
 * name sr_graph_info. */
sr_status sr_graph_info_get(const sr_graph *g, sr_graph_info *out);

/* Read-only view of page `page` (host pointers into the graph's pinned
 * pages; valid until the graph is repartitioned or destroyed). offsets are
 * rebased to 0 (n_p + 1 entries); src holds one 32-bit word per in-edge.
 * When every weight of the graph is below 256 and n <= 2^24, the weight is
 * packed into the edge word (lossless; 4 instead of 8 bytes per weighted
 * edge to stream): src_packed = 1, word = source | weight << 24, weights =
 * NULL. Otherwise src holds the source id and weights (uint32) follow. */
typedef struct {
  int32_t v_begin, v_end;    /* destination vertex range [v_begin, v_end) */
  int64_t num_edges;
  const int32_t *offsets;
  const uint32_t *src;       /* source id, or source | weight << 24 when src_packed */
  const uint32_t *weights;   /* NULL if unweighted or packed */
  int32_t src_packed;        /* 1: weights live in the top byte of src */
  uint64_t bytes;            /* bytes of the page buffer */
  uint64_t stream_bytes;     /* prefix a single-instance sweep copies (with weights) */
} sr_page_view;
sr_status sr_graph_page(const sr_graph *g, int32_t page, sr_page_view *out);
/* Vertex numbering of a graph loaded with SR_LOAD_REORDER (host arrays of n
 * entries, either may be NULL): internal_of[v] = internal id of the caller's
 * vertex v; caller_of[i] = caller's id of internal vertex i. SR_ESTATE if
 * the graph was loaded without reordering. */
sr_status sr_graph_order(const sr_graph *g, int32_t *internal_of, int32_t *caller_of);
void sr_graph_destroy(sr_graph *g);

/* -------------------------------------------------------------------- run */

/* Weak-predictor state diagram (Section 4.3: user-defined, the engine's
 * input). States 0..num_states-1 (<= 8); bit i of attempt_mask set = state i
 * attempts an update; an attempting state moves to on_success[i] if the
 * value changed and on_fail[i] otherwise; a dormant state always moves to
 * on_fail[i]. Every state must lead back to an attempting state. */
typedef struct {
  uint8_t num_states, initial_state, attempt_mask;
  uint8_t on_success[8], on_fail[8];
} sr_pvu_diagram;

/* The default diagram: attempt states {0,1,5}, dormant {2,3,4}; 0 -ok-> 0,
 * 0 -fail-> 5, 5 -ok-> 0, 5 -fail-> 3, 3 -> 2 -> 1, 1 -ok-> 0, 1 -fail-> 4,
 * 4 -> 3 (the text of Section 4.3; the 4 -> 3 edge is a reading of Fig. 6). */
sr_status sr_pvu_default_diagram(sr_pvu_diagram *out);

typedef struct {
  sr_algo algo;
  int32_t source;            /* BFS/SSSP source, PPR seed; ignored otherwise */
  double damping;            /* PageRank d (0 = 0.85) */
  double tol_l1;             /* PageRank stop: L1 change of a full pass (0 = 1e-9) */
  int32_t max_passes;        /* 0 = 10000 */
  int32_t max_inner_iters;   /* sweeps of a window before it slides (Section 3.2 re-entry bound); 0 = 4 */
  sr_pvu_mode pvu;
  const sr_pvu_diagram *diagram; /* NULL = default diagram */
  float pr_change_eps;       /* PageRank: |new-old| > eps counts as a valid update */
  uint32_t flags;            /* SR_RUN_* */
  int32_t copy_depth;        /* streamed pages: copies kept in flight ahead of the window (0 = 1,
                                the paper's S-1 computing + 1 transferring slots); with depth D
                                the window holds num_slots - D pages. 1 <= D < num_slots. */
  int32_t sparse_switch;     /* SR_RUN_HETERO: frontier size that switches to the host sparse
                                stage (0 = max(1024, n / 512)) */
  int32_t sparse_return;     /* SR_RUN_HETERO: host frontier size that sends the run back to the
                                device (0 = 32 * sparse_switch) */
} sr_run_params;

typedef struct {
  int32_t passes, sweeps, verify_passes, converged, stop_reason;
  int64_t edges_scanned;     /* in-edges read by attempted vertices */
  int64_t vertices_attempted, vertices_skipped, mispredicted;
  uint64_t h2d_bytes;        /* page bytes copied host -> device */
  double kernel_ms;          /* summed time of the sweep kernels and the kernels closing each sweep
                                (HIP events) */
  double h2d_ms;             /* summed page-copy time (HIP events) */
  double wall_ms;            /* host wall time of sr_run */
  double final_l1;           /* PageRank: L1 change of the last full pass */
  int64_t state_hist[8];     /* weak predictor: vertex-sweeps spent in each state */
  uint64_t algo_bytes;       /* algorithmic bytes of all sweeps: edge words, gathered values,
                                offsets, gate reads, value writes */
  int32_t sparse_stage;      /* SR_RUN_HETERO: 1 if the host sparse stage finished the run */
  int32_t sparse_rounds;     /* pull and push rounds of the sparse stage (all entries) */
  int64_t sparse_frontier;   /* vertices its last entry started from (changed in the last device pass,
                                or the vertices the next pass would have attempted) */
  int64_t sparse_relaxations;/* edges it relaxed (all entries) */
  double sparse_ms;          /* its wall time, transfers included (all entries) */
  int64_t pages_skipped;     /* SR_RUN_SKIP_CLEAN: page visits left out because no in-edge changed */
  double sweep_kernel_ms;    /* the part of kernel_ms spent in the sweep kernels alone (without the
                                kernels that close each sweep) */
  int64_t edges_narrow;      /* of edges_scanned, those read as u16 ids from split-width pages (0 when
                                the run copied full-width pages) */
  int32_t sparse_entries;    /* SR_RUN_HETERO: times the run switched to the host stage */
  int32_t sparse_returns;    /* ... and times the host stage gave the run back to the device */
  int32_t pr_delta_passes;   /* SR_RUN_PR_DELTA: passes of the residual phase */
  int32_t sweep_launches;    /* launches of the sweep kernel, including those of a window that had
                                already stopped changing (they exit at once and count no sweep) */
  uint64_t sparse_copy_bytes;/* SR_RUN_HETERO: vertex-value bytes the host stage copied between host
                                and device, both ways (lists and ids not counted; all entries) */
} sr_run_stats;

/* Run a vertex program to convergence on the graph (partitioned with
 * defaults if it was not). Pages are resident when the graph fits the
 * budget and SR_RUN_FORCE_STREAM is not set, otherwise they stream through
 * the slot window with up to max_inner_iters sweeps per window (Section
 * 3.2). Returns SR_ENOTCONV if max_passes ran out (values stay readable).
 * stats may be NULL. */
sr_status sr_run(sr_graph *g, const sr_run_params *params, sr_run_stats *stats);

/* Allocation-free solve, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): sr_run for BFS, SSSP or CC on a graph whose pages are already
 * resident on the device (an earlier sr_run made them resident: the graph
 * fits the budget and it ran without SR_RUN_FORCE_STREAM; SSSP needs pages
 * made resident by an SSSP run, since other programs copy no weights). The
 * graph must be loaded without SR_LOAD_REORDER, so the values are in the
 * caller's vertex ids.
 *   values_dev: device memory owned by the caller, 4n bytes: receives the
 *     u32 values (levels, distances or labels; SR_INF if unreached).
 *   status_dev: device memory owned by the caller, n bytes, the weak
 *     predictor's per-vertex states (workspace, contents undefined on
 *     return); may be NULL unless the predictor is weak (SR_PVU_DEFAULT
 *     resolves to weak for SSSP).
 * The control block and the counter stripes live in a static device array
 * of SR_NOALLOC_SCRATCH_BYTES that each GPU holds from library load to
 * process end; the heavy-vertex accumulators are the resident pages' own.
 * No device memory, event or stream is created and nothing is freed; the
 * call synchronises the context's compute stream. Every call on one GPU
 * shares that GPU's scratch array, and calls on one graph share its
 * accumulators, so calls that overlap on one GPU race (run them one at a
 * time). params as for sr_run; flags other than SR_RUN_AUDIT_PVU,
 * SR_RUN_NO_EARLY_BREAK and SR_RUN_DETERMINISTIC are refused; stats (may be
 * NULL) has no kernel timings. The values sr_read_values returns stay those
 * of the last sr_run. Errors: SR_EINVAL (bad argument, a reordered graph,
 * PageRank, a refused flag, status_dev NULL under weak prediction),
 * SR_ESTATE (pages not resident), SR_EBUSY (graph attached to a server),
 * SR_EDEVICE (host-only context, no scratch address, HIP error),
 * SR_ENOTCONV (max_passes ran out; values_dev holds the partial values). */
#define SR_NOALLOC_SCRATCH_BYTES 16384u
sr_status sr_run_noalloc(sr_graph *g, const sr_run_params *params, uint32_t *values_dev, uint8_t *status_dev,
                         sr_run_stats *stats);

/* Per-sweep trace of the last sr_run (the Fig. 10 / Section 5.4 instrumentation):
 * one record per sweep, in order. */
typedef struct {
  int32_t pass;              /* passes completed before this sweep */
  int32_t phase;             /* 1 = verification sweep (prediction off) */
  int64_t changed, attempted, skipped, edges;
  int64_t state_hist[8];     /* weak predictor: vertices visited in each state */
  double l1;                 /* PageRank: L1 change of the sweep */
} sr_sweep_record;
/* Copy up to max records of the last run into out (host); *count receives
 * the number of sweeps the run made (may exceed max). */
sr_status sr_run_sweeps(const sr_graph *g, sr_sweep_record *out, int32_t max, int32_t *count);

/* Copy the last run's vertex values to host memory: uint32 per vertex for
 * BFS (levels), SSSP (distances) and CC (labels), SR_INF if unreached;
 * float32 ranks for PageRank/PPR, in the caller's vertex ids. This is the
 * device-to-host transfer of the result that the paper counts in a solve's
 * time (Section 5.2: times include data transfers). host_dst (host memory,
 * owned by the caller) receives 4n bytes; dst_bytes must be >= 4n
 * (SR_EINVAL otherwise); SR_ESTATE if no run has produced values. */
sr_status sr_read_values(const sr_graph *g, void *host_dst, uint64_t dst_bytes);


/* ---------------------------------------------------------------- batched */

/* Many instances in one launch: beyond the paper, which runs one program
 * at a time. Instances are grouped per graph in groups of width K (8);
 * values of a group are laid out [vertex][K] so every in-edge read and
 * every neighbour gather is shared by the K instances. All groups of all
 * graphs are swept by one persistent kernel whose blocks take work items
 * from a device queue; the sweep is captured once in a HIP graph and
 * replayed until every instance has converged (PPR: L1 change of a sweep
 * below tol_l1, or the FP32 floor rule; SSSP/BFS: a sweep without change,
 * with the Table I strong conditions per instance). The schedule is chosen
 * by a built-in autotuner that times one sweep over every instance for each
 * candidate: the group width K (instance columns sharing each gathered row:
 * 8 or 16 for PPR, 8, 16 or 32 for SSSP/BFS), the vertex rounds per work item
 * (2, 4 or 8), the persistent grid size and the items taken per queue
 * access. The choice is cached per process, keyed by the algorithm and each
 * graph's scale bucket, edge factor and instance count, and in the text
 * file named by SR_TUNE_CACHE if set. The environment variable
 * SR_BATCH_SCHEDULE="K,rounds" fixes the width and rounds of a call (grid
 * and grab are still tuned; SR_EINVAL if malformed). Graphs must fit the
 * budget resident. */
typedef struct {
  sr_graph *g;
  sr_algo algo;      /* SR_PPR, SR_SSSP or SR_BFS; one family per call
                        (PPR alone, or any mix of SSSP and BFS) */
  int32_t source;    /* PPR seed or SSSP/BFS source */
} sr_instance;

typedef struct {
  int32_t sweeps;        /* graph replays (one sweep of every group each) */
  int32_t groups;        /* instance groups of width group_width */
  int32_t group_width;
  int32_t grid_blocks;   /* persistent grid chosen by the autotuner */
  int32_t grab;          /* work items per queue access */
  int32_t tuned;         /* 1: the autotuner ran in this call, 0: cached */
  double kernel_ms;      /* device time of the replays (HIP events) */
  double wall_ms;        /* host wall time of the whole call */
  uint64_t algo_bytes;   /* algorithmic bytes of all sweeps */
  int32_t rounds;        /* chosen vertex rounds per wavefront and work item (small in-degree bins) */
  int32_t width_candidates; /* group widths timed by the autotuner in this call (1: cached or fixed) */
} sr_batch_stats;

/* Run `count` instances to convergence. host_dsts[i] (host, 4n_i bytes)
 * receives instance i's values (f32 ranks for PPR, u32 levels/distances
 * with SR_INF unreached). common supplies damping, tol_l1, max_passes
 * (sweep cap) and pvu (SSSP/BFS: OFF or STRONG; DEFAULT = STRONG; PPR:
 * OFF). per_instance (may be NULL) receives count records; batch_stats may
 * be NULL. */
sr_status sr_batch_run(sr_ctx *ctx, const sr_instance *instances, int32_t count,
                       const sr_run_params *common, void *const *host_dsts,
                       sr_run_stats *per_instance, sr_batch_stats *batch_stats);

/* ---------------------------------------------------------------- serving */

/* A continuous-batching query server (beyond the paper): SSSP and BFS
 * source queries on resident graphs. Each graph owns max_slots_per_graph
 * (8, 16, 32 or 64) query slots whose state (a 16-bit distance or level per
 * vertex per slot, plus one 4 B-per-vertex result buffer per running query)
 * is allocated up front if state_budget_bytes allows, else as many slots as
 * fit. A progress thread admits queued queries into free slots as they
 * free up, sweeps every graph with active slots (one multi-source sweep
 * per graph, all its active slots together), retires converged slots (a
 * sweep without change under the Table I strong conditions), copies their
 * values to host and records latency = completion - submission. Results
 * are exact u32 values: a slot whose distances do not all fit (some vertex
 * at distance 32767 or more; the slots store values below 2^15 - 1 so that
 * a value plus an edge weight never wraps) is completed on the host when it
 * retires (label-correcting push from every reached vertex), which the
 * stats count. */
sr_status sr_server_create(sr_ctx *ctx, sr_graph *const *graphs, int32_t ngraphs,
                           uint64_t state_budget_bytes, int32_t max_slots_per_graph,
                           sr_server **out);
/* Queue a query (thread-safe). algo is SR_SSSP or SR_BFS. *ticket
 * identifies it for sr_server_poll. SR_EBUSY if the queue holds 1M
 * queries. */
sr_status sr_server_submit(sr_server *srv, int32_t graph, sr_algo algo, int32_t source,
                           uint64_t *ticket);
/* Non-blocking poll (thread-safe). When the query is done, *done = 1, its
 * values are copied to host_dst (if not NULL, bytes >= 4n) and *latency_ms
 * is set; the result is then released (a later poll returns SR_EINVAL). */
sr_status sr_server_poll(sr_server *srv, uint64_t ticket, void *host_dst, uint64_t bytes,
                         int *done, double *latency_ms);
typedef struct {
  uint64_t submitted, completed, sweeps;
  int32_t slots_per_graph[8];
  double busy_ms;        /* progress-thread time spent with work in flight */
  uint64_t narrow_fallbacks; /* retired queries whose 16-bit slot column overflowed and were completed
                                exactly on the host */
  double kernel_ms;      /* device time of the sweep replays (multi-source sweep, heavy-vertex and
                            close kernels; HIP events) */
  uint64_t algo_bytes;   /* algorithmic bytes of those sweeps: per sweep and live graph, its edge words
                            (and separate weights), offsets, bin lists and own values (4m (+4m) + 12n);
                            per retired query, 2 bytes (one 16-bit value) per in-edge its column scanned */
} sr_server_stats;
sr_status sr_server_stats_get(sr_server *srv, sr_server_stats *out);
/* Stop the progress thread after finishing admitted queries, free the
 * server's device state. Results not yet polled are discarded. */
sr_status sr_server_destroy(sr_server *srv);

/* Diagnostic, not part of any solve: the rate of the pull's random gather
 * alone (the gather of in-neighbour values in the pull of Section 4.1, the
 * memory-bound step Section 5.3 finds limiting). The m edge words at src
 * and the n u32 values at values (host memory, owned by the caller; the
 * source id of a word is word & src_mask) are copied to device memory the
 * library allocates within the context's budget and frees on return. The
 * probe reads every word and the value it names with the sweep kernel's
 * tiling (4096 words per block of 256 threads; thread t reads 8 groups of
 * 2 consecutive words starting at g * 512 + 2t, the 16 word loads and then
 * the 16 gathers issued together), with no gate, reduction or write beyond
 * one checksum add per block. One untimed launch gives *checksum = the sum of
 * values[word & src_mask] over all words, modulo 2^64; then `repeats`
 * launches are timed with HIP events on the context's compute stream and
 * *ms_per_launch receives their average. Ids at or above n are clamped to
 * n - 1, so nothing outside the values is read. SR_EINVAL: a null pointer,
 * m < 1, n < 1, repeats < 1 or m above 2^31 * 4096; SR_EBUDGET: the copies
 * do not fit the budget; SR_EDEVICE: a host-only context or a HIP error. */
sr_status sr_probe_gather(sr_ctx *ctx, const uint32_t *src, int64_t m, uint32_t src_mask,
                          const uint32_t *values, int32_t n, int32_t repeats, double *ms_per_launch,
                          uint64_t *checksum);

#ifdef __cplusplus
}
#endif
#endif /* SERAPH_H */
