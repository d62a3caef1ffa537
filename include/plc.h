/*
 * plc.h -- C ABI of libplc, a gfx950 (MI355X) implementation of parallel
 * local graph clustering: round-synchronous PR-Nibble followed by the sweep
 * cut, after Shun, Roosta-Khorasani, Fountoulakis and Mahoney, "Parallel
 * Local Graph Clustering" (arXiv 1604.07515).
 *
 * Conventions
 *  - Every call returns a plc_status: PLC_OK (0) or a negative code.  No C++
 *    exception crosses this boundary.
 *  - A context is used by one host thread at a time.
 *  - Device memory: the caller hands the library one device buffer (the
 *    arena) at plc_init and keeps it alive until plc_destroy.  The library
 *    never allocates device memory itself; every graph, query state and
 *    result lives in the arena, so the arena size is the memory budget.
 *    (It does allocate pinned host staging buffers with hipHostMalloc.)
 *  - Streams: all device work is issued on the hipStream_t given at plc_init
 *    (passed as void*; NULL means the default stream).  In the default
 *    launch mode the library also owns one non-blocking stream on which it
 *    only records graphs; nothing executes on it.
 *  - Graphs are undirected and unweighted (Sec. 2, "Graph Notation"): CSR
 *    with row offsets off[0..n] and neighbour ids nbr[0..off[n]), every
 *    undirected edge stored as two arcs, d(v) = off[v+1] - off[v],
 *    2m = off[n].
 */
#ifndef PLC_H
#define PLC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t plc_status;
#define PLC_OK 0
#define PLC_E_INVALID (-1)  /* bad argument, bad graph, bad query parameter   */
#define PLC_E_NOMEM (-2)    /* the arena cannot hold the graph or the query   */
#define PLC_E_BUSY (-3)     /* no batch slot or memory free now; retry later  */
#define PLC_E_NOTREADY (-4) /* the query has not finished                     */
#define PLC_E_NOTFOUND (-5) /* unknown or released query id                   */
#define PLC_E_LIMIT (-6)    /* max_rounds reached (watchdog)                  */
#define PLC_E_HIP (-7)      /* HIP runtime error; the context is unusable     */

/* Push rules of PR-Nibble (Sec. 3.3). */
#define PLC_RULE_OPT 0u  /* optimized rule ("An Optimization", Fig. alg:pr-nibble2):
                            p[v] += (2a/(1+a)) r[v]; r[w] += ((1-a)/(1+a)) r[v]/d(v); r[v] = 0 */
#define PLC_RULE_ORIG 1u /* original rule (Fig. alg:pr-nibble):
                            p[v] += a r[v]; r[w] += (1-a) r[v]/(2 d(v)); r[v] = (1-a) r[v]/2 */

/* plc_graph_load flags */
#define PLC_GRAPH_VALIDATE 1u /* check symmetry, sorted rows, no self-loops or
                                 duplicates, ids < n; PLC_E_INVALID otherwise */

typedef struct plc_ctx plc_ctx;
typedef struct plc_graph plc_graph;

/*
 * Launch modes.  PLC_LAUNCH_GRAPH (the default): the round loops are recorded
 * once as HIP graphs -- the plain path's chunks of rounds and its sweep, the
 * batched path's round -- and replayed with one hipGraphLaunch each on the
 * context's stream.  PLC_LAUNCH_DIRECT: every kernel is launched on its own.
 * Both run the same kernels with the same arguments; if recording a graph
 * fails the context falls back to direct launches.
 */
#define PLC_LAUNCH_GRAPH 0
#define PLC_LAUNCH_DIRECT 1

/*
 * Layouts of the batch engine's per-query state.  PLC_STATE_DENSE: every slot
 * owns dense arrays over all n vertices (40 bytes per vertex per slot,
 * reserved up front by plc_batch_reserve); the edge scatter indexes them
 * directly.  PLC_STATE_COMPACT: every admitted query owns an open-addressing
 * table (16-byte records, p beside them) plus its vertex lists, 36 bytes per
 * table record, taken from the arena at admission, sized for the seed's
 * first round and grown between rounds (at most half full before a round,
 * at most 3/4 after it), so memory follows the vertices a query touches.
 * Queued queries are admitted while a slot is free and the arena can hold
 * their first table; a query whose table cannot grow waits while others
 * run, and fails with PLC_E_NOMEM only when no other query can make
 * progress.  Results are the same in both layouts.
 */
#define PLC_STATE_DENSE 0
#define PLC_STATE_COMPACT 1

/*
 * The plain path's edge scatter (Sec. 3.3, UpdateNgh as a fetch-and-add) has
 * two forms.  Small rounds: one FP64 atomic add per edge.  Rounds of at
 * least bin_min_edges edges: destination-binned -- the round's (neighbour,
 * entry) pairs are sorted by destination range, each range's contributions
 * are summed in LDS, and every touched r[w] gets one update.  Results agree
 * to the order of the additions.  bin_min_edges: 0 = 524288, which
 * plc_autotune may change per graph (it also tries four times that and no
 * binning); > 0 = that threshold, kept by plc_autotune; < 0 = always the
 * atomic form.  (Graphs of more than 6,291,456 = 1536 x 4096 vertices
 * always use the atomic form.)  With 0 the library also learns from the
 * last queries at which launches of a query's first chunk of rounds such
 * rounds fall, and queues the binned form's second pass only there: a round
 * of that size elsewhere in the first chunk takes the atomic form (the same
 * result up to the order of the additions; plc_result_info.bin_rounds
 * counts the rounds that did bin).
 */
typedef struct {
  int32_t max_rounds;  /* watchdog on PR-Nibble rounds per query; 0 = 1<<20 */
  int32_t batch_slots; /* concurrent queries in the batched path; 0 = 256   */
  int32_t launch_mode; /* PLC_LAUNCH_GRAPH or PLC_LAUNCH_DIRECT             */
  int32_t batch_state; /* PLC_STATE_DENSE or PLC_STATE_COMPACT              */
  int32_t bin_min_edges; /* smallest plain round scattered through bins     */
  int32_t reserved[3];
} plc_options;

/*
 * One PR-Nibble query (Sec. 3.3): seed vertex x with d(x) >= 1, teleport
 * alpha in (0,1), tolerance eps (finite, 1e-250 <= eps).  The first round
 * always pushes the seed; afterwards a vertex is active in a round when
 * r[v] >= eps * d(v) at the start of that round.
 */
typedef struct {
  int32_t seed;
  uint32_t rule; /* PLC_RULE_OPT or PLC_RULE_ORIG */
  double alpha;
  double eps;
  uint32_t flags;    /* PLC_QF_* */
  uint32_t reserved; /* 0 */
} plc_query;

/* plc_query flags.  PLC_QF_NO_RESIDUAL: the result keeps p and the cluster
 * but not the final residual (r_nnz is still reported; plc_result_copy then
 * returns no r entries), for callers that only want the cluster. */
#define PLC_QF_NO_RESIDUAL 1u
#define PLC_QF_ALL 1u

typedef struct {
  int64_t n;           /* vertices                              */
  int64_t arcs;        /* 2m                                    */
  int64_t max_degree;
  int64_t bytes;       /* arena bytes held by the graph          */
} plc_graph_info;

/* Summary of a finished query.  cut, vol and phi describe the best sweep
 * prefix S_kstar (Sec. 3.1): phi = cut / min(vol, 2m - vol). */
typedef struct {
  int32_t status;     /* PLC_OK, PLC_E_LIMIT or PLC_E_NOMEM             */
  int32_t rounds;     /* rounds that pushed at least one vertex         */
  int64_t pushes;     /* sum over rounds of |frontier|                  */
  int64_t edges;      /* sum over rounds of sum_{v in frontier} d(v)    */
  int64_t support;    /* N = |{v : p[v] > 0}|                           */
  int64_t kstar;      /* cluster = first kstar vertices of the sweep    */
  int64_t cut;        /* |boundary(S_kstar)|                            */
  int64_t vol;        /* vol(S_kstar)                                   */
  double phi;         /* conductance of S_kstar                         */
  int64_t r_nnz;      /* nonzeros of r at exit                          */
  /* plain path only (0 elsewhere): self launches that did work, and the
   * rounds and edges among `rounds` and `edges` that a self launch ran on
   * its own (small frontiers, one workgroup, no scatter launch) */
  int32_t launches;
  int32_t loop_rounds;
  int64_t loop_edges;
  /* plain path only (0 elsewhere): wall time in the library from the
   * query's start to its recorded result (push, sweep and read-backs; the
   * copy into the result block is queued), in nanoseconds.  A query queued
   * behind the previous one of the same plc_run call starts when that one
   * is known to be done. */
  int64_t host_ns;
  /* device time of the query, from the GPU's constant-rate clock (read by
   * the kernels themselves): plain path, from its initialisation kernel to
   * the end of its sweep; batched path, from its admission into a slot to the
   * end of its sweep (so it includes rounds shared with other queries) */
  int64_t device_ns;
  /* plain path only: rounds whose edge scatter went through the destination
   * bins (plc_options.bin_min_edges), and their edges */
  int32_t bin_rounds;
  uint32_t flags;     /* the query's flags */
  int64_t bin_edges;
  /* plain path, plc_run only: 1 when this query's initialisation and first
   * rounds were queued behind the previous query's read-back and started
   * there; 2 when they were queued there but stood aside (the previous query
   * still needed work) and the query started afresh; 0 otherwise */
  int32_t pipelined;
  /* batched path with compact tables only (0 elsewhere): times the query's
   * table moved to a larger block, and its capacity in records when the
   * query finished pushing */
  int32_t table_grows;
  int64_t table_cap;
  /* plain path only: among bin_rounds, the rounds of at least half the
   * graph's arcs, which the bins pull from their own vertices' arcs */
  int32_t pull_rounds;
  int32_t reserved;
} plc_result_info;

/* Status code to a static string. */
const char* plc_status_str(plc_status s);

/*
 * Create a context on HIP device `device`, using the caller-owned device
 * buffer [dev_arena, dev_arena + arena_bytes) (256-byte aligned) as the only
 * device memory and `hip_stream` (a hipStream_t, may be NULL) for all work.
 * opt may be NULL.  On success *out receives the context.
 */
plc_status plc_init(plc_ctx** out, int32_t device, void* dev_arena, size_t arena_bytes,
                    void* hip_stream, const plc_options* opt);

/* Wait for outstanding work and free the library's host state.  Graphs and
 * results of the context become invalid.  The arena is not touched. */
plc_status plc_destroy(plc_ctx* ctx);

/*
 * Copy a host CSR graph (Sec. 2) into the arena and prepare its per-vertex
 * state.  offsets: n+1 entries of 32 or 64 bits (offsets_bits), host memory;
 * nbrs: num_arcs int32 ids, host memory.  The caller may free both on
 * return.  Errors: PLC_E_INVALID (sizes, offsets not monotone, or a failed
 * PLC_GRAPH_VALIDATE check), PLC_E_NOMEM (arena too small).
 */
plc_status plc_graph_load(plc_ctx* ctx, int64_t n, int64_t num_arcs, const void* offsets,
                          int32_t offsets_bits, const int32_t* nbrs, uint32_t flags,
                          plc_graph** out);

/* Wait for outstanding work, drop the graph's batch engine (queued and
 * running queries are dropped; finished results stay valid) and return its
 * arena memory.  PLC_E_INVALID if g does not belong to ctx. */
plc_status plc_graph_free(plc_ctx* ctx, plc_graph* g);

/* Sizes of a loaded graph (host-side bookkeeping, no device work). */
plc_status plc_graph_info_get(const plc_graph* g, plc_graph_info* out);

/*
 * Plain path: run `count` queries one after another, each as round-
 * synchronous PR-Nibble (Sec. 3.3, Figs. alg:pr-nibble / alg:pr-nibble2)
 * followed by the sweep cut (Sec. 3.1, Theorem 1), blocking until all are
 * done.  ids[i] (may be NULL) receives a handle whose vectors stay in the
 * arena until plc_release (the block is sized for the support and the
 * nonzeros of r); infos[i] (may be NULL) receives the summary.
 * A query rejected by parameter checks gets status PLC_E_INVALID in its info
 * and id 0, and the call still runs the others; the return value is the
 * first error met, or PLC_OK.
 */
plc_status plc_run(plc_ctx* ctx, plc_graph* g, const plc_query* q, int32_t count, uint64_t* ids,
                   plc_result_info* infos);

/*
 * Allocation-free variant of plc_run for one query, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): no context, no arena, and no call to
 * hipMalloc, hipFree, hipHostMalloc or any other allocating routine.  The
 * query's working state (state records, frontiers, sort and sweep buffers,
 * about 152 bytes per vertex plus 4 bytes per 1024 arcs) lives in one fixed
 * device array of PLC_NOALLOC_SCRATCH_BYTES inside the library, which every
 * GPU the library runs on holds until the process ends; graphs whose state
 * does not fit (about 400,000 vertices) get PLC_E_NOMEM.  Every call
 * re-initialises that array, so calls that overlap on one GPU (from several
 * host threads, or on several streams) race and must not be made; calls on
 * different GPUs are independent.
 *   device:      HIP device to run on (made current).
 *   hip_stream:  hipStream_t for all work, may be NULL; the call blocks until
 *                its work on that stream is done.
 *   d_off, d_nbr: the CSR graph in device memory (offsets n+1 int64, neighbour
 *                ids num_arcs int32, as in plc_graph_load), read only; the
 *                caller owns them.
 *   q:           the query (seed, alpha, eps, rule, flags as in plc_query).
 *   d_sweep_ids, d_sweep_p: caller-owned device buffers of n entries each;
 *                on return their first info->support entries hold the
 *                support in sweep order and p on it (the cluster is the
 *                first info->kstar).  No residual vector is returned.
 *   info:        host struct, filled as by plc_run (bin_rounds 0: this
 *                variant always uses the atomic scatter).
 * Errors: PLC_E_INVALID (null pointer, bad sizes, device or query
 * parameters, a seed of degree 0), PLC_E_NOMEM (state larger than the array;
 * nothing runs), PLC_E_HIP.  Same kernels and results as plc_run.
 */
#define PLC_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
plc_status plc_run_noalloc(int32_t device, void* hip_stream, int64_t n, int64_t num_arcs,
                           const int64_t* d_off, const int32_t* d_nbr, const plc_query* q,
                           int32_t* d_sweep_ids, double* d_sweep_p, plc_result_info* info);

/*
 * Plain path, one query from a seed set (Sec. 3: the local algorithms start
 * from a seed vertex or a set of seed vertices).  The paper leaves the
 * initial split of the unit mass open; it is split equally over the
 * distinct seeds: r = 1/|S| on each, and all of S forms the first frontier.
 * seeds: host array of nseeds vertex ids (duplicates allowed, counted
 * once), read before the call returns.  alpha, eps, rule as in plc_query.
 * *id (may be NULL) and *info (may be NULL) as for plc_run.  Blocks until
 * done.  Returns PLC_OK (also when max_rounds stopped the push: then
 * info->status is PLC_E_LIMIT and the partial p is swept), PLC_E_INVALID
 * (nseeds < 1, a seed out of range or of degree 0, bad alpha/eps/rule;
 * nothing runs), PLC_E_NOMEM (no room for the result: the counters are
 * still in *info) or PLC_E_HIP.
 */
plc_status plc_run_set(plc_ctx* ctx, plc_graph* g, const int32_t* seeds, int32_t nseeds,
                       double alpha, double eps, int32_t rule, uint64_t* id,
                       plc_result_info* info);

/*
 * Plain path, deterministic heat-kernel PageRank from seed x (Sec. 3.4,
 * the Kloster-Gleich procedure and Fig. alg:hkpr) followed by the sweep cut.
 * Level j = 0 .. N-1 is one synchronous round: every frontier vertex v adds
 * its level-j residual r to p[v]; for j + 1 < N each neighbour w gets
 * t r / ((j + 1) d(v)) at level j + 1, and the next frontier is every w whose
 * level-(j+1) residual reached ((e^-t eps) d(w)) / (2 N psi_{j+1}), with
 * psi_k = sum_{m=0}^{N-k} k!/(m+k)! t^m; on the last level (j + 1 = N) each
 * neighbour gets r / d(v) added to p directly.  Level-j residuals that never
 * reach the threshold are dropped.  Readings: the pseudocode's loop test
 * "j+1 == N" and its e^{t} contradict the text; the text's "j+1 < N" and
 * e^{-t} are taken.  N in [1, 1024], eps > 0 (at eps = 0 the printed
 * crossing test could never hold), t > 0.  Blocks until done.  *info: rounds = levels run, pushes = (vertex,
 * level) entries processed, edges = their degrees, support, the cluster;
 * no residual is reported (r_nnz = 0).  Errors: PLC_E_INVALID (bad seed,
 * N, eps or t; nothing runs), PLC_E_NOMEM (no room for the result: the
 * counters are still in *info), PLC_E_HIP.
 */
plc_status plc_run_hkpr(plc_ctx* ctx, plc_graph* g, int32_t seed, int32_t N, double eps,
                        double t, uint64_t* id, plc_result_info* info);

/*
 * Plain path, Nibble from seed x (Sec. 3.2, Fig. alg:nibble: the truncated
 * lazy random walk) followed by the sweep cut.  p_0 is x's indicator and
 * the first frontier is {x}; step t (1..T) forms p_t from the frontier of
 * p_{t-1}: each frontier vertex v keeps p_{t-1}[v]/2 and sends
 * p_{t-1}[v]/(2 d(v)) to every neighbour; the next frontier is every v with
 * p_t[v] >= eps d(v).  If it is empty, p_{t-1} is returned; else after T
 * steps p_T is.  The returned vector is swept whole (entries below eps d(v)
 * only stop propagating).  eps > 0, T in [0, 1024].  Blocks until done.
 * *info: rounds = steps computed, pushes = frontier entries processed,
 * edges = their degrees, support, the cluster; no residual (r_nnz = 0).
 * Errors: PLC_E_INVALID (bad seed, eps or T; nothing runs), PLC_E_NOMEM (no
 * room for the result: the counters are still in *info), PLC_E_HIP.
 */
plc_status plc_run_nibble(plc_ctx* ctx, plc_graph* g, int32_t seed, double eps, int32_t T,
                          uint64_t* id, plc_result_info* info);

/*
 * Plain path, the beta variant of PR-Nibble (end of Sec. 3.3): every round
 * pushes only the ceil(beta |S|) vertices of the active set S = {v : r[v] >=
 * eps d(v)} with the largest r[v]/d(v) (ties by ascending id), with the
 * round-synchronous updates of *q's rule among them; the others stay active.
 * beta in (0, 1]; beta = 1 is plc_run's algorithm.  *q as for plc_run (one
 * query); *id, *info as for plc_run.  Rounds are launched directly (not
 * replayed as graphs).  Returns PLC_OK (also when max_rounds stopped the
 * push: info->status is then PLC_E_LIMIT), PLC_E_INVALID (bad query or
 * beta; nothing runs), PLC_E_NOMEM (no room for the result) or PLC_E_HIP.
 */
plc_status plc_run_beta(plc_ctx* ctx, plc_graph* g, const plc_query* q, double beta,
                        uint64_t* id, plc_result_info* info);

/*
 * Batched path.  Many queries advance together: every global step runs one
 * PR-Nibble round for all admitted queries in the same kernel launches, and
 * the queries whose frontier emptied are swept together.  Results are the
 * same as plc_run's (same kernels' arithmetic; only the order of atomic
 * additions differs).
 *
 * plc_batch_reserve: give graph g a batch engine with up to `slots`
 * concurrent queries (1..1024; slots <= 0 takes plc_options.batch_slots),
 * in the context's state layout
 * (plc_options.batch_state).  Dense: each slot holds per-vertex state (about
 * 40 bytes per vertex), so fewer slots are granted when the arena is short
 * (max(64 MiB, 1/16 of the free arena) stays free for result blocks).
 * Compact: the slots themselves are small; queries take their tables from
 * the arena as they run.  *granted (may be NULL) receives the number.
 * PLC_E_NOMEM if not even one slot fits.  Calling it again re-creates the
 * engine (pending and running queries are dropped).
 */
plc_status plc_batch_reserve(plc_ctx* ctx, plc_graph* g, int32_t slots, int32_t* granted);

/*
 * Queue `count` queries on graph g's batch engine (non-blocking).  ids[i]
 * receives each query's handle, or 0 with the first error returned when a
 * query fails the parameter checks.  Queued queries are admitted into free
 * slots at the start of the next plc_progress step, in submission order.
 */
plc_status plc_submit(plc_ctx* ctx, plc_graph* g, const plc_query* q, int32_t count,
                      uint64_t* ids);

/*
 * Run one global step of g's batch engine: admit queued queries into free
 * slots, run one round for every admitted query, sweep the queries whose
 * frontier emptied in an earlier step, and retire finished queries.  Blocks
 * until the step's device work is done.  *in_flight (may be NULL) receives
 * the number of queries queued or running after the step.  The ids of the
 * queries that finished in this step are written to done_ids[0..*n_done)
 * (done_ids may be NULL; at most done_cap are written, *n_done counts all).
 */
plc_status plc_progress(plc_ctx* ctx, plc_graph* g, int32_t* in_flight, uint64_t* done_ids,
                        int32_t done_cap, int32_t* n_done);

/* *done = 1 if query `id` has finished (its result is ready), else 0. */
plc_status plc_poll(plc_ctx* ctx, uint64_t id, int32_t* done);

/*
 * Block until query `id` has finished, driving its graph's batch engine one
 * plc_progress step at a time (other queries advance and finish as well;
 * their results stay available to plc_poll and plc_result_*).  timeout_us < 0
 * waits without limit; otherwise PLC_E_NOTREADY is returned once that much
 * wall time has passed with the query still in flight.  PLC_OK when the
 * query has finished (also if it already had), PLC_E_NOTFOUND for unknown
 * ids.
 */
plc_status plc_wait(plc_ctx* ctx, uint64_t id, int64_t timeout_us);

/*
 * Upper bound on the arena bytes that one query q on graph g occupies on the
 * batch engine, in the context's state layout, plus its result block.
 * Dense: the state of one slot (residual record, p, two frontier buffers,
 * support and touched lists over all n vertices; plc_batch_reserve takes it
 * for every slot).  Compact: the largest table block the query can reach
 * (36 B per record, capacity twice its touched bound rounded up to a
 * multiple of 1024 records).
 * The bounds come from the push's work bound (Sec. 3.3): every push except
 * the seed's moves at least alpha' eps d(v) of the unit mass into p, with
 * alpha' = 2 alpha/(1+alpha) for the optimized rule and alpha for the
 * original, so at most 1 + 1/(alpha' eps) vertices are pushed and at most
 * 1 + d(seed) + 1/(alpha' eps) are touched (both also at most n).  Used by a
 * serving front end to budget admissions.  Returns 0 when g or q is invalid.
 */
size_t plc_query_bytes_estimate(const plc_graph* g, const plc_query* q);

/* Submit `count` queries and step g's batch engine until all have finished.
 * Throughput mode: queries that finish pushing while others still push are
 * swept together later (unless queued queries wait for their slots). */
plc_status plc_run_batched(plc_ctx* ctx, plc_graph* g, const plc_query* q, int32_t count,
                           uint64_t* ids, plc_result_info* infos);

/*
 * Launch-shape autotuner.  Runs the `count` sample queries (their results are
 * discarded) under candidate launch shapes and keeps, for graph g, the
 * fastest by wall time: for the plain path (which = PLC_TUNE_PLAIN) the
 * workgroup counts of the vertexMap, edgeMap and sweep kernels; for the
 * batched path (PLC_TUNE_BATCH, needs plc_batch_reserve first) the
 * workgroup counts of its vertexMap and edgeMap kernels.  The edgeMap
 * kernels give each workgroup a contiguous range of 1024-edge tiles, so the
 * workgroup count sets the frontier tiling.  out (may be NULL) receives the
 * chosen shapes.
 */
#define PLC_TUNE_PLAIN 1
#define PLC_TUNE_BATCH 2
typedef struct {
  int32_t plain_self, plain_scatter, plain_sweep;   /* workgroups per launch */
  int32_t batch_self, batch_scatter, batch_sweep;
  double plain_ms, batch_ms;                        /* best sample wall time */
  int32_t candidates;                               /* configurations tried */
  /* plain path: rounds of at least this many edges take the binned scatter
   * (-1: none).  Tuned among the default, four times it and none when
   * plc_options.bin_min_edges is 0; otherwise the context's setting. */
  int32_t plain_bin_min_edges;
} plc_tune;

plc_status plc_autotune(plc_ctx* ctx, plc_graph* g, const plc_query* sample, int32_t count,
                        int32_t which, plc_tune* out);

/* Summary of a finished query. PLC_E_NOTFOUND for unknown ids,
 * PLC_E_NOTREADY for queries still in flight. */
plc_status plc_result_info_get(plc_ctx* ctx, uint64_t id, plc_result_info* out);

/*
 * Copy a finished query's vectors to caller-owned host buffers (NULL skips
 * one): sweep_ids[support] = the support in sweep order (non-increasing
 * p/d, ties by ascending id), sweep_p[support] = p at those vertices, so the
 * cluster is sweep_ids[0..kstar); r_ids[r_nnz], r_vals[r_nnz] = nonzeros of
 * the final residual in unspecified order.  PLC_E_NOMEM for a query that
 * failed with PLC_E_NOMEM (it has no vectors).
 */
plc_status plc_result_copy(plc_ctx* ctx, uint64_t id, int32_t* sweep_ids, double* sweep_p,
                           int32_t* r_ids, double* r_vals);

/*
 * Several results at once, for serving loops that collect every query a
 * step finished: for each i < count the same as plc_result_copy(ctx,
 * ids[i], sweep_ids[i], sweep_p[i], r_ids[i], r_vals[i]), where a NULL
 * pointer array skips that part for every result and a NULL entry for one.
 * One kernel gathers the parts into pinned, device-mapped host staging
 * memory that the context keeps (grown as needed, freed with the context),
 * one wait, then host copies into the caller's buffers: one GPU round trip
 * for the whole set instead of one per result.  PLC_E_NOTFOUND for an
 * unknown id and PLC_E_NOMEM for a result without vectors (nothing copied
 * then), PLC_E_NOMEM also when the staging memory cannot be allocated.
 */
plc_status plc_result_copy_many(plc_ctx* ctx, int32_t count, const uint64_t* ids,
                                int32_t* const* sweep_ids, double* const* sweep_p,
                                int32_t* const* r_ids, double* const* r_vals);

/* Return a finished query's arena memory.  Does not wait for the GPU: any
 * work that reuses the memory is queued behind the query's pending result
 * copy on the context's stream.  PLC_E_NOTFOUND for an unknown id. */
plc_status plc_release(plc_ctx* ctx, uint64_t id);

/* Arena bytes currently free (largest free block in *largest, may be NULL). */
plc_status plc_arena_free_bytes(plc_ctx* ctx, size_t* total, size_t* largest);

/*
 * Device-time accounting with HIP events on the context's stream, off by
 * default.  While it is on, rounds are launched directly instead of from
 * recorded graphs, and the scatter and self kernels are launched with start
 * and stop events that take the kernel's own dispatch timestamps
 * (hipExtLaunchKernelGGL); the sweep is bracketed by an event pair.  Plain
 * path: only launches that did work are counted.  A self launch may run
 * whole small rounds itself (info->loop_rounds); their edges and pushes
 * are not the scatter's.  Batch engine: one scatter launch per step
 * (all scheduled queries' edges) and one sweep sequence per step that swept;
 * self is not timed.
 *   scatter: the edgeMap kernel; units = pushed edges, entries = pushes
 *            (of the rounds it pushed)
 *   self:    the vertexMap + frontier-scan kernel (and the small rounds it
 *            runs); units = pushes
 *   sweep:   the whole sweep-cut sequence; units = support volume vol(S_N),
 *            entries = support size N
 */
typedef struct {
  int64_t launches;
  double ms;       /* summed device time */
  int64_t units;
  int64_t entries;
} plc_kernel_time;

plc_status plc_timing_enable(plc_ctx* ctx, int32_t on);  /* also resets the counters */
plc_status plc_timing_get(plc_ctx* ctx, plc_kernel_time* scatter, plc_kernel_time* self,
                          plc_kernel_time* sweep);

#ifdef __cplusplus
}
#endif
#endif /* PLC_H */
