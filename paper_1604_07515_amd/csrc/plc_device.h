// plc_device.h -- device-side data layout and kernel entry points of libplc
// (plain path: one query at a time on dense per-vertex state).
//
// HBM layout for one resident graph (all inside the caller's arena):
//   off   int64[n+1]     CSR row offsets
//   nbr   int32[2m]      neighbour ids, rows sorted
//   vr    VRec[n]        per-vertex record {r, d(v), sweep rank}: the edge
//                        scatter's atomic on r and its read of d(w) hit one
//                        16-byte record, i.e. one cache line
//   p     double[n]      approximate PageRank vector
// plus work buffers sized by n (frontier ping-pong, per-entry coefficient,
// row offset and edge start, support and touched lists, sort buffers).
// Dense per-vertex state is reset at the end of every query's sweep through
// the touched and support lists, so a query's cost stays proportional to the
// vertices it touched.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_util.h"
#include "sort.h"

namespace plc {

struct __align__(16) VRec {
  double r;      // residual; +0.0 = never touched by this query, -0.0 = pushed (optimized rule)
  int32_t deg;   // d(v), constant for the graph
  int32_t rank;  // sweep rank 1..N while a sweep runs, 0 otherwise
};

// Query status in the control block.  ST_PUSH: rounds in progress (done when
// the current frontier is empty); ST_LIMIT: watchdog fired, sweep the partial
// p; ST_SWEEPING: sweep kernels running; ST_SWEPT: results ready.
enum : int32_t { ST_IDLE = 0, ST_PUSH = 1, ST_SWEPT = 2, ST_LIMIT = 4, ST_SWEEPING = 6 };

// Scan sites (each has its own descriptor buffers and ticket dispenser).
enum : int32_t { SCAN_FRONTIER = 0, SCAN_VOL = 1, SCAN_CUT = 2, NUM_SCANS = 3 };

// Last-workgroup counters.
enum : int32_t {
  DONE_SCATTER = 0, DONE_KEYS = 1, DONE_SORT = 2, DONE_FINISH = 3, DONE_SELF = 4, DONE_BIN = 5,
  NUM_DONE = 8
};

// Where the running sweep writes its results (the library's own buffers,
// set by k_sweep_keys; the host copies them into the query's result block).
struct SweepOut {
  int32_t* ids;     // [N] support in sweep order
  double* p;        // [N] p in sweep order
  int32_t* rid;     // [rcap] ids of the nonzeros of r
  double* rval;     // [rcap] their values
  long long rcap;   // capacity of rid and rval
  long long pad;
};

// Device control block of one plain-path query.  Written by kernels only,
// except at query start (k_query_init) and read back by the host.
struct __align__(64) Ctl {
  // query parameters
  double cs, cn, keep, eps;
  int32_t seed, rule, max_rounds, opt_rule;  // opt_rule = 1 for the optimized rule
  // round state
  int32_t status;
  int32_t round;          // rounds pushed so far; frontier of round t is fbuf[t&1], size cnt[t&1]
  int32_t cnt[2];
  int32_t ntiles;         // edge tiles of the current round (or of the sweep's edges)
  uint32_t bin_pairs;     // bit i: the round of a first chunk's launch pair i could bin or pull
  long long etotal;       // sum of degrees of the current frontier (or vol(S_N) in the sweep)
  long long pushes, edges;
  int32_t support_cnt;    // |support list|
  int32_t touched_cnt;    // |touched list|
  int32_t fault;          // set on an impossible state (bounded spin ran out, bad tile map)
  int32_t limited;        // the watchdog stopped the rounds
  ScanSite scan[NUM_SCANS];
  unsigned int done[NUM_DONE];
  // sweep
  int32_t N;              // support size
  int32_t sort_flip;      // which sort buffer holds the sorted support
  int32_t rnnz;
  int32_t pad1;
  long long vol_total;    // 2m
  long long best_cut, best_vol, best_den;
  long long kstar;
  double phi;
  SweepOut out;           // result destinations of the running sweep
  // HK-PR (Sec. 3.4): Taylor degree, t, e^-t * eps, and the lengths of the
  // three rotating per-level touched lists (level k uses list k % 3; Nibble
  // uses the same lists and arrays for its vectors)
  int32_t hk_N;
  int32_t hk_tlc[3];
  double hk_t, hk_A;
  // beta variant of PR-Nibble (end of Sec. 3.3): the fraction of the active
  // set pushed per round, and this round's active count and pushed count
  double beta;
  int32_t beta_nf, beta_k;
  // round bookkeeping: `selfed` is the round whose entries the last self
  // step built (the scatter pushes only that round); `steps` counts self
  // launches that did work; loop_rounds / loop_pushes / loop_edges count
  // the small rounds a self launch ran on its own
  int32_t selfed, steps;
  int32_t loop_rounds;
  int32_t init_held;  // a queued guarded initialisation found the previous query unfinished
  long long loop_pushes, loop_edges;
  // rounds whose scatter went through the destination bins, and their edges
  int32_t bin_rounds;
  int32_t pull_rounds;  // among bin_rounds: rounds in the pull form
  long long bin_edges;
  // constant-rate clock (wall_clock64) at the query's initialisation and at
  // the end of its sweep
  long long t_start, t_end;
};

// Arguments shared by the plain-path kernels (all device pointers).
// Per-vertex pull record: the vertex's coefficient cn rho / d in the round
// whose epoch is stamped.
struct __align__(16) PullRec {
  double coef;
  uint32_t stamp;
  int32_t pad;
};

struct PlainArgs {
  int64_t n;
  long long vol_total;
  const int64_t* off;
  const int32_t* nbr;
  VRec* vr;
  double* p;
  Ctl* ctl;
  // frontier
  int32_t* fbuf0;
  int32_t* fbuf1;
  double* coef;        // per entry: cn * rho / d
  int64_t* estart;     // per entry: start of its edges in the round's edge sequence
  int64_t* rowp;       // per entry: off[v]
  int32_t* tile_start; // per edge tile: index of the entry holding the tile's first edge
  int64_t tile_cap;    // capacity of tile_start
  unsigned long long* desc[NUM_SCANS];  // 2 x desc_cap words each
  int32_t desc_cap;
  int32_t* support;
  int32_t* touched;
  // sweep
  SortElem* sbuf[2];
  int32_t* sdeg;       // degree in sweep order
  int64_t* svol;       // inclusive volume prefix in sweep order
  int32_t* scnt;       // # earlier-ranked neighbours per sweep position
  double* sp;          // p in sweep order            } the sweep's results, copied
  int32_t* sid;        // vertex ids in sweep order   } into the query's result
  int32_t* rid;        // r nonzero ids               } block afterwards
  double* rval;        // r nonzero values            }
  // HK-PR: level k's residuals live in vr[].r (k even) or hk_r1 (k odd);
  // the vertices level k touched are listed in hk_tl[k % 3] (hk_tl[0] is
  // the touched list); hk_B[k] = 2 N psi_k, the threshold denominator
  double* hk_r1;
  int32_t* hk_tl[3];
  double* hk_B;
  long long* bbest;    // per-block argmin candidates (cut, den, k)
  int32_t* work_log;   // [2 kMaxChunk]: 1 where self (2i) / scatter (2i+1) launch i did work
  // hot destinations of the batched scatter (the highest-degree vertices,
  // combined in LDS there), kept with the graph
  const int32_t* hot_ids;  // [kHot] vertex of hot index j
  const int32_t* hotcode;  // [n] -(j+1) for hot vertex j, else 0
  // Destination-binned scatter of large rounds.  Bins are vertex ranges made
  // of whole 64-vertex blocks (so no cache line of state records spans two
  // bins), at most kBinWidth wide, with roughly equal volume.  Rounds of
  // bin_emin .. bin_cmax * kBinChunk edges are binned; nbins = 0 turns it off.
  int32_t nbins;
  int32_t bin_cmax;            // chunks the pair buffer holds
  long long bin_emin;
  const int32_t* bin_of_blk;   // [ceil(n / kBinGran)] bin of each block
  const int32_t* bin_lo;       // [nbins + 1] first vertex of each bin
  const long long* bin_vol;    // [nbins] sum of degrees over the bin
  int32_t* bin_T;              // [(nbins + 1) x bin_cmax]: start of bin b's run in chunk c
  int2* bin_pairs;             // [bin_cmax x kBinChunk]: (neighbour, entry) by bin per chunk
  // Pull form of a binned round, for rounds of at least pull_emin edges
  // (half the graph's arcs): each bin sums, over its own vertices' arcs, the
  // coefficients of the neighbours on the round's frontier, which the
  // round's scatter launch stamps with the round's epoch.  The epoch advances
  // at every round close and is never reset, so records of earlier rounds
  // and queries never match.  pull = null turns it off.
  PullRec* pull;               // [n]
  unsigned* pull_epoch;
  long long pull_emin;
};

// Launch configuration.
constexpr int kBlock = 256;                      // threads per workgroup
constexpr int kScanItems = 4;                    // items per thread in scan-type kernels
constexpr int kScanBlock = kBlock * kScanItems;  // items per scan block
constexpr int kEdgeTile = 1024;                  // edges per scatter / cut tile
constexpr int kEdgesPerThread = kEdgeTile / kBlock;
constexpr int kHkMaxLevels = 1024;               // largest HK-PR Taylor degree N
constexpr int kNbMaxSteps = 1024;                // largest Nibble step count T
constexpr int kHot = 2048;                       // hot destinations (batched scatter)
constexpr int kMaxChunk = 256;                   // rounds queued at once (work log size / 2)
// Small rounds: while the frontier fits one scan block and a round has at
// most kLoopEdges edges, workgroup 0 of the self launch runs whole rounds
// back to back (kLoopPass edges per pass, at most kLoopMaxRounds per launch).
constexpr int kLoopEdges = 4096;
constexpr int kLoopPass = 2048;
constexpr int kLoopMaxRounds = 256;
static_assert(kHot % kEdgeTile == 0, "the hot flush works in kEdgeTile chunks");
// Destination-binned scatter (large rounds): pass A sorts each chunk of
// kBinChunk edges by bin; pass B accumulates each bin (or a slice of a
// heavy bin's chunks) in an LDS array of kBinWidth doubles.
constexpr int kBinGran = 64;
constexpr int kBinWidth = 4096;
constexpr int kMaxBins = 2048;
constexpr int kBinChunkTiles = 2;
constexpr int kBinChunk = kBinChunkTiles * kEdgeTile;
constexpr int kBinItemChunks = 2048;   // chunks one pass-B item may span
constexpr int kBinQ = 4096;            // expected pairs per pass-B item
constexpr long long kBinEmin = 1 << 19;  // default smallest binned round (edges)
constexpr long long kBinEmax = 1 << 23;  // largest binned round the pair buffer is sized for
constexpr long long kBinOff = 1ll << 62;  // a threshold no round reaches: binning off
// larger graphs use the atomic scatter only (their width-bound bins alone
// would crowd out the volume-balanced ones)
constexpr long long kBinMaxVertices = (long long)kMaxBins * 3 / 4 * kBinWidth;
static_assert(kBinChunk <= 65536 && kMaxBins <= 32768, "pass A packs (bin, rank) in 32 bits");

// Whether a round of this graph can be binned or pulled (both need bins and
// a reachable threshold); otherwise k_bin_apply never has work and the
// scatter closes every round itself.
inline bool bins_possible(const PlainArgs& a) { return a.nbins > 0 && a.bin_emin < kBinOff; }

// Host-side launchers (return hipError_t of the launch).
hipError_t launch_graph_init(hipStream_t s, const PlainArgs& a);
hipError_t launch_query_init(hipStream_t s, const PlainArgs& a, int32_t seed, int32_t rule,
                             double alpha, double eps, int32_t max_rounds, double beta = 1.0);
// The same, queued before the previous query is known to have finished: it
// initialises only if that query was swept (else it sets init_held and
// leaves the state alone, so rounds queued behind it continue the previous
// query's push).
hipError_t launch_query_init_guarded(hipStream_t s, const PlainArgs& a, int32_t seed,
                                     int32_t rule, double alpha, double eps, int32_t max_rounds);
// beta variant: before a round, rank the active frontier by r/d and keep the
// top ceil(beta |F|) in front as the round's frontier; after it, append the
// rest to the next frontier (max_count bounds the frontier for the sort)
hipError_t launch_beta_pre(hipStream_t s, const PlainArgs& a, int grid, int64_t max_count);
hipError_t launch_beta_post(hipStream_t s, const PlainArgs& a, int grid);
// seed set: the nseeds distinct seeds are already in a.fbuf0
hipError_t launch_query_init_set(hipStream_t s, const PlainArgs& a, int32_t nseeds, int32_t rule,
                                 double alpha, double eps, int32_t max_rounds);
// HK-PR (Sec. 3.4): init from seed x (a.hk_B[0..N] already uploaded), one
// level (self + scatter; a level past the end exits at once), and the final
// clearing of both residual arrays
hipError_t launch_hk_init(hipStream_t s, const PlainArgs& a, int32_t x, int32_t N, double t,
                          double A);
hipError_t launch_hk_level(hipStream_t s, const PlainArgs& a, int grid_self, int grid_scatter);
hipError_t launch_hk_clear(hipStream_t s, const PlainArgs& a, int grid);
// Nibble (Sec. 3.2): init from seed x, one step (self + scatter; steps past
// an empty frontier or T exit at once), and the end (vector R of J steps
// into p and the support list, both vector arrays cleared)
hipError_t launch_nb_init(hipStream_t s, const PlainArgs& a, int32_t x, double eps, int32_t T);
hipError_t launch_nb_step(hipStream_t s, const PlainArgs& a, int grid_self, int grid_scatter);
hipError_t launch_nb_finish(hipStream_t s, const PlainArgs& a, int32_t R, int32_t J, int grid);
// With t0 set, the kernel is launched with start and stop events that take
// its own dispatch timestamps (hipExtLaunchKernelGGL); not for graph capture.
// With slot >= 0 (< kMaxChunk) a launch that does work sets
// a.work_log[2 slot] (self) or a.work_log[2 slot + 1] (scatter).
hipError_t launch_self(hipStream_t s, const PlainArgs& a, int grid, hipEvent_t t0 = nullptr,
                       hipEvent_t t1 = nullptr, int slot = -1);
// The scatter of a PR-Nibble round: k_scatter (the atomic scatter, or pass A
// of the binned scatter for rounds of a.bin_emin edges and more), then
// k_bin_apply (pass B; exits at once after an atomic round).  With t0 set,
// t0 stamps k_scatter's start and t1 the end of the last kernel queued.
// apply = false leaves k_bin_apply out (t1 then stamps k_scatter's end): the
// round then takes the atomic form whatever its size.  pair in [0, 32): the launch pair's index in a first chunk; a round
// that could bin or pull sets bit pair of the control block's bin_pairs.
hipError_t launch_scatter(hipStream_t s, const PlainArgs& a, int grid, hipEvent_t t0 = nullptr,
                          hipEvent_t t1 = nullptr, int slot = -1, int grid_bin = 1024,
                          int pair = -1, bool apply = true);
// max_count: bound on the support size, sets the sort's launches; a
// query with a larger support (or one still pushing) is left unswept, so the
// sweep may be queued before the push is known to have ended.  The sweep
// writes its results to a.sid, a.sp (support order, p) and a.rid, a.rval
// (nonzeros of r) and, in its last kernel, resets the query's dense state
// (r over the touched list, p and the rank over the support list).
// launch_copy_result copies N and R of them into a result block.
hipError_t launch_sweep(hipStream_t s, const PlainArgs& a, int grid, int64_t max_count);
hipError_t launch_copy_result(hipStream_t s, const PlainArgs& a, int32_t* ids, double* p,
                              int32_t* rid, double* rval, int N, int R, int grid);

// One part of a result to gather: `words` 4-byte words from src (device
// memory) to word dst_off of the gather destination.
struct GatherJob {
  const uint32_t* src;
  uint64_t dst_off;
  uint64_t words;
};
// Gather njobs parts into dst (device-visible, e.g. mapped pinned host
// memory); jobs may itself live in mapped host memory.
hipError_t launch_gather_results(hipStream_t s, const GatherJob* jobs, int njobs, uint32_t* dst);

}  // namespace plc
