// plc_device.h -- device-side data layout and kernel entry points of libplc.
//
// HBM layout for one resident graph (all inside the caller's arena):
//   off   int64[n+1]     CSR row offsets
//   nbr   int32[2m]      neighbour ids, rows sorted
//   vr    VRec[n]        per-vertex record {r, d(v), sweep rank}: the edge
//                        scatter's atomic on r and its read of d(w) hit one
//                        16-byte record, i.e. one cache line
//   p     double[n]      approximate PageRank vector
// plus the plain-path work buffers sized by n (frontier ping-pong, per-entry
// coefficients and edge starts, support and touched lists, sweep buffers).
// Dense per-vertex state is reset after every query through the touched list,
// so a query's cost stays proportional to the vertices it touched.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace plc {

struct __align__(16) VRec {
  double r;      // residual; +0.0 = never touched by this query, -0.0 = pushed (optimized rule)
  int32_t deg;   // d(v), constant for the graph
  int32_t rank;  // sweep rank 1..N while a sweep runs, 0 otherwise
};

// Single-pass scan (decoupled look-back) descriptor, one per block of items.
struct __align__(8) ScanDesc {
  unsigned long long tag;  // (epoch << 2) | flag ; flag 0 = none, 1 = aggregate, 2 = prefix
  long long agg;           // block aggregate, valid once flag >= 1
  long long incl;          // inclusive prefix, valid once flag == 2
  long long pad;
};

// Query status in the control block.  ST_PUSH: rounds in progress (done when
// the current frontier is empty); ST_LIMIT: watchdog fired, sweep the partial
// p; ST_SWEEPING: sweep kernels running; ST_SWEPT: results ready.
enum : int32_t { ST_IDLE = 0, ST_PUSH = 1, ST_SWEPT = 2, ST_LIMIT = 4, ST_SWEEPING = 6 };

// Scan sites (each has its own descriptor array, ticket and epoch).
enum : int32_t { SCAN_FRONTIER = 0, SCAN_VOL = 1, SCAN_CUT = 2, NUM_SCANS = 3 };

// Device control block of one plain-path query.  Written by kernels only,
// except at query start (plc_init_query kernel) and read back by the host.
struct __align__(64) Ctl {
  // query parameters
  double cs, cn, keep, eps;
  int32_t seed, rule, max_rounds, opt_rule;  // opt_rule = 1 for the optimized rule
  // round state
  int32_t status;
  int32_t round;          // rounds pushed so far; frontier of round t is fbuf[t&1], size cnt[t&1]
  int32_t cnt[3];
  int32_t ntiles;         // edge tiles of the current round
  long long etotal;       // sum of degrees of the current frontier
  long long pushes, edges;
  int32_t support_cnt;    // |support list|
  int32_t touched_cnt;    // |touched list|
  int32_t overflow;       // set if an append would exceed its buffer (never expected)
  int32_t limited;        // the watchdog stopped the rounds
  // scans
  unsigned int ticket[NUM_SCANS];
  unsigned int pad1;
  unsigned long long epoch[NUM_SCANS];
  unsigned int done[4];   // last-block counters
  // sweep
  int32_t N;              // support size
  int32_t sort_flip;      // radix ping-pong parity (0: data in A, 1: in B)
  int32_t pass_trivial;   // current radix pass has a single populated digit
  int32_t rnnz;
  long long vol_total;    // 2m
  long long best_cut, best_vol, best_den;
  long long kstar;
  double phi;
};

// Arguments shared by the plain-path kernels (all device pointers).
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
  int64_t* estart;     // per entry: global start of its edges in the round's edge sequence
  int64_t* rowp;       // per entry: off[v]
  int32_t* tile_start; // per edge tile: first entry overlapping it
  ScanDesc* desc[NUM_SCANS];
  int32_t* support;
  int32_t* touched;
  // sweep
  unsigned long long* keyA;
  unsigned long long* keyB;
  int32_t* idA;
  int32_t* idB;
  uint32_t* hist;      // radix histograms [256][max tiles]
  int32_t* sdeg;       // degree in sweep order
  int64_t* svol;       // inclusive volume prefix in sweep order
  int32_t* scnt;       // # earlier-ranked neighbours per sweep position
  double* sp;          // p in sweep order
  int32_t* rid;        // r nonzero ids
  double* rval;        // r nonzero values
  long long* bbest;    // per-block argmin candidates (cut, den, k) triples
  int32_t hist_tiles;  // capacity of hist per digit
  int64_t tile_cap;    // capacity of tile_start
  int32_t id_bits;     // bits needed for a vertex id
};

// Launch configuration.
constexpr int kBlock = 256;             // threads per workgroup
constexpr int kScanItems = 4;           // items per thread in scan-type kernels
constexpr int kScanBlock = kBlock * kScanItems;  // items per scan block
constexpr int kEdgeTile = 1024;         // edges per scatter / cut tile
constexpr int kSortTile = 2048;         // elements per radix tile
constexpr int kSortItems = kSortTile / kBlock;

// Host-side launchers (return hipError_t of the launch).
hipError_t launch_graph_init(hipStream_t s, const PlainArgs& a);
hipError_t launch_query_init(hipStream_t s, const PlainArgs& a, int32_t seed, int32_t rule,
                             double alpha, double eps, int32_t max_rounds);
hipError_t launch_self(hipStream_t s, const PlainArgs& a, int grid);
hipError_t launch_scatter(hipStream_t s, const PlainArgs& a, int grid);
hipError_t launch_sweep(hipStream_t s, const PlainArgs& a, int grid);
hipError_t launch_cleanup(hipStream_t s, const PlainArgs& a, int grid);

}  // namespace plc
