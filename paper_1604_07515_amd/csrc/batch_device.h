// batch_device.h -- device layout of the batched path: many queries advance
// together, one round-synchronous PR-Nibble round per global step, and the
// queries whose frontier emptied are swept together.
//
// Every slot q reaches its state through pointers in its Slot record (set by
// the host at admission):
//   tab   16-byte records {r, d or key, rank}
//   tp    p, parallel to tab
//   fb[2] frontier buffers, support, touched: vertex-id lists of list_cap
// Two state layouts share the kernels (a template parameter):
//   dense   (DenseState)   tab/tp are the slot's slices of engine-wide
//           arrays indexed by vertex id (n records per slot), like the plain
//           path; the scatter's atomic needs no probing.  Reset through the
//           touched list when the query retires.
//   compact (CompactState) tab/tp are a per-query open-addressing table of
//           tcap records (a multiple of 1024, linear probing from a
//           multiply-high home position; sized so that it is at most half
//           full and at most 3/4 full after the next round's worst case),
//           allocated from the arena at admission and grown between rounds,
//           so a query holds memory in proportion to the vertices it
//           touched rather than to n.  d(v) and the hot code sit in the
//           record beside the key (claimed with it in one 64-bit
//           compare-and-swap, from a graph-wide array), so the scatter's
//           probe returns them.
// Round buffers (per-entry coefficient, row, edge start, slot) are shared by
// all slots: a round's entries are the concatenation of the scheduled slots'
// frontiers, in slot order.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_util.h"
#include "plc_device.h"
#include "sort.h"

namespace plc {

enum : int32_t { SL_FREE = 0, SL_PUSH = 1, SL_PUSHED = 2, SL_SWEEP = 3 };

constexpr int32_t kEmptyKey = -1;  // key of a free compact-table record

struct __align__(64) Slot {
  double cs, cn, keep, eps;
  int32_t opt, status, seed, max_rounds;
  int32_t par;              // frontier buffer of the current round
  int32_t cnt[2];           // frontier sizes
  int32_t rounds;
  long long edge_next[2];   // sum of degrees of the vertices in frontier buffer k
  long long pushes, edges;
  int32_t support_cnt, touched_cnt;
  int32_t fbase;            // first entry of this slot in the round (-1: not scheduled)
  int32_t nf;               // entries scheduled this round
  int32_t limited, fault;
  long long round_edges;    // edges scheduled this round
  // sweep results
  long long kstar, best_cut, best_vol, best_den;
  double phi;
  int32_t rnnz;
  int32_t hold;             // compact: 1 = skip rounds until the table has grown
  // state (see above)
  VRec* tab;
  double* tp;
  int32_t* fb[2];
  int32_t* support;
  int32_t* touched;
  int32_t tcap;             // compact: table capacity (records)
  int32_t list_cap;         // capacity of each list
  // constant-rate clock (wall_clock64) at admission and at the sweep's argmin
  long long t_admit, t_done;
};

// One query's part of a sweep batch (written by the host before the sweep).
struct __align__(16) SweepSeg {
  int32_t slot;
  int32_t n_elem;           // support size
  long long elem_off;       // first element of the segment
  long long touch_off;      // first finish entry of the segment (flattened): touched-list
                            // positions (dense) or table records (compact)
  int32_t n_touch;          // touched-list length (dense) or table capacity (compact)
  int32_t pad;
  int32_t* out_ids;         // support in sweep order (NULL: discard the vectors)
  double* out_p;            // p at those vertices
  int32_t* out_rid;         // nonzeros of r
  double* out_rval;
};

enum : int32_t { BSCAN_FRONTIER = 0, BSCAN_VOL = 1, BSCAN_CUT = 2, BNUM_SCANS = 3 };

struct __align__(64) BatchCtl {
  int32_t nf_total;         // entries this round
  int32_t ntiles;           // edge tiles this round (or of the sweep)
  long long e_total;        // edges this round (or sweep volume)
  int32_t fault;
  int32_t sort_flip;
  int32_t sw_nseg;          // sweep: segments
  int32_t sw_total;         // sweep: elements
  long long sw_touch_total; // sweep: finish entries
  long long sw_etotal;      // sweep: volume of all swept supports
  int32_t sw_ntiles;        // sweep: edge tiles
  int32_t pad0;
  ScanSite scan[BNUM_SCANS];
  unsigned int done[8];
};

struct BatchArgs {
  int64_t n;
  long long vol_total;
  const int64_t* off;
  const int32_t* nbr;
  int32_t B;                // slots
  Slot* slots;
  VRec* vr;                 // dense: [B*n]
  double* p;                // dense: [B*n]
  BatchCtl* ctl;
  // round buffers
  int32_t* fprefix;         // [B+1]
  int32_t* eslot;           // [nf_cap]
  double* coef;             // [nf_cap]
  int64_t* estart;          // [nf_cap]
  int64_t* rowp;            // [nf_cap]
  int32_t nf_cap;
  long long e_cap;
  int32_t* tile_start;      // [tile_cap]
  int64_t tile_cap;
  unsigned long long* desc[BNUM_SCANS];
  int32_t desc_cap;
  // sweep buffers
  SweepSeg* segs;           // [B]
  SortElem* sbuf[2];        // [s_cap]
  int32_t* sdeg;            // [s_cap]
  int64_t* svol;            // [s_cap]
  int32_t* scnt;            // [s_cap]
  int64_t* scut;            // [s_cap]
  int64_t s_cap;
  const int32_t* hot_ids;   // [kHot] vertex of hot index j (graph-wide)
  const int32_t* hotcode;   // [n] -(j+1) for hot vertex j, else 0
  const int2* gdh;          // [n] {d(v), hot code} (graph-wide; compact layout)
};

// Admission record (host-written): the query and the slot's state pointers.
struct __align__(16) Admit {
  int32_t slot, seed, rule, max_rounds;
  double alpha, eps;
  int32_t seed_deg, tcap, list_cap, pad;
  VRec* tab;
  double* tp;
  int32_t* fb0;
  int32_t* fb1;
  int32_t* support;
  int32_t* touched;
};

// Compact layout: a table that moves to a larger block (host-written).
struct __align__(16) Grow {
  int32_t slot;
  int32_t old_cap, new_cap, list_cap;
  long long rec_off;        // first record of this table in the flattened rehash index
  long long list_off;       // first list entry of this slot in the flattened copy index
  int32_t par;              // current frontier buffer
  int32_t n_front, n_sup, n_touch;  // list lengths to move (host copy of the slot)
  VRec* tab;
  double* tp;
  int32_t* fb0;
  int32_t* fb1;
  int32_t* support;
  int32_t* touched;
};

// Compact layout: one table block to clear (host-written); off = first
// record of this job in the flattened index over all jobs of a launch.
struct __align__(16) ClearJob {
  VRec* tab;
  double* tp;
  long long cap;
  long long off;
};

hipError_t launch_batch_init(hipStream_t s, const BatchArgs& a);      // dense layout
hipError_t launch_gdh_init(hipStream_t s, const BatchArgs& a, int2* gdh);  // compact layout
hipError_t launch_batch_admit(hipStream_t s, const BatchArgs& a, const Admit* adm, int count,
                              bool compact);
hipError_t launch_batch_plan_self(hipStream_t s, const BatchArgs& a, int grid_self, bool compact);
// With t0 set: launched with start and stop events on its own dispatch
// timestamps (hipExtLaunchKernelGGL); not for graph capture.
hipError_t launch_batch_scatter(hipStream_t s, const BatchArgs& a, int grid_scatter,
                                bool compact, hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr);
hipError_t launch_batch_round_end(hipStream_t s, const BatchArgs& a);
hipError_t launch_batch_sweep(hipStream_t s, const BatchArgs& a, int nseg, int64_t max_elems,
                              int grid, bool compact);
// compact layout: clear table blocks (records and p), move grown tables,
// set the slots' hold flags (holds[i] = slot | flag << 16)
hipError_t launch_table_clear(hipStream_t s, const ClearJob* jobs, int count, long long total,
                              int grid);
hipError_t launch_table_grow(hipStream_t s, const BatchArgs& a, const Grow* gr, int count,
                             long long total_old, long long total_list, int grid);
hipError_t launch_slot_hold(hipStream_t s, const BatchArgs& a, const int32_t* holds, int count);

}  // namespace plc
