// batch_device.h -- device layout of the batched path: many queries advance
// together, one round-synchronous PR-Nibble round per global step, and the
// queries whose frontier emptied are swept together.
//
// Per batch slot q (dense, like the plain path, so that the scatter needs no
// probing): VRec vr[q*n + v], double p[q*n + v], two frontier buffers
// fbuf[(2q+k)*n + i], a support list and a touched list.  A slot's state is
// reset through its touched list when its query retires, so admitting the
// next query costs O(1).  Round buffers (per-entry coefficient, row, edge
// start, slot) are shared by all slots: a round's entries are the
// concatenation of the scheduled slots' frontiers, in slot order.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_util.h"
#include "plc_device.h"
#include "sort.h"

namespace plc {

enum : int32_t { SL_FREE = 0, SL_PUSH = 1, SL_PUSHED = 2, SL_SWEEP = 3 };

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
  int32_t rnnz, pad;
};

// One query's part of a sweep batch (written by the host before the sweep).
struct __align__(16) SweepSeg {
  int32_t slot;
  int32_t n_elem;           // support size
  long long elem_off;       // first element of the segment
  long long touch_off;      // first touched-list position of the segment (flattened)
  int32_t n_touch;
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
  long long sw_touch_total; // sweep: touched entries
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
  VRec* vr;                 // [B*n]
  double* p;                // [B*n]
  int32_t* fbuf;            // [2*B*n]
  int32_t* support;         // [B*n]
  int32_t* touched;         // [B*n]
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
};

// Admission record (host-written).
struct __align__(16) Admit {
  int32_t slot, seed, rule, max_rounds;
  double alpha, eps;
  int32_t seed_deg, pad;
};

hipError_t launch_batch_init(hipStream_t s, const BatchArgs& a);
hipError_t launch_batch_admit(hipStream_t s, const BatchArgs& a, const Admit* adm, int count);
hipError_t launch_batch_plan_self(hipStream_t s, const BatchArgs& a, int grid_self);
hipError_t launch_batch_scatter(hipStream_t s, const BatchArgs& a, int grid_scatter);
hipError_t launch_batch_round_end(hipStream_t s, const BatchArgs& a);
hipError_t launch_batch_sweep(hipStream_t s, const BatchArgs& a, int nseg, int64_t max_elems,
                              int grid);

}  // namespace plc
