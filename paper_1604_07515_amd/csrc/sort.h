// sort.h -- interface of the device merge sort used by the sweep cut.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace plc {

// Sort element: ordered by (seg, key, id) ascending.
struct __align__(16) SortElem {
  unsigned long long key;  // bit-inverted IEEE pattern of p/d (ascending = non-increasing ratio)
  int32_t id;              // vertex id (or a payload index)
  int32_t seg;             // segment: which query's support this element belongs to
};

struct SortArgs {
  SortElem* buf[2];        // ping-pong buffers; *flip says which holds the data
  const int32_t* count;    // element count (device)
  int32_t* flip;           // 0 or 1 (device); flipped by every merge launch that runs
  unsigned* done;          // last-workgroup counter (device, zero between launches)
  const int32_t* active;   // optional gate: the sort runs only if *active == active_value
  int32_t active_value;
  // Optional: one word per element for the small-count path (the per-element
  // rank accumulators of the one-launch merge); null selects merge passes
  // at every count.
  unsigned long long* rank;
  // Optional side job of the block-sort launch, taken first by its
  // workgroups that hold no tile: for each id in side_ids[0 .. *side_count)
  // (at most side_out_cap of them), the double at side_val[id * side_stride]
  // is read and set to +0.0, and every nonzero one is appended as (id,
  // value) to side_out_id / side_out_val at slots taken from *side_out_cnt
  // (a slot at or past side_out_cap sets *side_fault instead).  The order
  // of the appended pairs is unspecified.  Null side_ids: no side job.
  const int32_t* side_ids = nullptr;
  const int32_t* side_count = nullptr;
  double* side_val = nullptr;
  int side_stride = 0;
  int32_t* side_out_id = nullptr;
  double* side_out_val = nullptr;
  int32_t* side_out_cnt = nullptr;
  long long side_out_cap = 0;
  int32_t* side_fault = nullptr;
};

// Counts up to this many elements take the small-count path when
// SortArgs::rank is set: after the block sort, one launch places every
// element at its rank among all tiles instead of the merge passes.
constexpr int64_t kRankMaxCount = 65536;

// Queue the sort of up to max_count elements (the element count itself is
// read on the device): the small-count path when rank is set and max_count
// is at most kRankMaxCount, else every merge pass needed for max_count
// elements after the block sort (passes beyond the actual count return at
// once).
hipError_t launch_sort(hipStream_t st, const SortArgs& s, int64_t max_count, int grid);

}  // namespace plc
