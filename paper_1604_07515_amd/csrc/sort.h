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
