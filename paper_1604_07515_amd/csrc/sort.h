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
  int32_t* flip;           // 0 or 1 (device); flipped by every merge pass that runs
  unsigned* done;          // last-workgroup counter (device, zero between launches)
  const int32_t* active;   // optional gate: the sort runs only if *active == active_value
  int32_t active_value;
};

// Queue the block sort and every merge pass needed for up to max_count
// elements; passes beyond the actual count return at once.
hipError_t launch_sort(hipStream_t st, const SortArgs& s, int64_t max_count, int grid);

}  // namespace plc
