// sort.hip -- device sort of the sweep order (Sec. 3.1: the support sorted
// by non-increasing p/d).  Elements are (seg, key, id) triples ordered
// lexicographically ascending: seg separates the supports of different
// queries, key is the bit-inverted IEEE pattern of the positive ratio p/d
// (ascending key = non-increasing ratio) and id breaks ties (ascending id).
//
// Merge sort: one launch sorts 1024-element tiles in LDS (bitonic network),
// then each merge pass doubles the sorted run length.  A pass produces
// 1024-element output tiles; the two split points of a tile on the merge
// path are found by a cooperative 128-ary search (a few rounds of parallel
// global loads instead of a serial binary search), the inputs are staged in
// LDS and every thread merges four outputs.  The element count lives in
// device memory; passes whose run length already covers it return at once,
// so the whole sequence is queued without a host round trip.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_util.h"
#include "sort.h"

namespace plc {

constexpr int kSortBlk = 256;
constexpr int kTileS = 1024;        // elements per tile
constexpr int kPerThr = kTileS / kSortBlk;

__device__ __forceinline__ bool elem_lt(const SortElem& a, const SortElem& b) {
  if (a.seg != b.seg) return a.seg < b.seg;
  if (a.key != b.key) return a.key < b.key;
  return a.id < b.id;
}

__device__ __forceinline__ bool sort_enabled(const SortArgs& s) {
  return s.active == nullptr || *s.active == s.active_value;
}

__global__ __launch_bounds__(kSortBlk) void k_block_sort(SortArgs s) {
  if (!sort_enabled(s)) return;
  const int N = *s.count;
  const int flip = *s.flip;
  SortElem* buf = s.buf[flip];
  __shared__ SortElem sh[kTileS];
  const int ntiles = (N + kTileS - 1) / kTileS;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int base = tile * kTileS;
    for (int k = 0; k < kPerThr; k++) {
      int i = k * kSortBlk + threadIdx.x;
      SortElem e;
      if (base + i < N) {
        e = buf[base + i];
      } else {
        e.seg = INT32_MAX; e.key = ~0ull; e.id = INT32_MAX;
      }
      sh[i] = e;
    }
    __syncthreads();
    for (int k = 2; k <= kTileS; k <<= 1) {
      for (int j = k >> 1; j > 0; j >>= 1) {
        for (int q = 0; q < kTileS / 2 / kSortBlk; q++) {
          int p = q * kSortBlk + threadIdx.x;           // pair index 0..511
          int i = 2 * j * (p / j) + (p % j);
          int l = i + j;
          bool up = (i & k) == 0;
          SortElem a = sh[i], b = sh[l];
          if (elem_lt(b, a) == up) { sh[i] = b; sh[l] = a; }
        }
        __syncthreads();
      }
    }
    for (int k = 0; k < kPerThr; k++) {
      int i = k * kSortBlk + threadIdx.x;
      if (base + i < N) buf[base + i] = sh[i];
    }
    __syncthreads();
  }
}

// Merge-path splits of one output tile: the number of A elements among the
// first d0 (threads 0..127) and d1 (threads 128..255) outputs of merge(A, B),
// i.e. the first i with A[i] > B[d-1-i] (or the upper end of the range).
// Found by a cooperative 128-ary search: each round every thread tests one
// position, which shrinks the range by a factor of 128.  Every thread of the
// workgroup must call it; the result for both halves lands in s_res[0..3]
// as (lo, hi) pairs with lo == hi.
__device__ void merge_splits(const SortElem* A, int la, const SortElem* B, int lb, int d0, int d1,
                             int* s_flag /* 256 */, int* s_res /* 4 */) {
  const int half = threadIdx.x >> 7;
  const int t = threadIdx.x & 127;
  if (t == 0) {
    int d = half ? d1 : d0;
    s_res[half * 2] = d - lb > 0 ? d - lb : 0;
    s_res[half * 2 + 1] = d < la ? d : la;
  }
  __syncthreads();
  for (int it = 0; it < 8; it++) {  // 128^5 > 2^31: the loop always converges before 8
    int lo = s_res[half * 2], hi = s_res[half * 2 + 1];
    bool done = s_res[0] == s_res[1] && s_res[2] == s_res[3];
    __syncthreads();
    if (done) break;
    const int d = half ? d1 : d0;
    int span = hi - lo;
    int step = (span + 127) / 128;
    if (step < 1) step = 1;
    int pos = lo + t * step;
    int test = 1;
    if (span > 0 && pos < hi) test = elem_lt(B[d - 1 - pos], A[pos]) ? 1 : 0;
    s_flag[threadIdx.x] = test;
    __syncthreads();
    if (t == 0 && span > 0) {
      int first = 128;
      for (int u = 0; u < 128; u++)
        if (s_flag[half * 128 + u]) { first = u; break; }
      // positions lo + u*step are false for u < first and true at u = first
      int nlo = first == 0 ? lo : lo + (first - 1) * step + 1;
      int cap = lo + first * step;
      int nhi = cap < hi ? cap : hi;
      if (nlo > nhi) nlo = nhi;
      s_res[half * 2] = nlo;
      s_res[half * 2 + 1] = nhi;
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(kSortBlk) void k_merge_pass(SortArgs s, int L) {
  if (!sort_enabled(s)) return;
  const int N = *s.count;
  if (L >= N) return;
  const int flip = *s.flip;
  const SortElem* src = s.buf[flip];
  SortElem* dst = s.buf[flip ^ 1];
  __shared__ SortElem sm[kTileS];
  __shared__ int s_flag[256];
  __shared__ int s_res[4];
  __shared__ int s_last;
  const int ntiles = (N + kTileS - 1) / kTileS;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const long long o0 = (long long)tile * kTileS;
    const long long o1 = o0 + kTileS < N ? o0 + kTileS : N;
    const long long pb = (o0 / (2ll * L)) * (2ll * L);
    const int la = (int)(pb + L < N ? L : N - pb);
    const int lb = (int)(pb + 2ll * L < N ? L : (N - pb - la > 0 ? N - pb - la : 0));
    const SortElem* A = src + pb;
    const SortElem* B = src + pb + la;
    const int d0 = (int)(o0 - pb), d1 = (int)(o1 - pb);
    merge_splits(A, la, B, lb, d0, d1, s_flag, s_res);
    const int a0 = s_res[0], a1 = s_res[2];
    const int b0 = d0 - a0, b1 = d1 - a1;
    const int na = a1 - a0, nb = b1 - b0;
    for (int j = threadIdx.x; j < na + nb; j += kSortBlk)
      sm[j] = j < na ? A[a0 + j] : B[b0 + (j - na)];
    __syncthreads();
    // each thread merges kPerThr consecutive outputs of the tile
    const int d = threadIdx.x * kPerThr;
    if (d < na + nb) {
      int lo = d - nb > 0 ? d - nb : 0;
      int hi = d < na ? d : na;
      while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (elem_lt(sm[na + (d - 1 - mid)], sm[mid])) hi = mid; else lo = mid + 1;
      }
      int ia = lo, ib = d - lo;
      for (int k = 0; k < kPerThr && d + k < na + nb; k++) {
        bool takeA;
        if (ia >= na) takeA = false;
        else if (ib >= nb) takeA = true;
        else takeA = elem_lt(sm[ia], sm[na + ib]);
        dst[o0 + d + k] = takeA ? sm[ia++] : sm[na + ib++];
      }
    }
    __syncthreads();
  }
  if (last_block(s.done, &s_last, false)) {
    if (threadIdx.x == 0) *s.flip = flip ^ 1;
  }
}

hipError_t launch_sort(hipStream_t st, const SortArgs& s, int64_t max_count, int grid) {
  hipLaunchKernelGGL(k_block_sort, dim3(grid), dim3(kSortBlk), 0, st, s);
  for (int64_t L = kTileS; L < max_count; L <<= 1)
    hipLaunchKernelGGL(k_merge_pass, dim3(grid), dim3(kSortBlk), 0, st, s, (int)L);
  return hipGetLastError();
}

}  // namespace plc
