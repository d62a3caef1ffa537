// sort.hip -- device sort of the sweep order (Sec. 3.1: the support sorted
// by non-increasing p/d).  Elements are (seg, key, id) triples ordered
// lexicographically ascending: seg separates the supports of different
// queries, key is the bit-inverted IEEE pattern of the positive ratio p/d
// (ascending key = non-increasing ratio) and id breaks ties (ascending id).
//
// Merge sort: one launch sorts 4096-element tiles in LDS (each of 512
// threads sorts 8 elements in registers with a bitonic network, then nine
// rounds of merge-path merges in LDS double the sorted runs up to the tile),
// then
// each merge pass doubles the sorted run length.  A pass produces
// 1024-element output tiles; the two split points of a tile on the merge
// path are found by a cooperative 128-ary search (a few rounds of parallel
// global loads, each resolved with wave ballots instead of a serial binary
// search), the inputs are staged in LDS and every thread merges four
// outputs.  The element count lives in
// device memory; passes whose run length already covers it return at once,
// so the whole sequence is queued without a host round trip.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_util.h"
#include "sort.h"

namespace plc {

constexpr int kSortBlk = 256;
constexpr int kTileS = 1024;        // elements per merge-pass output tile
constexpr int kPerThr = kTileS / kSortBlk;
constexpr int kBSBlk = 512;         // threads of the block sort
constexpr int kBT = 8;              // elements per thread in the block sort
constexpr int kTileB = kBSBlk * kBT;    // elements per block-sort tile

// The largest element: pads a tile past the element count.
constexpr SortElem kMaxElem = {~0ull, INT32_MAX, INT32_MAX};

// LDS index of element i of a block-sort tile: one spare slot after every
// kBT elements, so the kBT-element rows of consecutive threads start on
// different banks.
__device__ __forceinline__ int lds_pad(int i) { return i + i / kBT; }

__device__ __forceinline__ bool elem_lt(const SortElem& a, const SortElem& b) {
  if (a.seg != b.seg) return a.seg < b.seg;
  if (a.key != b.key) return a.key < b.key;
  return a.id < b.id;
}

__device__ __forceinline__ bool sort_enabled(const SortArgs& s) {
  return s.active == nullptr || *s.active == s.active_value;
}

// Compare-exchange: afterwards a <= b when up, a >= b otherwise.
__device__ __forceinline__ void cswap(SortElem& a, SortElem& b, bool up) {
  if (elem_lt(b, a) == up) {
    SortElem t = a;
    a = b;
    b = t;
  }
}

__global__ __launch_bounds__(kBSBlk) void k_block_sort(SortArgs s) {
  if (!sort_enabled(s)) return;
  const int N = *s.count;
  const int flip = *s.flip;
  SortElem* buf = s.buf[flip];
  __shared__ SortElem sh[kTileB + kTileB / kBT];
  const int ntiles = (N + kTileB - 1) / kTileB;
  const int t = threadIdx.x;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int base = tile * kTileB;
    // coalesced load (element k*256 + t), padded past N with the largest element
#pragma unroll
    for (int k = 0; k < kBT; k++) {
      const int i = k * kBSBlk + t;
      sh[lds_pad(i)] = base + i < N ? buf[base + i] : kMaxElem;
    }
    __syncthreads();
    // elements kBT*t .. kBT*t + kBT - 1, sorted in registers (bitonic network)
    SortElem x[kBT];
#pragma unroll
    for (int k = 0; k < kBT; k++) x[k] = sh[lds_pad(t * kBT + k)];
#pragma unroll
    for (int k = 2; k <= kBT; k <<= 1) {
#pragma unroll
      for (int j = k >> 1; j > 0; j >>= 1) {
#pragma unroll
        for (int i = 0; i < kBT; i++) {
          const int l = i ^ j;
          if (l > i) cswap(x[i], x[l], (i & k) == 0);
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kBT; k++) sh[lds_pad(t * kBT + k)] = x[k];
    __syncthreads();
    // merge runs of L into runs of 2L; thread t produces outputs
    // [kBT*t, kBT*t + kBT) of the tile, i.e. diagonal d of its pair of runs
    for (int L = kBT; L < kTileB; L <<= 1) {
      const int o = t * kBT;
      const int pb = (o / (2 * L)) * (2 * L);
      const int d = o - pb;
      const int A = pb, B = pb + L;  // run starts (tile positions)
      int lo = d - L > 0 ? d - L : 0;
      int hi = d < L ? d : L;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (elem_lt(sh[lds_pad(B + d - 1 - mid)], sh[lds_pad(A + mid)])) hi = mid; else lo = mid + 1;
      }
      // the two run heads stay in registers; an exhausted run shows the
      // largest element, equal to the tile padding, so either choice
      // between the two then outputs the same value
      int ia = lo, ib = d - lo;
      SortElem ha = ia < L ? sh[lds_pad(A + ia)] : kMaxElem;
      SortElem hb = ib < L ? sh[lds_pad(B + ib)] : kMaxElem;
#pragma unroll
      for (int k = 0; k < kBT; k++) {
        if (!elem_lt(hb, ha)) {
          x[k] = ha;
          ia++;
          ha = ia < L ? sh[lds_pad(A + ia)] : kMaxElem;
        } else {
          x[k] = hb;
          ib++;
          hb = ib < L ? sh[lds_pad(B + ib)] : kMaxElem;
        }
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < kBT; k++) sh[lds_pad(o + k)] = x[k];
      __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < kBT; k++) {
      const int i = k * kBSBlk + t;
      if (base + i < N) buf[base + i] = sh[lds_pad(i)];
    }
    __syncthreads();
  }
}

// Merge-path splits of one output tile: the number of A elements among the
// first d0 (threads 0..127) and d1 (threads 128..255) outputs of merge(A, B),
// i.e. the first i with A[i] > B[d-1-i] (or the upper end of the range).
// Found by a cooperative 128-ary search: each round every thread tests one
// position, which shrinks the range by a factor of 128; the tests are
// monotone in the position, so the first true one is the count of false
// ones, summed from the two wave ballots of the half.  Every thread of the
// workgroup must call it; the splits of both halves land in s_res[0..1].
__device__ void merge_splits(const SortElem* A, int la, const SortElem* B, int lb, int d0, int d1,
                             int* s_cnt /* 4 */, int* s_done /* 2 */, int* s_res /* 2 */) {
  const int half = threadIdx.x >> 7;
  const int t = threadIdx.x & 127;
  const int wave = threadIdx.x >> 6;
  const int d = half ? d1 : d0;
  int lo = d - lb > 0 ? d - lb : 0;
  int hi = d < la ? d : la;
  for (int it = 0; it < 8; it++) {  // 128^5 > 2^31: the loop always converges before 8
    if (t == 0) s_done[half] = lo == hi;
    __syncthreads();
    const bool done = s_done[0] && s_done[1];
    if (done) break;
    const int span = hi - lo;
    int step = (span + 127) / 128;
    if (step < 1) step = 1;
    const int pos = lo + t * step;
    bool test = true;
    if (span > 0 && pos < hi) test = elem_lt(B[d - 1 - pos], A[pos]);
    const unsigned long long falses = __ballot(!test);
    if ((threadIdx.x & 63) == 0) s_cnt[wave] = __popcll(falses);
    __syncthreads();
    if (span > 0) {
      // positions lo + u*step are false for u < first and true at u = first
      const int first = s_cnt[2 * half] + s_cnt[2 * half + 1];
      int nlo = first == 0 ? lo : lo + (first - 1) * step + 1;
      const int cap = lo + first * step;
      const int nhi = cap < hi ? cap : hi;
      if (nlo > nhi) nlo = nhi;
      lo = nlo;
      hi = nhi;
    }
  }
  if (t == 0) s_res[half] = lo;
  __syncthreads();
}

__global__ __launch_bounds__(kSortBlk) void k_merge_pass(SortArgs s, int L) {
  if (!sort_enabled(s)) return;
  const int N = *s.count;
  if (L >= N) return;
  const int flip = *s.flip;
  const SortElem* src = s.buf[flip];
  SortElem* dst = s.buf[flip ^ 1];
  __shared__ SortElem sm[kTileS];
  __shared__ int s_cnt[4], s_done[2], s_res[2];
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
    merge_splits(A, la, B, lb, d0, d1, s_cnt, s_done, s_res);
    const int a0 = s_res[0], a1 = s_res[1];
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
  hipLaunchKernelGGL(k_block_sort, dim3(grid), dim3(kBSBlk), 0, st, s);
  for (int64_t L = kTileB; L < max_count; L <<= 1)
    hipLaunchKernelGGL(k_merge_pass, dim3(grid), dim3(kSortBlk), 0, st, s, (int)L);
  return hipGetLastError();
}

}  // namespace plc
