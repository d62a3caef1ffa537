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
//
// Small counts (a bound of at most kRankMaxCount elements known when the
// sort is queued) replace the merge passes with one launch: each element's
// place is its position in its own block-sorted tile plus its count in
// every other tile, found by a binary search in that tile held in LDS, and
// the last of those additions places it.
//
// The block-sort launch can carry a side job (SortArgs::side_ids) for its
// workgroups that hold no tile: with supports of a few tiles most of the
// launch's workgroups would otherwise only exit.
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

// The comparison and the selects take whole elements by value and use no
// short-circuit operators: every field of both operands is loaded up front
// (one 16-byte load each) instead of one dependent load per field compared.
__device__ __forceinline__ bool elem_lt(const SortElem a, const SortElem b) {
  const bool seg_lt = a.seg < b.seg, seg_eq = a.seg == b.seg;
  const bool key_lt = a.key < b.key, key_eq = a.key == b.key;
  return seg_lt | (seg_eq & (key_lt | (key_eq & (a.id < b.id))));
}

__device__ __forceinline__ SortElem elem_sel(bool c, const SortElem a, const SortElem b) {
  SortElem r;
  r.key = c ? a.key : b.key;
  r.id = c ? a.id : b.id;
  r.seg = c ? a.seg : b.seg;
  return r;
}

// Element i of a sorted run in LDS (index through idx), or the largest
// element once i reaches the run's length: the load uses a clamped index,
// so it stays an LDS load and never needs the constant from memory.
template <typename F>
__device__ __forceinline__ SortElem run_head(const SortElem* sh, F idx, int i, int len) {
  const SortElem v = sh[idx(i < len ? i : len - 1)];
  return elem_sel(i < len, v, kMaxElem);
}

__device__ __forceinline__ bool sort_enabled(const SortArgs& s) {
  return s.active == nullptr || *s.active == s.active_value;
}

// Compare-exchange: afterwards a <= b when up, a >= b otherwise.
__device__ __forceinline__ void cswap(SortElem& a, SortElem& b, bool up) {
  const bool sw = elem_lt(b, a) == up;
  const SortElem lo = elem_sel(sw, b, a);
  const SortElem hi = elem_sel(sw, a, b);
  a = lo;
  b = hi;
}

constexpr int kSideItems = 4;                    // side-job entries per thread and step
constexpr int kSideStep = kBSBlk * kSideItems;
constexpr int kSideGrid = 512;                   // block-sort workgroups when a side job rides along

// The block-sort launch's side job (SortArgs::side_ids), in steps of
// kSideStep ids per workgroup: the workgroups are renumbered so that those
// holding no tile take the first steps; the ones that sorted a tile join
// only when there are more steps than workgroups without one.  Each step
// places its nonzeros with one workgroup scan and one global atomic.
__device__ void side_job(const SortArgs& s, int ntiles) {
  long long T = *s.side_count;
  if (T > s.side_out_cap) T = s.side_out_cap;
  if (T <= 0) return;
  __shared__ long long sh[kBSBlk / 64 + 1];
  __shared__ long long s_base;
  const int G = gridDim.x;
  const int busy = ntiles < G ? ntiles : G;
  const int w = ((int)blockIdx.x - busy + G) % G;
  const int t = threadIdx.x;
  for (long long base = (long long)w * kSideStep; base < T; base += (long long)G * kSideStep) {
    int32_t v[kSideItems];
    double x[kSideItems];
#pragma unroll
    for (int k = 0; k < kSideItems; k++) {
      const long long i = base + k * kBSBlk + t;
      v[k] = i < T ? s.side_ids[i] : -1;
    }
#pragma unroll
    for (int k = 0; k < kSideItems; k++)
      x[k] = v[k] >= 0 ? s.side_val[(long long)v[k] * s.side_stride] : 0.0;
    long long cnt = 0;
#pragma unroll
    for (int k = 0; k < kSideItems; k++) {
      if (v[k] >= 0) s.side_val[(long long)v[k] * s.side_stride] = 0.0;
      cnt += x[k] != 0.0;
    }
    long long tot;
    const long long off = block_excl_scan<kBSBlk>(cnt, &tot, sh);
    if (t == 0) s_base = tot > 0 ? atomicAdd(s.side_out_cnt, (int32_t)tot) : 0;
    __syncthreads();
    long long slot = s_base + off;
#pragma unroll
    for (int k = 0; k < kSideItems; k++) {
      if (x[k] != 0.0) {
        if (slot < s.side_out_cap) {
          s.side_out_id[slot] = v[k];
          s.side_out_val[slot] = x[k];
        } else {
          *s.side_fault = 1;
        }
        slot++;
      }
    }
    __syncthreads();
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
      const int gi = base + i < N ? base + i : N - 1;
      sh[lds_pad(i)] = elem_sel(base + i < N, buf[gi], kMaxElem);
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
        const SortElem b = sh[lds_pad(B + d - 1 - mid)];
        const SortElem a = sh[lds_pad(A + mid)];
        if (elem_lt(b, a)) hi = mid; else lo = mid + 1;
      }
      // the two run heads stay in registers; an exhausted run shows the
      // largest element, equal to the tile padding, so either choice
      // between the two then outputs the same value
      int ia = lo, ib = d - lo;
      SortElem ha = run_head(sh, [&](int i) { return lds_pad(A + i); }, ia, L);
      SortElem hb = run_head(sh, [&](int i) { return lds_pad(B + i); }, ib, L);
#pragma unroll
      for (int k = 0; k < kBT; k++) {
        const bool ta = !elem_lt(hb, ha);
        x[k] = elem_sel(ta, ha, hb);
        ia += ta;
        ib += !ta;
        // one load: the next head of the run just taken
        const int r0 = ta ? A : B;
        const int ri = ta ? ia : ib;
        const SortElem nx = run_head(sh, [&](int i) { return lds_pad(r0 + i); }, ri, L);
        ha = elem_sel(ta, nx, ha);
        hb = elem_sel(ta, hb, nx);
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < kBT; k++) sh[lds_pad(o + k)] = x[k];
      __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < kBT; k++) {
      const int i = k * kBSBlk + t;
      if (base + i < N) {
        buf[base + i] = sh[lds_pad(i)];
        if (s.rank != nullptr) s.rank[base + i] = (unsigned long long)i;
      }
    }
    __syncthreads();
  }
  if (s.side_ids != nullptr) side_job(s, ntiles);
}

// ------------------------------------------------------ small-count path

constexpr int kRankBlk = 512;                          // threads of the rank merge
constexpr int kRankGrid = 512;                         // its workgroups, split among the tiles
static_assert(kRankMaxCount % kTileB == 0, "whole block-sort tiles");

// Places every element of the block-sorted tiles at its rank in the whole
// order.  Workgroup (j, g) of the per workgroups of tile j holds tile j in
// LDS and takes every per-th element outside it: each lane counts the
// elements of tile j that precede its element (those not greater when tile
// j comes first, those less when it comes later, so equal elements of
// different tiles keep tile order) and adds the count to the element's rank
// word (set by the block sort to its position in its own tile), whose upper
// half counts the additions; the addition that completes the T - 1 of them
// writes the element out.  Tiles beyond tiles_max (a count above the bound
// the launch was sized for) are taken in further turns.
__global__ __launch_bounds__(kRankBlk) void k_rank_merge(SortArgs s, int tiles_max, int per) {
  if (!sort_enabled(s)) return;
  const int N = *s.count;
  const int T = (N + kTileB - 1) / kTileB;
  if (T <= 1) return;
  const int flip = *s.flip;
  const SortElem* src = s.buf[flip];
  SortElem* dst = s.buf[flip ^ 1];
  __shared__ SortElem sh[kTileB];
  __shared__ int s_last;
  const int g = blockIdx.x % per;
  for (int j = blockIdx.x / per; j < T; j += tiles_max) {
    const int base = j * kTileB;
    const int len = N - base < kTileB ? N - base : kTileB;
    __syncthreads();
    for (int x = threadIdx.x; x < len; x += kRankBlk) sh[x] = src[base + x];
    __syncthreads();
    const int others = N - len;
    for (int q = g * kRankBlk + threadIdx.x; q < others; q += per * kRankBlk) {
      const int k = q < base ? q : q + len;
      const SortElem e = src[k];
      int lo = 0, hi = len;
      if (k >= base) {
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (elem_lt(e, sh[mid])) hi = mid; else lo = mid + 1;
        }
      } else {
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (elem_lt(sh[mid], e)) lo = mid + 1; else hi = mid;
        }
      }
      const unsigned long long old = atomicAdd(&s.rank[k], (1ull << 32) | (unsigned long long)lo);
      if ((int)(old >> 32) == T - 2) dst[(long long)(old & 0xffffffffull) + lo] = e;
    }
  }
  if (last_block(s.done, &s_last, false)) {
    if (threadIdx.x == 0) *s.flip = flip ^ 1;
  }
}

// ------------------------------------------------------------ merge passes

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

// Element i of the run of length len staged at sm[r0..], or the largest
// element past its end; the index is clamped into the staging tile so the
// load is always an in-bounds LDS load.
__device__ __forceinline__ SortElem staged_head(const SortElem* sm, int r0, int i, int len) {
  int li = r0 + (i < len ? i : len - 1);
  li = li < 0 ? 0 : (li < kTileS ? li : kTileS - 1);
  return elem_sel(i < len, sm[li], kMaxElem);
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
      // run heads in registers, an exhausted run showing the largest
      // element (no element of a sort equals it)
      SortElem ha = staged_head(sm, 0, ia, na);
      SortElem hb = staged_head(sm, na, ib, nb);
      for (int k = 0; k < kPerThr && d + k < na + nb; k++) {
        const bool ta = !elem_lt(hb, ha);
        dst[o0 + d + k] = elem_sel(ta, ha, hb);
        ia += ta;
        ib += !ta;
        const SortElem nx = staged_head(sm, ta ? 0 : na, ta ? ia : ib, ta ? na : nb);
        ha = elem_sel(ta, nx, ha);
        hb = elem_sel(ta, hb, nx);
      }
    }
    __syncthreads();
  }
  if (last_block(s.done, &s_last, false)) {
    if (threadIdx.x == 0) *s.flip = flip ^ 1;
  }
}

hipError_t launch_sort(hipStream_t st, const SortArgs& s, int64_t max_count, int grid) {
  // a side job takes the workgroups without a tile: two per CU fit the
  // tile's LDS, so up to that many keep the gather from outlasting the sort
  const int bs_grid = s.side_ids != nullptr && grid < kSideGrid ? kSideGrid : grid;
  hipLaunchKernelGGL(k_block_sort, dim3(bs_grid), dim3(kBSBlk), 0, st, s);
  if (s.rank != nullptr && max_count <= kRankMaxCount) {
    const int tiles = (int)((max_count + kTileB - 1) / kTileB);
    if (tiles > 1) {
      const int per = kRankGrid / tiles;
      hipLaunchKernelGGL(k_rank_merge, dim3(tiles * per), dim3(kRankBlk), 0, st, s, tiles, per);
    }
    return hipGetLastError();
  }
  for (int64_t L = kTileB; L < max_count; L <<= 1)
    hipLaunchKernelGGL(k_merge_pass, dim3(grid), dim3(kSortBlk), 0, st, s, (int)L);
  return hipGetLastError();
}

}  // namespace plc
