// device_util.h -- wavefront / workgroup building blocks shared by the
// libplc kernels (CDNA, 64-lane wavefronts, 256-thread workgroups).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace plc {

#define PLC_LANE (threadIdx.x & 63)
#define PLC_WID (threadIdx.x >> 6)

__device__ __forceinline__ unsigned long long lanemask_lt() {
  unsigned l = PLC_LANE;
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

__device__ __forceinline__ long long wave_incl_scan(long long x) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    long long y = __shfl_up(x, o);
    if ((int)PLC_LANE >= o) x += y;
  }
  return x;
}

// Exclusive scan over a workgroup of NT threads; sh holds NT/64 + 1 slots.
template <int NT>
__device__ __forceinline__ long long block_excl_scan(long long x, long long* total, long long* sh) {
  constexpr int NW = NT / 64;
  long long inc = wave_incl_scan(x);
  if (PLC_LANE == 63) sh[PLC_WID] = inc;
  __syncthreads();
  if (threadIdx.x < 64) {
    long long v = (int)threadIdx.x < NW ? sh[threadIdx.x] : 0;
    long long vi = wave_incl_scan(v);
    if ((int)threadIdx.x < NW) sh[threadIdx.x] = vi - v;
    if ((int)threadIdx.x == NW - 1) sh[NW] = vi;
  }
  __syncthreads();
  long long ex = inc - x + sh[PLC_WID];
  *total = sh[NW];
  __syncthreads();
  return ex;
}

// ----------------------------------------------------------- look-back scan
//
// Single-pass (decoupled look-back) scan over blocks taken in ticket order.
// One 64-bit word per block holds the flag (bits 63..62: 0 none,
// 1 aggregate, 2 inclusive prefix) and a 62-bit two's-complement value, so a
// reader never needs a memory fence between flag and value.  Each scan site
// owns two descriptor buffers used on alternate launches; every launch clears
// the slots the previous launch used in the other buffer, so the next launch
// starts from zeroed flags.

struct ScanSite {
  unsigned int ticket;   // next block ticket
  unsigned int parity;   // descriptor buffer of the current launch
  int prev_nblk;         // blocks used by the previous launch
  int pad;
};

__device__ __forceinline__ unsigned long long desc_pack(unsigned flag, long long v) {
  return ((unsigned long long)flag << 62) | ((unsigned long long)v & ((1ull << 62) - 1));
}
__device__ __forceinline__ long long desc_value(unsigned long long w) {
  return ((long long)(w << 2)) >> 2;
}
__device__ __forceinline__ unsigned long long atomic_ld64(unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void atomic_st64(unsigned long long* p, unsigned long long v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

constexpr long kSpinLimit = 1L << 24;

// Clear the other buffer's slots used by the previous launch (all workgroups
// share the work).  Call once per workgroup at kernel start.
__device__ __forceinline__ void scan_clear_prev(ScanSite* site, unsigned long long* desc2,
                                                int cap) {
  unsigned par = site->parity;
  int prev = site->prev_nblk;
  if (prev > cap) prev = cap;
  unsigned long long* other = desc2 + (size_t)(par ^ 1u) * cap;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < prev; j += gridDim.x * blockDim.x)
    other[j] = 0ull;
}

// Decoupled look-back for block b, by the 64 lanes of wave 0 together (call
// from threads 0..63; every lane gets the result).  Each round reads the
// descriptors of the 64 nearest unresolved predecessors at once and sums
// back to the nearest inclusive prefix; lanes past block 0 count as an
// inclusive prefix of 0.  A round that meets a predecessor without a
// descriptor before any inclusive one waits and reads again.  Predecessors
// claimed their tickets earlier, so they are running or done; the wait is
// bounded and raises *fault if it ever runs out.  Returns the exclusive
// prefix.
__device__ long long scan_lookback(unsigned long long* desc, int b, long long agg, int* fault) {
  const int lane = PLC_LANE;
  if (b == 0) {
    if (lane == 0) atomic_st64(&desc[0], desc_pack(2, agg));
    return 0;
  }
  if (lane == 0) atomic_st64(&desc[b], desc_pack(1, agg));
  long long excl = 0;
  int j = b - 1;  // nearest predecessor not yet summed
  long spins = 0;
  for (;;) {
    const int idx = j - lane;
    const unsigned long long w = idx >= 0 ? atomic_ld64(&desc[idx]) : desc_pack(2, 0);
    const unsigned flag = (unsigned)(w >> 62);
    const unsigned long long incl = __ballot(flag == 2);
    const unsigned long long none = __ballot(flag == 0);
    const int fi = incl ? __ffsll((long long)incl) - 1 : 64;
    const int fz = none ? __ffsll((long long)none) - 1 : 64;
    if (fz < fi) {
      if (++spins > kSpinLimit) {
        if (lane == 0) atomicExch(fault, 1);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
      continue;
    }
    long long v = lane <= fi ? desc_value(w) : 0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    excl += v;
    if (fi < 64) break;
    j -= 64;
  }
  if (lane == 0) atomic_st64(&desc[b], desc_pack(2, excl + agg));
  return excl;
}

// Ticket dispenser.  Returns the next block index (>= nblk when exhausted).
// The workgroup drawing the last ticket (nblk + gridDim.x - 1) retires the
// launch: it resets the dispenser, flips the descriptor buffer and records
// nblk for the next launch's clearing pass.  *is_last tells the caller.
__device__ __forceinline__ int scan_ticket(ScanSite* site, int nblk, int* sh, bool* is_last) {
  if (threadIdx.x == 0) {
    unsigned t = atomicAdd(&site->ticket, 1u);
    int last = 0;
    if (t == (unsigned)nblk + gridDim.x - 1) {
      site->ticket = 0;
      site->parity ^= 1u;
      site->prev_nblk = nblk;
      last = 1;
    }
    sh[0] = (int)t;
    sh[1] = last;
  }
  __syncthreads();
  int b = sh[0];
  *is_last = sh[1] != 0;
  __syncthreads();
  return b;
}

// Last-workgroup detection: true in exactly one workgroup, after all others
// of the launch called it.  with_acquire makes the other workgroups' global
// writes visible to the last one (device-scope fences).
// last_block_of: the same among the first `members` workgroups only (the
// others must not call it).
__device__ __forceinline__ bool last_block_of(unsigned* done, int* sh, bool with_acquire,
                                              unsigned members) {
  __syncthreads();
  if (threadIdx.x == 0) {
    if (with_acquire) __threadfence();
    unsigned prev = atomicAdd(done, 1u);
    int last = prev == members - 1;
    if (last) {
      if (with_acquire) __threadfence();
      *done = 0;
    }
    *sh = last;
  }
  __syncthreads();
  int l = *sh;
  __syncthreads();
  return l != 0;
}

__device__ __forceinline__ bool last_block(unsigned* done, int* sh, bool with_acquire) {
  __syncthreads();
  if (threadIdx.x == 0) {
    if (with_acquire) __threadfence();
    unsigned prev = atomicAdd(done, 1u);
    int last = prev == gridDim.x - 1;
    if (last) {
      if (with_acquire) __threadfence();
      *done = 0;
    }
    *sh = last;
  }
  __syncthreads();
  int l = *sh;
  __syncthreads();
  return l != 0;
}

// Wavefront-ballot append into an LDS staging buffer: the lanes of the
// calling wave with pred set store v at consecutive slots of buf, reserved
// with one LDS atomic per wave (the popcount of the ballot); a lane's slot
// is the number of set lanes below it.  Safe in divergent code: only the
// active lanes take part.
__device__ __forceinline__ void wave_append(bool pred, int32_t v, int32_t* buf, int* cnt) {
  const unsigned long long m = __ballot(pred);
  if (m == 0ull) return;
  const int leader = __ffsll((long long)m) - 1;
  int base = 0;
  if ((int)PLC_LANE == leader) base = atomicAdd(cnt, __popcll(m));
  base = __shfl(base, leader);
  if (pred) buf[base + __popcll(m & lanemask_lt())] = v;
}

// Workgroup-aggregated append of the values staged in an LDS buffer:
// one global atomic per call.  Every thread must call it.  Writes
// dst[base + j] = buf[j] for j < *count (slots >= cap raise *fault).
__device__ __forceinline__ void block_flush(int32_t* counter, int32_t* dst, int64_t cap,
                                            const int32_t* buf, int* count, int* s_base,
                                            int* fault) {
  __syncthreads();
  int cnt = *count;
  if (threadIdx.x == 0) *s_base = cnt > 0 ? atomicAdd(counter, cnt) : 0;
  __syncthreads();
  long long base = *s_base;
  for (int j = threadIdx.x; j < cnt; j += blockDim.x) {
    long long slot = base + j;
    if (slot < cap) dst[slot] = buf[j]; else *fault = 1;
  }
  __syncthreads();
  if (threadIdx.x == 0) *count = 0;
  __syncthreads();
}

// The dispatcher hands workgroups to the 8 XCDs round-robin (XCD =
// blockIdx % 8), and each XCD has its own L2.  xcd_block renumbers the
// workgroups of a grid of G so that those of one XCD get consecutive numbers
// (a bijection on [0, G)).  A kernel that gives contiguous work ranges by
// this number keeps neighbouring work -- in the batched kernels, the edges of
// one slot, whose state lines they share -- inside one L2.
__device__ __forceinline__ int xcd_block(int b, int G) {
  const int q = G >> 3, r = G & 7, x = b & 7, i = b >> 3;
  return x * q + (x < r ? x : r) + i;
}

// a/b < c/d exactly, for b, d > 0.
__device__ __forceinline__ bool ratio_lt(long long a, long long b, long long c, long long d) {
  return (__int128)a * (__int128)d < (__int128)c * (__int128)b;
}

}  // namespace plc
