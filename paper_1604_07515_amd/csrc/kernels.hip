// kernels.hip -- gfx950 kernels of the plain (one query at a time) path:
// round-synchronous PR-Nibble (Sec. 3.3) and the parallel sweep cut
// (Sec. 3.1, Theorem 1).
//
// Round t of PR-Nibble is two launches:
//   k_self    vertexMap(Frontier, UpdateSelf): snapshot rho_v = r[v], update
//             p[v] and r[v], compute the per-entry coefficient cn*rho/d(v), and
//             (single-pass decoupled look-back scan) the start of each entry's
//             edges in the round's flattened edge sequence; entries write the
//             first-entry index of every 1024-edge tile they overlap.
//   k_scatter edgeMap(G, Frontier, UpdateNgh): one workgroup per edge tile
//             (persistent grid), entries staged in LDS, coalesced neighbour
//             reads, FP64 atomic add into r[w].  The filter of the paper is
//             folded in: r only grows during a scatter, so w joins the next
//             frontier exactly when one atomic's (old, old + c) pair straddles
//             eps*d(w); that atomic appends w with a wave-aggregated counter.
// Kernels read the round number and frontier size from the device control
// block and return at once when the query has finished, so rounds can be
// queued ahead of the host's termination check.
//
// Arithmetic matches the paper's updates evaluated in a fixed way: the
// constants cs, cn, keep are rounded once, p[v] + cs*rho, keep*rho and
// (cn*rho)/d are each rounded separately (the library is built with
// -ffp-contract=off), and the threshold is eps*(double)d.  Only the order of
// the atomic additions into r differs from a sequential evaluation.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "plc_device.h"

namespace plc {

#define LANE (threadIdx.x & 63)
#define WID (threadIdx.x >> 6)

__device__ __forceinline__ unsigned long long lanemask_lt() {
  unsigned l = LANE;
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// Wave-aggregated append: every lane of the wave must call it.  Returns the
// slot for lanes with pred, -1 otherwise.  One atomic per wave.
__device__ __forceinline__ long long wave_append(int32_t* counter, bool pred) {
  unsigned long long m = __ballot(pred);
  if (m == 0) return -1;
  int leader = __ffsll((long long)m) - 1;
  int base = 0;
  if ((int)LANE == leader) base = atomicAdd(counter, (int)__popcll(m));
  base = __shfl(base, leader);
  return pred ? (long long)base + __popcll(m & lanemask_lt()) : -1;
}

__device__ __forceinline__ long long wave_incl_scan(long long x) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    long long y = __shfl_up(x, o);
    if ((int)LANE >= o) x += y;
  }
  return x;
}

// Exclusive block scan over kBlock threads; sh needs kBlock/64 + 1 slots.
__device__ __forceinline__ long long block_excl_scan(long long x, long long* total,
                                                     long long* sh) {
  constexpr int NW = kBlock / 64;
  long long inc = wave_incl_scan(x);
  if (LANE == 63) sh[WID] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long s = 0;
    for (int w = 0; w < NW; w++) { long long t = sh[w]; sh[w] = s; s += t; }
    sh[NW] = s;
  }
  __syncthreads();
  long long ex = inc - x + sh[WID];
  *total = sh[NW];
  __syncthreads();
  return ex;
}

__device__ __forceinline__ long long block_sum(long long x, long long* sh) {
  long long tot;
  (void)block_excl_scan(x, &tot, sh);
  return tot;
}

__device__ __forceinline__ unsigned long long ld_acq_tag(unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_tag(unsigned long long* p, unsigned long long v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ long long ld_ll(long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_ll(long long* p, long long v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

constexpr long kSpinLimit = 1L << 24;

// Decoupled look-back for block b (thread 0 only).  Publishes the block's
// aggregate, walks back over predecessors (which claimed their tickets
// earlier and so are running or done) and publishes the inclusive prefix.
// Returns the exclusive prefix.  The spin is bounded; on exhaustion the
// fault flag is raised and the partial prefix returned.
__device__ long long lookback(ScanDesc* desc, int b, long long agg, unsigned long long epoch,
                              int32_t* fault) {
  ScanDesc* me = desc + b;
  if (b == 0) {
    st_ll(&me->incl, agg);
    __threadfence();
    st_tag(&me->tag, (epoch << 2) | 2ull);
    return 0;
  }
  st_ll(&me->agg, agg);
  __threadfence();
  st_tag(&me->tag, (epoch << 2) | 1ull);
  long long excl = 0;
  int j = b - 1;
  long spins = 0;
  while (j >= 0) {
    unsigned long long t = ld_acq_tag(&desc[j].tag);
    unsigned flag = (unsigned)(t & 3ull);
    if ((t >> 2) != epoch || flag == 0) {
      if (++spins > kSpinLimit) { atomicExch(fault, 1); break; }
      __builtin_amdgcn_s_sleep(1);
      continue;
    }
    __threadfence();
    if (flag == 2) { excl += ld_ll(&desc[j].incl); break; }
    excl += ld_ll(&desc[j].agg);
    --j;
  }
  st_ll(&me->incl, excl + agg);
  __threadfence();
  st_tag(&me->tag, (epoch << 2) | 2ull);
  return excl;
}

// Ticket dispenser for single-pass scans: returns the next block index, or
// a value >= nblk when the work is exhausted.  The workgroup that draws the
// very last ticket (nblk + gridDim.x - 1) resets the dispenser and advances
// the epoch, so the next launch starts clean.
__device__ __forceinline__ int next_ticket(Ctl* c, int site, int nblk, int* sh) {
  if (threadIdx.x == 0) {
    unsigned t = atomicAdd(&c->ticket[site], 1u);
    if (t == (unsigned)nblk + gridDim.x - 1) {
      c->ticket[site] = 0;
      c->epoch[site] = c->epoch[site] + 1;
    }
    *sh = (int)t;
  }
  __syncthreads();
  int b = *sh;
  __syncthreads();
  return b;
}

// Last-workgroup detection: true in exactly one workgroup, after every other
// workgroup of the launch has called it.  Resets the counter.
__device__ __forceinline__ bool last_block(unsigned* done, int* sh) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    unsigned prev = atomicAdd(done, 1u);
    int last = prev == gridDim.x - 1;
    if (last) { __threadfence(); *done = 0; }
    *sh = last;
  }
  __syncthreads();
  int l = *sh;
  __syncthreads();
  return l != 0;
}

// ---------------------------------------------------------------- init

__global__ void k_graph_init(PlainArgs a) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < a.n;
       v += (int64_t)gridDim.x * blockDim.x) {
    VRec rec;
    rec.r = 0.0;
    rec.deg = (int32_t)(a.off[v + 1] - a.off[v]);
    rec.rank = 0;
    a.vr[v] = rec;
    a.p[v] = 0.0;
  }
}

// Seed initialisation (Fig. alg:pr-nibble: r = {(x,1)}, Frontier = {x}).
__global__ void k_query_init(PlainArgs a, int32_t seed, int32_t rule, double alpha, double eps,
                             int32_t max_rounds) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  Ctl* c = a.ctl;
  if (rule == 1) {  // original rule
    c->cs = alpha;
    c->cn = (1.0 - alpha) / 2.0;
    c->keep = (1.0 - alpha) / 2.0;
    c->opt_rule = 0;
  } else {          // optimized rule
    c->cs = 2.0 * alpha / (1.0 + alpha);
    c->cn = (1.0 - alpha) / (1.0 + alpha);
    c->keep = 0.0;
    c->opt_rule = 1;
  }
  c->eps = eps;
  c->seed = seed;
  c->rule = rule;
  c->max_rounds = max_rounds;
  c->round = 0;
  c->cnt[0] = 1;
  c->cnt[1] = 0;
  c->cnt[2] = 0;
  c->ntiles = 0;
  c->etotal = 0;
  c->pushes = 0;
  c->edges = 0;
  c->support_cnt = 0;
  c->touched_cnt = 1;
  c->overflow = 0;
  c->limited = 0;
  c->N = 0;
  c->sort_flip = 0;
  c->pass_trivial = 0;
  c->rnnz = 0;
  c->vol_total = a.vol_total;
  c->best_cut = 0;
  c->best_vol = 0;
  c->best_den = 0;
  c->kstar = 0;
  c->phi = 0.0;
  a.fbuf0[0] = seed;
  a.touched[0] = seed;
  a.vr[seed].r = 1.0;
  __threadfence();
  c->status = ST_PUSH;
}

// ---------------------------------------------------------------- round

__device__ __forceinline__ bool push_active(const Ctl* c, int64_t a_n_cap, int* t_out, int* nf_out) {
  if (c->status != ST_PUSH) return false;
  int t = c->round;
  int nf = c->cnt[t & 1];
  if (nf <= 0) return false;
  if ((int64_t)nf > a_n_cap) nf = (int)a_n_cap;
  *t_out = t;
  *nf_out = nf;
  return true;
}

// vertexMap(Frontier, UpdateSelf) + degree scan of the frontier.
__global__ __launch_bounds__(kBlock) void k_self(PlainArgs a) {
  Ctl* c = a.ctl;
  int t, nf;
  if (!push_active(c, a.n, &t, &nf)) return;
  if (t >= c->max_rounds) {
    if (blockIdx.x == 0 && threadIdx.x == 0) { c->limited = 1; c->status = ST_LIMIT; }
    return;
  }
  __shared__ long long sh[kBlock / 64 + 1];
  __shared__ long long s_excl;
  __shared__ int s_tk;
  const int32_t* F = (t & 1) ? a.fbuf1 : a.fbuf0;
  int32_t* Fn = (t & 1) ? a.fbuf0 : a.fbuf1;
  int32_t* cntn = &c->cnt[(t + 1) & 1];
  const double cs = c->cs, cn = c->cn, keep = c->keep, eps = c->eps;
  const bool opt = c->opt_rule != 0;
  const unsigned long long epoch = c->epoch[SCAN_FRONTIER];
  const int nblk = (nf + kScanBlock - 1) / kScanBlock;
  const int64_t ncap = a.n;

  for (;;) {
    int b = next_ticket(c, SCAN_FRONTIER, nblk, &s_tk);
    if (b >= nblk) break;
    int32_t dk[kScanItems];
    long long dsum = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; k++) {
      int i = b * kScanBlock + k * kBlock + (int)threadIdx.x;
      bool valid = i < nf;
      bool first_push = false, stay = false;
      int32_t v = 0;
      int32_t d = 0;
      if (valid) {
        v = F[i];
        VRec rec = a.vr[v];
        double rho = rec.r;
        d = rec.deg;
        double pold = a.p[v];
        a.p[v] = pold + cs * rho;
        double nr = opt ? -0.0 : keep * rho;
        a.vr[v].r = nr;
        a.coef[i] = (cn * rho) / (double)d;
        a.rowp[i] = a.off[v];
        first_push = (pold == 0.0);
        stay = !opt && (nr >= eps * (double)d);
      }
      dk[k] = d;
      dsum += d;
      long long slot = wave_append(&c->support_cnt, first_push);
      if (first_push) {
        if (slot < ncap) a.support[slot] = v; else c->overflow = 1;
      }
      slot = wave_append(cntn, stay);
      if (stay) {
        if (slot < ncap) Fn[slot] = v; else c->overflow = 1;
      }
    }
    long long agg = block_sum(dsum, sh);
    if (threadIdx.x == 0) s_excl = lookback(a.desc[SCAN_FRONTIER], b, agg, epoch, &c->overflow);
    __syncthreads();
    long long base = s_excl;
    // per-slice exclusive scans give each entry its global edge start
    for (int k = 0; k < kScanItems; k++) {
      int i = b * kScanBlock + k * kBlock + (int)threadIdx.x;
      long long tot;
      long long ex = block_excl_scan(dk[k], &tot, sh);
      if (i < nf) {
        long long s = base + ex;
        a.estart[i] = s;
        long long d = dk[k];
        long long t0 = (s + kEdgeTile - 1) / kEdgeTile;
        long long t1 = (s + d - 1) / kEdgeTile;
        if (t1 >= a.tile_cap) { c->overflow = 1; t1 = a.tile_cap - 1; }
        for (long long tt = t0; tt <= t1; tt++) a.tile_start[tt] = i;
      }
      base += tot;
    }
    if (b == nblk - 1 && threadIdx.x == 0) {
      c->etotal = base;
      c->ntiles = (int)((base + kEdgeTile - 1) / kEdgeTile);
    }
    __syncthreads();
  }
}

// edgeMap(G, Frontier, UpdateNgh) with the filter folded in.
__global__ __launch_bounds__(kBlock) void k_scatter(PlainArgs a) {
  Ctl* c = a.ctl;
  int t, nf;
  if (!push_active(c, a.n, &t, &nf)) return;
  if (t >= c->max_rounds) return;
  __shared__ int32_t s_start[kEdgeTile + 1];
  __shared__ int64_t s_row[kEdgeTile + 1];
  __shared__ double s_coef[kEdgeTile + 1];
  __shared__ int s_last;
  const int ntiles = (int64_t)c->ntiles > a.tile_cap ? (int)a.tile_cap : c->ntiles;
  const long long E = c->etotal;
  const double eps = c->eps;
  int32_t* Fn = (t & 1) ? a.fbuf0 : a.fbuf1;
  int32_t* cntn = &c->cnt[(t + 1) & 1];
  const int64_t ncap = a.n;

  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    long long e0 = (long long)tile * kEdgeTile;
    long long e1 = e0 + kEdgeTile < E ? e0 + kEdgeTile : E;
    int i0 = a.tile_start[tile];
    int i1 = tile + 1 < ntiles ? a.tile_start[tile + 1] : nf - 1;
    if (i0 < 0 || i1 < i0 || i1 >= nf || i1 - i0 + 1 > kEdgeTile + 1) {
      c->overflow = 1;  // inconsistent tile map: skip the tile, report a fault
      continue;
    }
    int cnt = i1 - i0 + 1;
    for (int j = threadIdx.x; j < cnt; j += kBlock) {
      s_start[j] = (int32_t)(a.estart[i0 + j] - e0);
      s_row[j] = a.rowp[i0 + j];
      s_coef[j] = a.coef[i0 + j];
    }
    __syncthreads();
    for (int k = 0; k < kEdgeTile / kBlock; k++) {
      int rel = k * kBlock + (int)threadIdx.x;
      bool valid = e0 + rel < e1;
      bool cross = false, first = false;
      int32_t w = 0;
      if (valid) {
        int lo = 0, hi = cnt - 1;
        while (lo < hi) {
          int mid = (lo + hi + 1) >> 1;
          if (s_start[mid] <= rel) lo = mid; else hi = mid - 1;
        }
        w = a.nbr[s_row[lo] + (rel - s_start[lo])];
        double cf = s_coef[lo];
        int32_t dw = a.vr[w].deg;
        double old = unsafeAtomicAdd(&a.vr[w].r, cf);
        double thr = eps * (double)dw;
        cross = (old < thr) && (old + cf >= thr);
        first = __double_as_longlong(old) == 0;
      }
      long long slot = wave_append(cntn, cross);
      if (cross) {
        if (slot < ncap) Fn[slot] = w; else c->overflow = 1;
      }
      slot = wave_append(&c->touched_cnt, first);
      if (first) {
        if (slot < ncap) a.touched[slot] = w; else c->overflow = 1;
      }
    }
    __syncthreads();
  }
  if (last_block(&c->done[0], &s_last)) {
    if (threadIdx.x == 0) {
      c->pushes += nf;
      c->edges += E;
      c->cnt[t & 1] = 0;
      c->round = t + 1;
      __threadfence();
    }
  }
}

// ---------------------------------------------------------------- sweep

// The sweep may start once the frontier is empty (or the watchdog fired).
__device__ __forceinline__ bool sweep_ready(const Ctl* c) {
  if (c->status == ST_LIMIT) return true;
  return c->status == ST_PUSH && c->cnt[c->round & 1] == 0;
}

// Sort keys: non-increasing p/d is ascending order of the bit-inverted IEEE
// pattern of the positive ratio; ties fall to the id passes (ascending id).
__global__ __launch_bounds__(kBlock) void k_sweep_keys(PlainArgs a) {
  Ctl* c = a.ctl;
  if (!sweep_ready(c)) return;
  __shared__ int s_last;
  const int N = (int64_t)c->support_cnt > a.n ? (int)a.n : c->support_cnt;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < N; i += gridDim.x * kBlock) {
    int32_t v = a.support[i];
    double ratio = a.p[v] / (double)a.vr[v].deg;
    a.keyA[i] = ~(unsigned long long)__double_as_longlong(ratio);
    a.idA[i] = v;
  }
  if (last_block(&c->done[1], &s_last)) {
    if (threadIdx.x == 0) {
      c->N = N;
      c->sort_flip = 0;
      c->status = ST_SWEEPING;
    }
  }
}

__device__ __forceinline__ unsigned digit_of(unsigned long long key, int32_t id, int is_id,
                                             int shift) {
  return is_id ? (((unsigned)id >> shift) & 255u) : (unsigned)((key >> shift) & 255ull);
}

__global__ __launch_bounds__(kBlock) void k_radix_hist(PlainArgs a, int is_id, int shift) {
  Ctl* c = a.ctl;
  if (c->status != ST_SWEEPING) return;
  const int N = c->N;
  const int ntl = (N + kSortTile - 1) / kSortTile;
  const unsigned long long* key = c->sort_flip ? a.keyB : a.keyA;
  const int32_t* id = c->sort_flip ? a.idB : a.idA;
  __shared__ unsigned s_h[256];
  for (int tile = blockIdx.x; tile < ntl; tile += gridDim.x) {
    s_h[threadIdx.x] = 0;
    __syncthreads();
    for (int k = 0; k < kSortItems; k++) {
      int i = tile * kSortTile + k * kBlock + (int)threadIdx.x;
      if (i < N) atomicAdd(&s_h[digit_of(key[i], id[i], is_id, shift)], 1u);
    }
    __syncthreads();
    a.hist[(size_t)threadIdx.x * ntl + tile] = s_h[threadIdx.x];
    __syncthreads();
  }
}

// One workgroup: exclusive scan of the digit-major histogram.
__global__ __launch_bounds__(1024) void k_radix_scan(PlainArgs a) {
  Ctl* c = a.ctl;
  if (c->status != ST_SWEEPING) return;
  const int N = c->N;
  const int ntl = (N + kSortTile - 1) / kSortTile;
  const long long total = 256ll * ntl;
  const long long per = (total + 1023) / 1024;
  const long long lo = threadIdx.x * per;
  const long long hi = lo + per < total ? lo + per : total;
  __shared__ long long s_part[1024];
  __shared__ int s_triv;
  long long sum = 0;
  for (long long j = lo; j < hi; j++) sum += a.hist[j];
  s_part[threadIdx.x] = sum;
  if (threadIdx.x == 0) s_triv = 0;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long s = 0;
    for (int w = 0; w < 1024; w++) { long long x = s_part[w]; s_part[w] = s; s += x; }
  }
  __syncthreads();
  long long run = s_part[threadIdx.x];
  for (long long j = lo; j < hi; j++) {
    unsigned x = a.hist[j];
    a.hist[j] = (unsigned)run;
    run += x;
  }
  __syncthreads();
  if (threadIdx.x < 256) {
    long long b0 = a.hist[(size_t)threadIdx.x * ntl];
    long long b1 = threadIdx.x < 255 ? (long long)a.hist[(size_t)(threadIdx.x + 1) * ntl] : N;
    if (b1 - b0 == N) s_triv = 1;
  }
  __syncthreads();
  if (threadIdx.x == 0) c->pass_trivial = s_triv;
}

// Stable scatter of one radix pass (tile order, then element order within a
// tile, is preserved for equal digits).
__global__ __launch_bounds__(kBlock) void k_radix_scatter(PlainArgs a, int is_id, int shift) {
  Ctl* c = a.ctl;
  if (c->status != ST_SWEEPING || c->pass_trivial) return;
  const int N = c->N;
  const int ntl = (N + kSortTile - 1) / kSortTile;
  const int flip = c->sort_flip;
  const unsigned long long* ks = flip ? a.keyB : a.keyA;
  const int32_t* is = flip ? a.idB : a.idA;
  unsigned long long* kd = flip ? a.keyA : a.keyB;
  int32_t* id_dst = flip ? a.idA : a.idB;
  constexpr int NW = kBlock / 64;
  __shared__ unsigned s_run[256];
  __shared__ unsigned s_wc[NW][256];
  __shared__ int s_last;
  for (int tile = blockIdx.x; tile < ntl; tile += gridDim.x) {
    s_run[threadIdx.x] = 0;
    for (int k = 0; k < kSortItems; k++) {
      for (int w = 0; w < NW; w++) s_wc[w][threadIdx.x] = 0;
      __syncthreads();
      int i = tile * kSortTile + k * kBlock + (int)threadIdx.x;
      bool valid = i < N;
      unsigned long long key = valid ? ks[i] : 0ull;
      int32_t idv = valid ? is[i] : 0;
      unsigned dg = valid ? digit_of(key, idv, is_id, shift) : 256u;
      // lanes of this wave with the same digit
      unsigned long long peers = __ballot(valid);
#pragma unroll
      for (int bit = 0; bit < 8; bit++) {
        unsigned long long bm = __ballot((dg >> bit) & 1u);
        peers &= ((dg >> bit) & 1u) ? bm : ~bm;
      }
      unsigned rank_w = (unsigned)__popcll(peers & lanemask_lt());
      if (valid && rank_w == 0) s_wc[WID][dg] = (unsigned)__popcll(peers);
      __syncthreads();
      if (valid) {
        unsigned before = s_run[dg];
        for (int w = 0; w < (int)WID; w++) before += s_wc[w][dg];
        long long dst = (long long)a.hist[(size_t)dg * ntl + tile] + before + rank_w;
        if (dst >= 0 && dst < N) {
          kd[dst] = key;
          id_dst[dst] = idv;
        } else {
          c->overflow = 1;
        }
      }
      __syncthreads();
      {
        unsigned add = 0;
        for (int w = 0; w < NW; w++) add += s_wc[w][threadIdx.x];
        s_run[threadIdx.x] += add;
      }
      __syncthreads();
    }
  }
  if (last_block(&c->done[2], &s_last)) {
    if (threadIdx.x == 0) c->sort_flip = flip ^ 1;
  }
}

// Rank map (rank[v_k] = k, outside = 0) and per-position degree and p.
__global__ __launch_bounds__(kBlock) void k_sweep_rank(PlainArgs a) {
  Ctl* c = a.ctl;
  if (c->status != ST_SWEEPING) return;
  const int N = c->N;
  const int32_t* ids = c->sort_flip ? a.idB : a.idA;
  for (int k = blockIdx.x * kBlock + threadIdx.x; k < N; k += gridDim.x * kBlock) {
    int32_t v = ids[k];
    a.vr[v].rank = k + 1;
    a.sdeg[k] = a.vr[v].deg;
    a.sp[k] = a.p[v];
    a.scnt[k] = 0;
  }
}

// Inclusive volume prefix vol(S_k) and edge-tile starts over the support's
// edges in sweep order (the offsets of the Z array in Theorem 1's proof).
__global__ __launch_bounds__(kBlock) void k_vol_scan(PlainArgs a) {
  Ctl* c = a.ctl;
  if (c->status != ST_SWEEPING) return;
  const int N = c->N;
  if (N <= 0) return;
  __shared__ long long sh[kBlock / 64 + 1];
  __shared__ long long s_excl;
  __shared__ int s_tk;
  const unsigned long long epoch = c->epoch[SCAN_VOL];
  const int nblk = (N + kScanBlock - 1) / kScanBlock;
  for (;;) {
    int b = next_ticket(c, SCAN_VOL, nblk, &s_tk);
    if (b >= nblk) break;
    int32_t dk[kScanItems];
    long long dsum = 0;
    for (int k = 0; k < kScanItems; k++) {
      int i = b * kScanBlock + k * kBlock + (int)threadIdx.x;
      dk[k] = i < N ? a.sdeg[i] : 0;
      dsum += dk[k];
    }
    long long agg = block_sum(dsum, sh);
    if (threadIdx.x == 0) s_excl = lookback(a.desc[SCAN_VOL], b, agg, epoch, &c->overflow);
    __syncthreads();
    long long base = s_excl;
    for (int k = 0; k < kScanItems; k++) {
      int i = b * kScanBlock + k * kBlock + (int)threadIdx.x;
      long long tot;
      long long ex = block_excl_scan(dk[k], &tot, sh);
      if (i < N) {
        long long s = base + ex;
        long long d = dk[k];
        a.svol[i] = s + d;
        long long t0 = (s + kEdgeTile - 1) / kEdgeTile;
        long long t1 = (s + d - 1) / kEdgeTile;
        if (t1 >= a.tile_cap) { c->overflow = 1; t1 = a.tile_cap - 1; }
        for (long long tt = t0; tt <= t1; tt++) a.tile_start[tt] = i;
      }
      base += tot;
    }
    if (b == nblk - 1 && threadIdx.x == 0) {
      c->etotal = base;
      c->ntiles = (int)((base + kEdgeTile - 1) / kEdgeTile);
    }
    __syncthreads();
  }
}

// For every support edge (v_k, w): count w with 1 <= rank[w] < k.  Then
// delta_k = d(v_k) - 2 * count_k is the change of the boundary when v_k joins
// S_{k-1}; it equals the sum of Z's first values at rank k (Theorem 1).
__global__ __launch_bounds__(kBlock) void k_cut_count(PlainArgs a) {
  Ctl* c = a.ctl;
  if (c->status != ST_SWEEPING) return;
  const int N = c->N;
  if (N <= 0) return;
  __shared__ int32_t s_start[kEdgeTile + 1];
  __shared__ int64_t s_row[kEdgeTile + 1];
  __shared__ int32_t s_cnt[kEdgeTile + 1];
  const int ntiles = (int64_t)c->ntiles > a.tile_cap ? (int)a.tile_cap : c->ntiles;
  const long long E = c->etotal;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    long long e0 = (long long)tile * kEdgeTile;
    long long e1 = e0 + kEdgeTile < E ? e0 + kEdgeTile : E;
    int i0 = a.tile_start[tile];
    int i1 = tile + 1 < ntiles ? a.tile_start[tile + 1] : N - 1;
    if (i0 < 0 || i1 < i0 || i1 >= N || i1 - i0 + 1 > kEdgeTile + 1) {
      c->overflow = 1;
      continue;
    }
    int cnt = i1 - i0 + 1;
    for (int j = threadIdx.x; j < cnt; j += kBlock) {
      int k = i0 + j;
      s_start[j] = (int32_t)(a.svol[k] - a.sdeg[k] - e0);
      s_row[j] = a.off[(c->sort_flip ? a.idB : a.idA)[k]];
      s_cnt[j] = 0;
    }
    __syncthreads();
    for (int kk = 0; kk < kEdgeTile / kBlock; kk++) {
      int rel = kk * kBlock + (int)threadIdx.x;
      if (e0 + rel < e1) {
        int lo = 0, hi = cnt - 1;
        while (lo < hi) {
          int mid = (lo + hi + 1) >> 1;
          if (s_start[mid] <= rel) lo = mid; else hi = mid - 1;
        }
        int32_t w = a.nbr[s_row[lo] + (rel - s_start[lo])];
        int32_t rw = a.vr[w].rank;
        int own = i0 + lo + 1;
        if (rw != 0 && rw < own) atomicAdd(&s_cnt[lo], 1);
      }
    }
    __syncthreads();
    for (int j = threadIdx.x; j < cnt; j += kBlock)
      if (s_cnt[j] != 0) atomicAdd(&a.scnt[i0 + j], s_cnt[j]);
    __syncthreads();
  }
}

// a/b < c/d exactly (b, d > 0).
__device__ __forceinline__ bool ratio_lt(long long a, long long b, long long cc, long long d) {
  return (__int128)a * (__int128)d < (__int128)cc * (__int128)b;
}

// Inclusive prefix of the boundary deltas gives |boundary(S_k)|; with vol_k
// the conductance of every prefix follows, and a min-reduction (first k on
// exact ties, den = 0 excluded) picks the cluster (Sec. 3.1, Theorem 1).
__global__ __launch_bounds__(kBlock) void k_cut_scan(PlainArgs a) {
  Ctl* c = a.ctl;
  if (c->status != ST_SWEEPING) return;
  const int N = c->N;
  if (N <= 0) return;
  __shared__ long long sh[kBlock / 64 + 1];
  __shared__ long long s_excl;
  __shared__ int s_tk;
  __shared__ long long s_bc[kBlock], s_bd[kBlock], s_bk[kBlock];
  const unsigned long long epoch = c->epoch[SCAN_CUT];
  const int nblk = (N + kScanBlock - 1) / kScanBlock;
  const long long vt = c->vol_total;
  for (;;) {
    // Only a block's last ticket-holder may finish the launch; remember the
    // block count before next_ticket can reset the dispenser.
    int b = 0;
    if (threadIdx.x == 0) {
      unsigned tk = atomicAdd(&c->ticket[SCAN_CUT], 1u);
      s_tk = (int)tk;
    }
    __syncthreads();
    b = s_tk;
    __syncthreads();
    if (b >= nblk) {
      if (b == nblk + (int)gridDim.x - 1 && threadIdx.x == 0) {
        // every block has published its candidate: final reduction
        __threadfence();
        long long bc = -1, bd = 1, bk = 0;
        for (int j = 0; j < nblk; j++) {
          long long jc = a.bbest[3 * j], jd = a.bbest[3 * j + 1], jk = a.bbest[3 * j + 2];
          if (jk <= 0) continue;
          if (bc < 0 || ratio_lt(jc, jd, bc, bd)) { bc = jc; bd = jd; bk = jk; }
        }
        c->kstar = bc < 0 ? 0 : bk;
        c->best_cut = bc < 0 ? 0 : bc;
        c->best_den = bc < 0 ? 0 : bd;
        c->best_vol = bk > 0 ? a.svol[bk - 1] : 0;
        c->phi = bc < 0 ? 0.0 : (double)bc / (double)bd;
        c->ticket[SCAN_CUT] = 0;
        c->epoch[SCAN_CUT] = c->epoch[SCAN_CUT] + 1;
      }
      break;
    }
    long long dk[kScanItems];
    long long dsum = 0;
    for (int k = 0; k < kScanItems; k++) {
      int i = b * kScanBlock + k * kBlock + (int)threadIdx.x;
      dk[k] = i < N ? (long long)a.sdeg[i] - 2ll * a.scnt[i] : 0;
      dsum += dk[k];
    }
    long long agg = block_sum(dsum, sh);
    if (threadIdx.x == 0) s_excl = lookback(a.desc[SCAN_CUT], b, agg, epoch, &c->overflow);
    __syncthreads();
    long long base = s_excl;
    long long mc = -1, md = 1, mk = 0;
    for (int k = 0; k < kScanItems; k++) {
      int i = b * kScanBlock + k * kBlock + (int)threadIdx.x;
      long long tot;
      long long ex = block_excl_scan(dk[k], &tot, sh);
      if (i < N) {
        long long cut = base + ex + dk[k];
        long long vol = a.svol[i];
        long long den = vol < vt - vol ? vol : vt - vol;
        if (den > 0 && (mc < 0 || ratio_lt(cut, den, mc, md))) { mc = cut; md = den; mk = i + 1; }
      }
      base += tot;
    }
    // block argmin: smaller ratio, then smaller k
    s_bc[threadIdx.x] = mc; s_bd[threadIdx.x] = md; s_bk[threadIdx.x] = mk;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o) {
        long long oc = s_bc[threadIdx.x + o], od = s_bd[threadIdx.x + o], ok = s_bk[threadIdx.x + o];
        long long xc = s_bc[threadIdx.x], xd = s_bd[threadIdx.x], xk = s_bk[threadIdx.x];
        bool take = false;
        if (ok > 0) {
          if (xk <= 0) take = true;
          else if (ratio_lt(oc, od, xc, xd)) take = true;
          else if (!ratio_lt(xc, xd, oc, od) && ok < xk) take = true;
        }
        if (take) { s_bc[threadIdx.x] = oc; s_bd[threadIdx.x] = od; s_bk[threadIdx.x] = ok; }
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      a.bbest[3 * b] = s_bc[0];
      a.bbest[3 * b + 1] = s_bd[0];
      a.bbest[3 * b + 2] = s_bk[0];
      __threadfence();
    }
    __syncthreads();
  }
}

// Gather the nonzeros of r over the touched list; mark the sweep finished.
__global__ __launch_bounds__(kBlock) void k_sweep_finish(PlainArgs a) {
  Ctl* c = a.ctl;
  if (c->status != ST_SWEEPING) return;
  __shared__ int s_last;
  const int T = (int64_t)c->touched_cnt > a.n ? (int)a.n : c->touched_cnt;
  const int64_t ncap = a.n;
  for (int base = blockIdx.x * kBlock; base < T; base += gridDim.x * kBlock) {
    int i = base + (int)threadIdx.x;
    bool nz = false;
    int32_t v = 0;
    double rv = 0.0;
    if (i < T) {
      v = a.touched[i];
      rv = a.vr[v].r;
      nz = rv != 0.0;
    }
    long long slot = wave_append(&c->rnnz, nz);
    if (nz) {
      if (slot < ncap) { a.rid[slot] = v; a.rval[slot] = rv; } else c->overflow = 1;
    }
  }
  if (last_block(&c->done[3], &s_last)) {
    if (threadIdx.x == 0) { c->status = ST_SWEPT; __threadfence(); }
  }
}

// Reset the dense per-vertex state of every touched vertex.
__global__ __launch_bounds__(kBlock) void k_cleanup(PlainArgs a) {
  Ctl* c = a.ctl;
  const int T = (int64_t)c->touched_cnt > a.n ? (int)a.n : c->touched_cnt;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < T; i += gridDim.x * kBlock) {
    int32_t v = a.touched[i];
    a.vr[v].r = 0.0;
    a.vr[v].rank = 0;
    a.p[v] = 0.0;
  }
}

// ---------------------------------------------------------------- launchers

hipError_t launch_graph_init(hipStream_t s, const PlainArgs& a) {
  int grid = (int)((a.n + kBlock - 1) / kBlock);
  if (grid > 4096) grid = 4096;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(k_graph_init, dim3(grid), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_query_init(hipStream_t s, const PlainArgs& a, int32_t seed, int32_t rule,
                             double alpha, double eps, int32_t max_rounds) {
  hipLaunchKernelGGL(k_query_init, dim3(1), dim3(64), 0, s, a, seed, rule, alpha, eps,
                     max_rounds);
  return hipGetLastError();
}

hipError_t launch_self(hipStream_t s, const PlainArgs& a, int grid) {
  hipLaunchKernelGGL(k_self, dim3(grid), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_scatter(hipStream_t s, const PlainArgs& a, int grid) {
  hipLaunchKernelGGL(k_scatter, dim3(grid), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_sweep(hipStream_t s, const PlainArgs& a, int grid) {
  hipLaunchKernelGGL(k_sweep_keys, dim3(grid), dim3(kBlock), 0, s, a);
  // LSD radix: id digits first (ties in p/d resolve to ascending id), then
  // the 64-bit key; passes whose digit is constant are skipped on device.
  for (int shift = 0; shift < a.id_bits; shift += 8) {
    hipLaunchKernelGGL(k_radix_hist, dim3(grid), dim3(kBlock), 0, s, a, 1, shift);
    hipLaunchKernelGGL(k_radix_scan, dim3(1), dim3(1024), 0, s, a);
    hipLaunchKernelGGL(k_radix_scatter, dim3(grid), dim3(kBlock), 0, s, a, 1, shift);
  }
  for (int shift = 0; shift < 64; shift += 8) {
    hipLaunchKernelGGL(k_radix_hist, dim3(grid), dim3(kBlock), 0, s, a, 0, shift);
    hipLaunchKernelGGL(k_radix_scan, dim3(1), dim3(1024), 0, s, a);
    hipLaunchKernelGGL(k_radix_scatter, dim3(grid), dim3(kBlock), 0, s, a, 0, shift);
  }
  hipLaunchKernelGGL(k_sweep_rank, dim3(grid), dim3(kBlock), 0, s, a);
  hipLaunchKernelGGL(k_vol_scan, dim3(grid), dim3(kBlock), 0, s, a);
  hipLaunchKernelGGL(k_cut_count, dim3(grid), dim3(kBlock), 0, s, a);
  hipLaunchKernelGGL(k_cut_scan, dim3(grid), dim3(kBlock), 0, s, a);
  hipLaunchKernelGGL(k_sweep_finish, dim3(grid), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_cleanup(hipStream_t s, const PlainArgs& a, int grid) {
  hipLaunchKernelGGL(k_cleanup, dim3(grid), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

}  // namespace plc
