// batch.hip -- gfx950 kernels of the batched path: the same round-synchronous
// PR-Nibble round (Sec. 3.3) and sweep cut (Sec. 3.1, Theorem 1) as the plain
// path, applied to many queries in the same launches.
//
// A global step runs one round for every scheduled slot:
//   k_b_plan      (one workgroup) picks the slots whose frontier is non-empty,
//                 within the round-buffer capacity, and lays their frontiers
//                 end to end (entry prefix per slot).
//   k_b_self      vertexMap(UpdateSelf) on every scheduled entry + single-pass
//                 scan of degrees over the concatenated frontiers.
//   k_b_scatter   edgeMap(UpdateNgh) over all scheduled edges in 1024-edge
//                 tiles; threshold crossings append to the owning slot's next
//                 frontier.  Entries of a tile are slot-sorted, so appends are
//                 counted per slot in LDS and reserved with one global atomic
//                 per slot and tile.
//   k_b_round_end (one workgroup) per-slot bookkeeping and frontier swap.
// Queries whose frontier emptied are swept together: their supports form
// the segments of one merge sort (segment = query), then the rank map,
// volume scan, boundary deltas and boundary scan run over the concatenation
// and one workgroup per segment takes the exact argmin.
//
// The kernels that touch per-query state are templates over the state layout
// (DenseState or CompactState, see batch_device.h).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "batch_device.h"
#include "device_util.h"
#include "sort.h"

namespace plc {

constexpr int kMaxSlots = 1024;
// Per-tile slot range aggregated in LDS, and the hot destinations whose
// contributions the scatter sums in LDS (the first kHotB of the graph's kHot
// hot vertices): sized so that four scatter workgroups fit in a CU's LDS.
constexpr int kSlotRange = 128;
constexpr int kHotB = 1024;
static_assert(kHotB <= kHot, "the batched hot set is a prefix of the graph's");

__device__ __forceinline__ int slot_of(const int32_t* pref, int B, long long g) {
  // largest q in [0, B) with pref[q] <= g (pref[B] = total > g)
  int lo = 0, hi = B - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if ((long long)pref[mid] <= g) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ int seg_of(const long long* off, int nseg, long long k) {
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= k) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// ---------------------------------------------------------------- state layouts

// 32-bit finaliser of MurmurHash3 (a bijection on 32-bit words): spreads the
// clustered ids of high-degree R-MAT vertices over the table.
__device__ __forceinline__ uint32_t vhash(uint32_t x) {
  x ^= x >> 16;
  x *= 0x85ebca6bu;
  x ^= x >> 13;
  x *= 0xc2b2ae35u;
  x ^= x >> 16;
  return x;
}

// Home position of v in a table of `cap` records (any capacity: the hash is
// mapped onto [0, cap) by a multiply-high), and the next position of a probe.
__device__ __forceinline__ uint32_t home_of(int32_t v, uint32_t cap) {
  return (uint32_t)(((unsigned long long)vhash((uint32_t)v) * cap) >> 32);
}
__device__ __forceinline__ uint32_t probe_next(uint32_t h, uint32_t cap) {
  return h + 1 == cap ? 0u : h + 1;
}

// The part of a slot's state the edge scatter needs (staged in LDS per tile).
struct TabView {
  VRec* tab;
  int32_t tcap;
};

// Dense: record v of the slot's n records; always present.  The scatter's
// first load is the record's {d(v), hot code} word, which needs no probing.
struct DenseState {
  static constexpr bool kCompact = false;
  __device__ static unsigned long long probe_start(const BatchArgs&, const TabView& t, int32_t v,
                                                   uint32_t*) {
    return *reinterpret_cast<const unsigned long long*>(&t.tab[v].deg);
  }
  // record of v, its degree and hot index (-1 when not hot)
  __device__ static VRec* probe_finish(const BatchArgs&, const TabView& t, int32_t v, uint32_t,
                                       unsigned long long w, int32_t* d, int32_t* hj) {
    *d = (int32_t)(uint32_t)w;
    *hj = -(int32_t)(uint32_t)(w >> 32) - 1;
    return t.tab + v;
  }
  __device__ static int32_t hot_deg(const BatchArgs&, int32_t, int32_t d) { return d; }
  __device__ static VRec* find(const Slot& S, int32_t v) { return S.tab + v; }
  __device__ static VRec* insert(const BatchArgs&, const Slot& S, int32_t v) { return S.tab + v; }
  __device__ static int32_t rank_of(const Slot& S, int32_t v) { return S.tab[v].rank; }
  __device__ static int32_t rank_at(const VRec* tab, int32_t, int32_t v) { return tab[v].rank; }
  __device__ static double* pp(const Slot& S, int32_t v, const VRec*) { return S.tp + v; }
  __device__ static int2 deg_hot(const BatchArgs&, const Slot& S, int32_t v) {
    return *reinterpret_cast<const int2*>(&S.tab[v].deg);
  }
  __device__ static int32_t deg_rec(const BatchArgs&, int32_t, const VRec* rec) { return rec->deg; }
};

// Compact: linear probing from home_of(v).  A record's deg field holds the key
// (kEmptyKey when free) and its rank field, while the query pushes, a tag
// written together with the key: -(j+1) for hot vertex j, else
// -(1 + kHot + d(v)), so the scatter learns d(v) and hotness from the probe
// itself; the sweep overwrites the tags of the support with ranks >= 1 (its
// rank lookups treat any value < 1 as "not in the support").
struct CompactState {
  static constexpr bool kCompact = true;
  __device__ static int32_t tag_of(int2 dh) { return dh.y < 0 ? dh.y : -1 - kHot - dh.x; }
  __device__ static unsigned long long word(int32_t key, int32_t tag) {
    return (unsigned long long)(uint32_t)key | ((unsigned long long)(uint32_t)tag << 32);
  }
  __device__ static unsigned long long* kw(const TabView& t, uint32_t h) {
    return reinterpret_cast<unsigned long long*>(&t.tab[h].deg);
  }
  __device__ static unsigned long long probe_load(const unsigned long long* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  // record holding v, or nullptr when v is not in the table (valid after the
  // kernel that inserted v has finished)
  __device__ static VRec* find(const Slot& S, int32_t v) {
    const uint32_t cap = (uint32_t)S.tcap;
    uint32_t h = home_of(v, cap);
    for (uint32_t i = 0; i < cap; i++) {
      const int32_t k = S.tab[h].deg;
      if (k == v) return S.tab + h;
      if (k == kEmptyKey) return nullptr;
      h = probe_next(h, cap);
    }
    return nullptr;
  }
  // Resolve a probe of v that saw `w` at position h: the record holding v,
  // claimed together with its tag by a 64-bit compare-and-swap when v is new
  // (tag: the tag to write, or 0 to take it from gdh when needed); concurrent
  // inserts of v agree on one record.  *tag_out: the record's tag.  nullptr
  // only if the table is full.
  __device__ static VRec* claim(const BatchArgs& a, const TabView& t, int32_t v, uint32_t h,
                                unsigned long long w, int32_t tag, int32_t* tag_out) {
    const uint32_t cap = (uint32_t)t.tcap;
    for (uint32_t i = 0; i < cap; i++) {
      int32_t k = (int32_t)(uint32_t)w;
      if (k == kEmptyKey) {
        if (tag >= 0) tag = tag_of(a.gdh[v]);
        const unsigned long long old = atomicCAS(kw(t, h), w, word(v, tag));
        if (old == w) {
          *tag_out = tag;
          return t.tab + h;
        }
        w = old;  // taken meanwhile: by v, or by another key
        k = (int32_t)(uint32_t)w;
      }
      if (k == v) {
        *tag_out = (int32_t)(uint32_t)(w >> 32);
        return t.tab + h;
      }
      h = probe_next(h, cap);
      w = probe_load(kw(t, h));
    }
    return nullptr;
  }
  __device__ static VRec* insert_tag(const BatchArgs& a, const TabView& t, int32_t v, int32_t tag) {
    uint32_t h;
    const unsigned long long w = probe_start(a, t, v, &h);
    int32_t got;
    return claim(a, t, v, h, w, tag, &got);
  }
  __device__ static VRec* insert(const BatchArgs& a, const Slot& S, int32_t v) {
    return insert_tag(a, TabView{S.tab, S.tcap}, v, 0);
  }
  // The scatter's probe in two steps so that a thread's first loads overlap:
  // probe_start loads the {key, tag} word at v's home position, probe_finish
  // resolves it (probing on, or claiming a free record).
  __device__ static unsigned long long probe_start(const BatchArgs&, const TabView& t, int32_t v,
                                                   uint32_t* h) {
    *h = home_of(v, (uint32_t)t.tcap);
    return probe_load(kw(t, *h));
  }
  // record of v, its degree (-1 for a hot vertex: see hot_deg) and hot index
  // (-1 when not hot)
  __device__ static VRec* probe_finish(const BatchArgs& a, const TabView& t, int32_t v, uint32_t h,
                                       unsigned long long w, int32_t* d, int32_t* hj) {
    int32_t tag = 0;
    VRec* rec = (int32_t)(uint32_t)w == v ? t.tab + h : claim(a, t, v, h, w, 0, &tag);
    if ((int32_t)(uint32_t)w == v) tag = (int32_t)(uint32_t)(w >> 32);
    *hj = tag >= -kHot ? -tag - 1 : -1;
    *d = tag >= -kHot ? -1 : -1 - kHot - tag;
    return rec;
  }
  __device__ static int32_t hot_deg(const BatchArgs& a, int32_t v, int32_t d) {
    return d >= 0 ? d : a.gdh[v].x;
  }
  __device__ static int32_t deg_rec(const BatchArgs& a, int32_t v, const VRec* rec) {
    const int32_t tag = rec->rank;
    return tag < -kHot ? -1 - kHot - tag : a.gdh[v].x;
  }
  __device__ static int32_t rank_of(const Slot& S, int32_t v) { return rank_at(S.tab, S.tcap, v); }
  __device__ static int32_t rank_at(const VRec* tab, int32_t tcap, int32_t v) {
    const uint32_t cap = (uint32_t)tcap;
    uint32_t h = home_of(v, cap);
    for (uint32_t i = 0; i < cap; i++) {
      const int2 kr = *reinterpret_cast<const int2*>(&tab[h].deg);  // {key, rank or tag}
      if (kr.x == v) return kr.y;
      if (kr.x == kEmptyKey) return 0;
      h = probe_next(h, cap);
    }
    return 0;
  }
  __device__ static double* pp(const Slot& S, int32_t, const VRec* rec) {
    return S.tp + (rec - S.tab);
  }
  __device__ static int2 deg_hot(const BatchArgs& a, const Slot&, int32_t v) { return a.gdh[v]; }
};

// ---------------------------------------------------------------- init

__global__ void k_b_init(BatchArgs a) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < a.n;
       v += (int64_t)gridDim.x * blockDim.x) {
    VRec rec;
    rec.r = 0.0;
    rec.deg = (int32_t)(a.off[v + 1] - a.off[v]);
    rec.rank = a.hotcode[v];
    for (int q = 0; q < a.B; q++) {
      a.vr[(int64_t)q * a.n + v] = rec;
      a.p[(int64_t)q * a.n + v] = 0.0;
    }
  }
}

// Compact layout: graph-wide {d(v), hot code} records.
__global__ void k_gdh_init(BatchArgs a, int2* gdh) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < a.n;
       v += (int64_t)gridDim.x * blockDim.x)
    gdh[v] = make_int2((int32_t)(a.off[v + 1] - a.off[v]), a.hotcode[v]);
}

template <class St>
__global__ void k_b_admit(BatchArgs a, const Admit* adm, int count) {
  for (int i = threadIdx.x; i < count; i += blockDim.x) {
    Admit ad = adm[i];
    if (ad.slot < 0 || ad.slot >= a.B || ad.seed < 0 || ad.seed >= a.n || ad.list_cap < 1) continue;
    Slot& S = a.slots[ad.slot];
    if (ad.rule == 1) {
      S.cs = ad.alpha;
      S.cn = (1.0 - ad.alpha) / 2.0;
      S.keep = (1.0 - ad.alpha) / 2.0;
      S.opt = 0;
    } else {
      S.cs = 2.0 * ad.alpha / (1.0 + ad.alpha);
      S.cn = (1.0 - ad.alpha) / (1.0 + ad.alpha);
      S.keep = 0.0;
      S.opt = 1;
    }
    S.eps = ad.eps;
    S.seed = ad.seed;
    S.max_rounds = ad.max_rounds;
    S.par = 0;
    S.cnt[0] = 1;
    S.cnt[1] = 0;
    S.rounds = 0;
    S.edge_next[0] = ad.seed_deg;
    S.edge_next[1] = 0;
    S.pushes = 0;
    S.edges = 0;
    S.support_cnt = 0;
    S.touched_cnt = 1;
    S.fbase = -1;
    S.nf = 0;
    S.limited = 0;
    S.fault = 0;
    S.round_edges = 0;
    S.kstar = 0;
    S.best_cut = 0;
    S.best_vol = 0;
    S.best_den = 0;
    S.phi = 0.0;
    S.rnnz = 0;
    S.hold = 0;
    S.tab = ad.tab;
    S.tp = ad.tp;
    S.fb[0] = ad.fb0;
    S.fb[1] = ad.fb1;
    S.support = ad.support;
    S.touched = ad.touched;
    S.tcap = ad.tcap;
    S.list_cap = ad.list_cap;
    S.fb[0][0] = ad.seed;
    S.touched[0] = ad.seed;
    VRec* rec = St::insert(a, S, ad.seed);  // a fresh (cleared) table: never full
    if (rec) rec->r = 1.0; else S.fault = 1;
    S.t_admit = (long long)wall_clock64();
    S.t_done = 0;
    S.status = SL_PUSH;
  }
}

// ---------------------------------------------------------------- round

__global__ __launch_bounds__(kMaxSlots) void k_b_plan(BatchArgs a) {
  __shared__ long long sh[kMaxSlots / 64 + 1];
  const int q = threadIdx.x;
  BatchCtl* c = a.ctl;
  long long nf = 0, e = 0;
  if (q < a.B) {
    Slot& S = a.slots[q];
    S.fbase = -1;
    S.nf = 0;
    S.round_edges = 0;
    if (S.status == SL_PUSH && !S.hold) {
      int cur = S.cnt[S.par];
      if (cur <= 0) {
        S.status = SL_PUSHED;
      } else if (S.rounds >= S.max_rounds) {
        S.limited = 1;
        S.status = SL_PUSHED;
      } else {
        nf = cur < S.list_cap ? cur : S.list_cap;
        e = S.edge_next[S.par];
      }
    }
  }
  long long tot_nf, tot_e;
  long long ex_nf = block_excl_scan<kMaxSlots>(nf, &tot_nf, sh);
  long long ex_e = block_excl_scan<kMaxSlots>(e, &tot_e, sh);
  // Slots are taken in order while the round buffers can hold them.
  const bool inc = nf > 0 && ex_nf + nf <= a.nf_cap && ex_e + e <= a.e_cap;
  long long inf = inc ? nf : 0, ie = inc ? e : 0;
  long long tot_inf, tot_ie;
  long long p_nf = block_excl_scan<kMaxSlots>(inf, &tot_inf, sh);
  (void)block_excl_scan<kMaxSlots>(ie, &tot_ie, sh);
  if (q < a.B) {
    a.fprefix[q] = (int32_t)p_nf;
    Slot& S = a.slots[q];
    if (inc) {
      S.fbase = (int32_t)p_nf;
      S.nf = (int32_t)inf;
      S.round_edges = ie;
    }
  }
  if (q == 0) {
    a.fprefix[a.B] = (int32_t)tot_inf;
    c->nf_total = (int32_t)tot_inf;
    c->e_total = tot_ie;
    c->ntiles = (int)((tot_ie + kEdgeTile - 1) / kEdgeTile);
  }
}

template <class St>
__global__ __launch_bounds__(kBlock) void k_b_self(BatchArgs a) {
  BatchCtl* c = a.ctl;
  const int NF = c->nf_total;
  if (NF <= 0) return;
  const int B = a.B;
  __shared__ int32_t s_pref[kMaxSlots + 1];
  __shared__ long long sh[kBlock / 64 + 1];
  __shared__ long long s_excl;
  __shared__ int s_tk[2];
  __shared__ int s_qlo, s_qhi;
  __shared__ int s_csup[kScanBlock], s_cstay[kScanBlock];
  __shared__ unsigned long long s_estay[kScanBlock];
  __shared__ int s_bsup[kScanBlock], s_bstay[kScanBlock];
  for (int j = threadIdx.x; j <= B; j += kBlock) s_pref[j] = a.fprefix[j];
  ScanSite* site = &c->scan[BSCAN_FRONTIER];
  scan_clear_prev(site, a.desc[BSCAN_FRONTIER], a.desc_cap);
  unsigned long long* desc = a.desc[BSCAN_FRONTIER] + (size_t)site->parity * a.desc_cap;
  const int nblk = (NF + kScanBlock - 1) / kScanBlock;
  __syncthreads();

  for (;;) {
    bool last;
    int b = scan_ticket(site, nblk, s_tk, &last);
    if (b >= nblk) break;
    if (threadIdx.x == 0) {
      long long g0 = (long long)b * kScanBlock;
      long long g1 = g0 + kScanBlock - 1 < NF - 1 ? g0 + kScanBlock - 1 : NF - 1;
      s_qlo = slot_of(s_pref, B, g0);
      s_qhi = slot_of(s_pref, B, g1);
    }
    __syncthreads();
    const int qlo = s_qlo;
    const int range = s_qhi - qlo + 1;  // <= kScanBlock: each entry is one slot
    for (int j = threadIdx.x; j < range; j += kBlock) {
      s_csup[j] = 0;
      s_cstay[j] = 0;
      s_estay[j] = 0ull;
    }
    __syncthreads();
    int32_t vk[kScanItems], dk[kScanItems], qk[kScanItems], rsup[kScanItems], rstay[kScanItems];
    long long dsum = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; k++) {
      const long long g = (long long)b * kScanBlock + k * kBlock + threadIdx.x;
      vk[k] = -1;
      dk[k] = 0;
      qk[k] = 0;
      rsup[k] = -1;
      rstay[k] = -1;
      if (g < NF) {
        const int q = slot_of(s_pref, B, g);
        const Slot& S = a.slots[q];
        const int i = (int)(g - s_pref[q]);
        const int32_t v = S.fb[S.par][i];
        VRec* rp = St::find(S, v);
        double rho = 0.0;
        int32_t d = 0;
        if (rp) {
          rho = rp->r;
          d = St::deg_rec(a, v, rp);
          double* pv = St::pp(S, v, rp);
          const double pold = *pv;
          *pv = pold + S.cs * rho;
          const double nr = S.opt ? -0.0 : S.keep * rho;
          rp->r = nr;
          if (pold == 0.0) rsup[k] = atomicAdd(&s_csup[q - qlo], 1);
          if (!S.opt && nr >= S.eps * (double)d) {
            rstay[k] = atomicAdd(&s_cstay[q - qlo], 1);
            atomicAdd(&s_estay[q - qlo], (unsigned long long)d);
          }
        } else {
          c->fault = 1;  // a frontier vertex always has a record
        }
        a.coef[g] = d > 0 ? (S.cn * rho) / (double)d : 0.0;
        a.rowp[g] = a.off[v];
        a.eslot[g] = q;
        vk[k] = v;
        dk[k] = d;
        qk[k] = q;
      }
      dsum += dk[k];
    }
    __syncthreads();
    for (int j = threadIdx.x; j < range; j += kBlock) {
      Slot& S = a.slots[qlo + j];
      s_bsup[j] = s_csup[j] > 0 ? atomicAdd(&S.support_cnt, s_csup[j]) : 0;
      if (s_cstay[j] > 0) {
        const int nxt = S.par ^ 1;
        s_bstay[j] = atomicAdd(&S.cnt[nxt], s_cstay[j]);
        atomicAdd((unsigned long long*)&S.edge_next[nxt], s_estay[j]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kScanItems; k++) {
      if (vk[k] < 0) continue;
      const Slot& S = a.slots[qk[k]];
      if (rsup[k] >= 0) {
        const long long pos = (long long)s_bsup[qk[k] - qlo] + rsup[k];
        if (pos < S.list_cap) S.support[pos] = vk[k]; else c->fault = 1;
      }
      if (rstay[k] >= 0) {
        const long long pos = (long long)s_bstay[qk[k] - qlo] + rstay[k];
        if (pos < S.list_cap) S.fb[S.par ^ 1][pos] = vk[k]; else c->fault = 1;
      }
    }
    long long agg;
    (void)block_excl_scan<kBlock>(dsum, &agg, sh);
    if (threadIdx.x < 64) {
      const long long ex0 = scan_lookback(desc, b, agg, &c->fault);
      if (threadIdx.x == 0) s_excl = ex0;
    }
    __syncthreads();
    long long run = s_excl;
    for (int k = 0; k < kScanItems; k++) {
      const long long g = (long long)b * kScanBlock + k * kBlock + threadIdx.x;
      long long tot;
      long long ex = block_excl_scan<kBlock>(dk[k], &tot, sh);
      if (g < NF) {
        const long long s = run + ex;
        a.estart[g] = s;
        long long t0 = (s + kEdgeTile - 1) / kEdgeTile;
        long long t1 = (s + dk[k] - 1) / kEdgeTile;
        if (t1 >= a.tile_cap) { c->fault = 1; t1 = a.tile_cap - 1; }
        for (long long tt = t0; tt <= t1; tt++) a.tile_start[tt] = (int32_t)g;
      }
      run += tot;
    }
    if (b == nblk - 1 && threadIdx.x == 0) {
      if (run != c->e_total) c->fault = 1;  // planned and scanned edge counts must agree
    }
    __syncthreads();
  }
}

// Append w to slot q's next frontier and/or touched list with direct global
// reservations (used for the few decisions taken outside the tile loop).
__device__ __forceinline__ void b_decide_direct(const BatchArgs& a, int q, int32_t w, int32_t dw,
                                                double old, double c, int* fault) {
  Slot& S = a.slots[q];
  const double thr = S.eps * (double)dw;
  if (old < thr && old + c >= thr) {
    const int nxt = S.par ^ 1;
    long long pos = atomicAdd(&S.cnt[nxt], 1);
    atomicAdd((unsigned long long*)&S.edge_next[nxt], (unsigned long long)dw);
    if (pos < S.list_cap) S.fb[nxt][pos] = w; else *fault = 1;
  }
  if (__double_as_longlong(old) == 0) {
    long long pos = atomicAdd(&S.touched_cnt, 1);
    if (pos < S.list_cap) S.touched[pos] = w; else *fault = 1;
  }
}

// Add the LDS sums of slot hs's hot destinations to r (one atomic each) and
// clear them.  Every thread of the workgroup must call it.
template <class St>
__device__ void b_flush_hot(const BatchArgs& a, int hs, double* s_hacc, int* fault) {
  __syncthreads();
  if (hs >= 0) {
    const Slot& S = a.slots[hs];
    for (int j = threadIdx.x; j < kHotB; j += kBlock) {
      const double sum = s_hacc[j];
      if (sum != 0.0) {
        s_hacc[j] = 0.0;
        const int32_t w = a.hot_ids[j];
        VRec* rec = St::insert(a, S, w);
        if (!rec) {
          *fault = 1;
          continue;
        }
        const double old = unsafeAtomicAdd(&rec->r, sum);
        b_decide_direct(a, hs, w, St::deg_hot(a, S, w).x, old, sum, fault);
      }
    }
  }
  __syncthreads();
}

// edgeMap over all scheduled edges.  Each workgroup takes a contiguous range
// of tiles, numbered XCD-major (xcd_block) so that a slot's edges stay within
// one XCD's L2 (12 % less fetched from memory on R-MAT 2^22 with 256 slots);
// contributions to hot destinations of the slot that owns the current tiles
// are summed in LDS and flushed when the range moves to another slot, and at
// the end.
template <class St>
__global__ __launch_bounds__(kBlock) void k_b_scatter(BatchArgs a) {
  BatchCtl* c = a.ctl;
  const int NF = c->nf_total;
  if (NF <= 0) return;
  const int ntiles = (int64_t)c->ntiles > a.tile_cap ? (int)a.tile_cap : c->ntiles;
  const long long E = c->e_total;
  __shared__ int32_t s_start[kEdgeTile + 1];
  __shared__ int64_t s_row[kEdgeTile + 1];
  __shared__ double s_coef[kEdgeTile + 1];
  __shared__ int32_t s_slot[kEdgeTile + 1];
  __shared__ int s_cfn[kSlotRange], s_ctv[kSlotRange], s_bfn[kSlotRange], s_btv[kSlotRange];
  __shared__ unsigned long long s_efn[kSlotRange];
  __shared__ TabView s_view[kSlotRange];
  __shared__ double s_eps[kSlotRange];
  __shared__ double s_hacc[kHotB];
  int hs = -1;  // slot whose hot sums s_hacc holds
  const int per = (ntiles + gridDim.x - 1) / gridDim.x;
  const int tb = xcd_block(blockIdx.x, gridDim.x) * per;
  const int te = tb + per < ntiles ? tb + per : ntiles;
  if (tb >= te) return;  // no tiles for this workgroup
  for (int j = threadIdx.x; j < kHotB; j += kBlock) s_hacc[j] = 0.0;
  __syncthreads();

  for (int tile = tb; tile < te; tile++) {
    const long long e0 = (long long)tile * kEdgeTile;
    const long long e1 = e0 + kEdgeTile < E ? e0 + kEdgeTile : E;
    const int i0 = a.tile_start[tile];
    const int i1 = tile + 1 < ntiles ? a.tile_start[tile + 1] : NF - 1;
    if (i0 < 0 || i1 < i0 || i1 >= NF || i1 - i0 + 1 > kEdgeTile + 1) {
      c->fault = 1;
      continue;
    }
    const int cnt = i1 - i0 + 1;
    const int tile_hs = a.eslot[i1];
    if (tile_hs != hs) {
      b_flush_hot<St>(a, hs, s_hacc, &c->fault);
      hs = tile_hs;
    }
    // the tile's entries belong to slots qlo..tile_hs (ascending)
    const int qlo = a.eslot[i0];
    const int range = tile_hs - qlo + 1;
    const int rr = range < kSlotRange ? range : kSlotRange;
    for (int j = threadIdx.x; j < rr; j += kBlock) {
      const Slot& S = a.slots[qlo + j];
      s_view[j] = TabView{S.tab, S.tcap};
      s_eps[j] = S.eps;
    }
    for (int j = threadIdx.x; j < cnt; j += kBlock) {
      s_start[j] = (int32_t)(a.estart[i0 + j] - e0);
      s_row[j] = a.rowp[i0 + j];
      s_coef[j] = a.coef[i0 + j];
      s_slot[j] = a.eslot[i0 + j];
    }
    for (int j = threadIdx.x; j < kSlotRange; j += kBlock) {
      s_cfn[j] = 0;
      s_ctv[j] = 0;
      s_efn[j] = 0ull;
    }
    __syncthreads();
    int32_t w[kEdgesPerThread], q[kEdgesPerThread];
    double cf[kEdgesPerThread];
#pragma unroll
    for (int k = 0; k < kEdgesPerThread; k++) {
      const int rel = k * kBlock + (int)threadIdx.x;
      w[k] = -1;
      q[k] = 0;
      cf[k] = 0.0;
      if (e0 + rel < e1) {
        int lo = 0, hi = cnt - 1;
        while (lo < hi) {
          int mid = (lo + hi + 1) >> 1;
          if (s_start[mid] <= rel) lo = mid; else hi = mid - 1;
        }
        w[k] = a.nbr[s_row[lo] + (rel - s_start[lo])];
        cf[k] = s_coef[lo];
        q[k] = s_slot[lo];
      }
    }
    // first load of every edge (dense: the record's {d, hot code} word;
    // compact: the {key, tag} word at the home position), then resolution
    // (compact: probing on or claiming a record); hot destinations of the
    // current slot are then combined in LDS, the others take the atomics
    TabView tv[kEdgesPerThread];
    uint32_t hp[kEdgesPerThread];
    unsigned long long k0[kEdgesPerThread];
#pragma unroll
    for (int k = 0; k < kEdgesPerThread; k++) {
      if (w[k] < 0) continue;
      const int j = q[k] - qlo;
      const Slot& S = a.slots[q[k]];
      tv[k] = j < kSlotRange ? s_view[j] : TabView{S.tab, S.tcap};
      k0[k] = St::probe_start(a, tv[k], w[k], &hp[k]);
    }
    VRec* rec[kEdgesPerThread];
    int32_t dw[kEdgesPerThread];
    double old[kEdgesPerThread];
    bool pend[kEdgesPerThread];
#pragma unroll
    for (int k = 0; k < kEdgesPerThread; k++) {
      rec[k] = nullptr;
      dw[k] = 0;
      old[k] = 0.0;
      pend[k] = w[k] >= 0;
    }
    // resolve edge k's first word into its record, then the LDS sum (hot
    // destination of the current slot) or the atomic on r
    auto settle = [&](int k) {
      pend[k] = false;
      int32_t hj;
      rec[k] = St::probe_finish(a, tv[k], w[k], hp[k], k0[k], &dw[k], &hj);
      if (!rec[k]) {
        c->fault = 1;  // full table: the host sizes tables so that this cannot happen
        w[k] = -1;
        return;
      }
      if (hj >= 0) {
        if (q[k] == hs && hj < kHotB) {
          atomicAdd(&s_hacc[hj], cf[k]);
          w[k] = -1;
          return;
        }
        dw[k] = St::hot_deg(a, w[k], dw[k]);
      }
      old[k] = unsafeAtomicAdd(&rec[k]->r, cf[k]);
    };
    if constexpr (St::kCompact) {
      // destinations found at home: their atomics go out at once; then those
      // whose home record was free: their tags and every claim of the thread
      // in flight together (a lost claim leaves the record's current word for
      // the resolution below to probe on from)
#pragma unroll
      for (int k = 0; k < kEdgesPerThread; k++)
        if (pend[k] && (int32_t)(uint32_t)k0[k] == w[k]) settle(k);
      int32_t tg[kEdgesPerThread];
#pragma unroll
      for (int k = 0; k < kEdgesPerThread; k++) {
        tg[k] = 0;
        if (pend[k] && (int32_t)(uint32_t)k0[k] == kEmptyKey)
          tg[k] = CompactState::tag_of(a.gdh[w[k]]);
      }
#pragma unroll
      for (int k = 0; k < kEdgesPerThread; k++) {
        if (tg[k] >= 0) continue;
        const unsigned long long want = CompactState::word(w[k], tg[k]);
        const unsigned long long got = atomicCAS(CompactState::kw(tv[k], hp[k]), k0[k], want);
        k0[k] = got == k0[k] ? want : got;
      }
    }
#pragma unroll
    for (int k = 0; k < kEdgesPerThread; k++)
      if (pend[k]) settle(k);
    // decisions: rank within (slot, list) from LDS counters, or a direct
    // global reservation when the tile spans more slots than the LDS range
    int rfn[kEdgesPerThread], rtv[kEdgesPerThread];
#pragma unroll
    for (int k = 0; k < kEdgesPerThread; k++) {
      rfn[k] = -1;
      rtv[k] = -1;
      if (w[k] < 0) continue;
      const int j = q[k] - qlo;
      if (j < kSlotRange) {
        const double thr = s_eps[j] * (double)dw[k];
        if (old[k] < thr && old[k] + cf[k] >= thr) {
          rfn[k] = atomicAdd(&s_cfn[j], 1);
          atomicAdd(&s_efn[j], (unsigned long long)dw[k]);
        }
        if (__double_as_longlong(old[k]) == 0) rtv[k] = atomicAdd(&s_ctv[j], 1);
      } else {
        b_decide_direct(a, q[k], w[k], dw[k], old[k], cf[k], &c->fault);
      }
    }
    __syncthreads();
    for (int j = threadIdx.x; j < rr; j += kBlock) {
      Slot& S = a.slots[qlo + j];
      const int nxt = S.par ^ 1;
      s_bfn[j] = 0;
      s_btv[j] = 0;
      if (s_cfn[j] > 0) {
        s_bfn[j] = atomicAdd(&S.cnt[nxt], s_cfn[j]);
        atomicAdd((unsigned long long*)&S.edge_next[nxt], s_efn[j]);
      }
      if (s_ctv[j] > 0) s_btv[j] = atomicAdd(&S.touched_cnt, s_ctv[j]);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kEdgesPerThread; k++) {
      if (rfn[k] < 0 && rtv[k] < 0) continue;
      const int j = q[k] - qlo;
      const Slot& S = a.slots[q[k]];
      if (rfn[k] >= 0) {
        const long long pos = (long long)s_bfn[j] + rfn[k];
        if (pos < S.list_cap) S.fb[S.par ^ 1][pos] = w[k]; else c->fault = 1;
      }
      if (rtv[k] >= 0) {
        const long long pos = (long long)s_btv[j] + rtv[k];
        if (pos < S.list_cap) S.touched[pos] = w[k]; else c->fault = 1;
      }
    }
    __syncthreads();
  }
  b_flush_hot<St>(a, hs, s_hacc, &c->fault);
}

__global__ __launch_bounds__(kMaxSlots) void k_b_round_end(BatchArgs a) {
  const int q = threadIdx.x;
  if (q >= a.B) return;
  Slot& S = a.slots[q];
  if (S.fbase < 0 || S.status != SL_PUSH) return;
  S.pushes += S.nf;
  S.edges += S.round_edges;
  S.rounds += 1;
  S.cnt[S.par] = 0;
  S.edge_next[S.par] = 0;
  S.par ^= 1;
  S.fbase = -1;
  if (S.cnt[S.par] == 0) S.status = SL_PUSHED;
}

// ---------------------------------------------------------------- compact tables

constexpr int kMaxClearJobs = 2 * kMaxSlots;  // admissions + growths of one step

// Tables are processed in runs of 256 records (4 per lane of a wave):
// capacities are multiples of kScanBlock records, so a run of the
// concatenated tables lies in one table and one search finds it.
constexpr int kTabRun = 4 * 64;
static_assert(kScanBlock % kTabRun == 0, "table runs lie in one table");

// Clear every record (key kEmptyKey, r 0, rank 0) and p of each job's
// block; the runs cover the records of all jobs end to end.
__global__ __launch_bounds__(kBlock) void k_c_clear(const ClearJob* jobs, int count,
                                                    long long total) {
  __shared__ long long s_off[kMaxClearJobs];
  for (int j = threadIdx.x; j < count; j += kBlock) s_off[j] = jobs[j].off;
  __syncthreads();
  const long long nrun = total / kTabRun;
  const long long nw = (long long)gridDim.x * (kBlock / 64);
  VRec r;
  r.r = 0.0;
  r.deg = kEmptyKey;
  r.rank = 0;
  for (long long wr = (long long)blockIdx.x * (kBlock / 64) + PLC_WID; wr < nrun; wr += nw) {
    const long long x0 = wr * kTabRun;
    const int j = seg_of(s_off, count, x0);
    const ClearJob& J = jobs[j];
    const long long i0 = x0 - s_off[j];
    if (i0 + kTabRun > J.cap) continue;
#pragma unroll
    for (int k = 0; k < 4; k++) {
      J.tab[i0 + k * 64 + PLC_LANE] = r;
      J.tp[i0 + k * 64 + PLC_LANE] = 0.0;
    }
  }
}

// Re-insert every record of the growing tables into their new (cleared)
// tables; the runs cover the old records of all growing tables end to end.
__global__ __launch_bounds__(kBlock) void k_c_rehash(BatchArgs a, const Grow* gr, int count,
                                                     long long total) {
  __shared__ long long s_off[kMaxSlots];
  for (int j = threadIdx.x; j < count; j += kBlock) s_off[j] = gr[j].rec_off;
  __syncthreads();
  const long long nrun = total / kTabRun;
  const long long nw = (long long)gridDim.x * (kBlock / 64);
  for (long long wr = (long long)blockIdx.x * (kBlock / 64) + PLC_WID; wr < nrun; wr += nw) {
    const long long x0 = wr * kTabRun;
    const int j = seg_of(s_off, count, x0);
    const Grow& G = gr[j];
    const Slot& S = a.slots[G.slot];  // still the old table
    const long long i0 = x0 - s_off[j];
    if (i0 + kTabRun > G.old_cap) continue;
    VRec rec[4];
#pragma unroll
    for (int k = 0; k < 4; k++) rec[k] = S.tab[i0 + k * 64 + PLC_LANE];
#pragma unroll
    for (int k = 0; k < 4; k++) {
      if (rec[k].deg == kEmptyKey) continue;
      VRec* dst = CompactState::insert_tag(a, TabView{G.tab, G.new_cap}, rec[k].deg, rec[k].rank);
      if (!dst) {
        a.ctl->fault = 1;
        continue;
      }
      dst->r = rec[k].r;  // (the key and its tag went in with the claim)
      G.tp[dst - G.tab] = S.tp[i0 + k * 64 + PLC_LANE];
    }
  }
}

// Copy the current frontier, support and touched lists of the growing slots
// to their new blocks; x runs over those entries of all slots end to end.
__global__ __launch_bounds__(kBlock) void k_c_move_lists(BatchArgs a, const Grow* gr, int count,
                                                         long long total) {
  __shared__ long long s_off[kMaxSlots];
  for (int j = threadIdx.x; j < count; j += kBlock) s_off[j] = gr[j].list_off;
  __syncthreads();
  for (long long x = (long long)blockIdx.x * kBlock + threadIdx.x; x < total;
       x += (long long)gridDim.x * kBlock) {
    const int j = seg_of(s_off, count, x);
    const Grow& G = gr[j];
    const Slot& S = a.slots[G.slot];  // still the old block
    long long i = x - s_off[j];
    if (i < G.n_front) {
      (G.par == 0 ? G.fb0 : G.fb1)[i] = S.fb[G.par][i];
      continue;
    }
    i -= G.n_front;
    if (i < G.n_sup) {
      G.support[i] = S.support[i];
      continue;
    }
    i -= G.n_sup;
    if (i < G.n_touch) G.touched[i] = S.touched[i];
  }
}

// Point each growing slot at its new block (after the rehash and the copy).
__global__ void k_c_commit(BatchArgs a, const Grow* gr, int count) {
  for (int j = threadIdx.x; j < count; j += blockDim.x) {
    const Grow& G = gr[j];
    Slot& S = a.slots[G.slot];
    if (S.par != G.par || S.cnt[G.par] != G.n_front || S.cnt[G.par ^ 1] != 0 ||
        S.support_cnt != G.n_sup || S.touched_cnt != G.n_touch || G.n_touch > G.list_cap)
      a.ctl->fault = 1;  // the host's copy of the slot was stale
    S.tab = G.tab;
    S.tp = G.tp;
    S.fb[0] = G.fb0;
    S.fb[1] = G.fb1;
    S.support = G.support;
    S.touched = G.touched;
    S.tcap = G.new_cap;
    S.list_cap = G.list_cap;
    S.hold = 0;
  }
}

__global__ void k_slot_hold(BatchArgs a, const int32_t* holds, int count) {
  for (int i = threadIdx.x; i < count; i += blockDim.x) {
    const int q = holds[i] & 0xffff;
    if (q < a.B) a.slots[q].hold = holds[i] >> 16;
  }
}

// ---------------------------------------------------------------- sweep

template <class St>
__global__ __launch_bounds__(kBlock) void k_sw_keys(BatchArgs a) {
  BatchCtl* c = a.ctl;
  const int nseg = c->sw_nseg;
  const long long total = c->sw_total;
  __shared__ long long s_off[kMaxSlots];
  for (int j = threadIdx.x; j < nseg; j += kBlock) s_off[j] = a.segs[j].elem_off;
  if (blockIdx.x == 0 && threadIdx.x == 0) c->sort_flip = 0;
  __syncthreads();
  for (long long k = (long long)blockIdx.x * kBlock + threadIdx.x; k < total;
       k += (long long)gridDim.x * kBlock) {
    const int s = seg_of(s_off, nseg, k);
    const SweepSeg& sg = a.segs[s];
    const Slot& S = a.slots[sg.slot];
    const int32_t v = S.support[k - s_off[s]];
    const VRec* rp = St::find(S, v);
    double ratio = 0.0;
    if (rp) ratio = *St::pp(S, v, rp) / (double)St::deg_hot(a, S, v).x;
    else c->fault = 1;
    SortElem e;
    e.key = ~(unsigned long long)__double_as_longlong(ratio);
    e.id = v;
    e.seg = s;
    a.sbuf[0][k] = e;
  }
}

template <class St>
__global__ __launch_bounds__(kBlock) void k_sw_rank(BatchArgs a) {
  BatchCtl* c = a.ctl;
  const long long total = c->sw_total;
  const SortElem* el = a.sbuf[c->sort_flip & 1];
  for (long long k = (long long)blockIdx.x * kBlock + threadIdx.x; k < total;
       k += (long long)gridDim.x * kBlock) {
    const SortElem e = el[k];
    const SweepSeg& sg = a.segs[e.seg];
    const Slot& S = a.slots[sg.slot];
    const long long i = k - sg.elem_off;
    VRec* rp = St::find(S, e.id);
    if (!rp) {
      c->fault = 1;
      continue;
    }
    rp->rank = (int32_t)(i + 1);
    a.sdeg[k] = St::deg_hot(a, S, e.id).x;
    if (sg.out_ids) {
      sg.out_ids[i] = e.id;
      sg.out_p[i] = *St::pp(S, e.id, rp);
    }
    a.scnt[k] = 0;
  }
}

// Inclusive scan of src[k] (or of sdeg - 2*scnt when cut) into dst, and,
// for the volume scan, the edge-tile map over the concatenated supports.
template <bool CUT>
__global__ __launch_bounds__(kBlock) void k_sw_scan(BatchArgs a) {
  BatchCtl* c = a.ctl;
  const long long total = c->sw_total;
  if (total <= 0) return;
  __shared__ long long sh[kBlock / 64 + 1];
  __shared__ long long s_excl;
  __shared__ int s_tk[2];
  const int site_id = CUT ? BSCAN_CUT : BSCAN_VOL;
  ScanSite* site = &c->scan[site_id];
  scan_clear_prev(site, a.desc[site_id], a.desc_cap);
  unsigned long long* desc = a.desc[site_id] + (size_t)site->parity * a.desc_cap;
  const int nblk = (int)((total + kScanBlock - 1) / kScanBlock);
  for (;;) {
    bool last;
    int b = scan_ticket(site, nblk, s_tk, &last);
    if (b >= nblk) break;
    long long xk[kScanItems];
    long long xsum = 0;
    for (int k = 0; k < kScanItems; k++) {
      const long long i = (long long)b * kScanBlock + k * kBlock + threadIdx.x;
      xk[k] = 0;
      if (i < total) xk[k] = CUT ? (long long)a.sdeg[i] - 2ll * a.scnt[i] : (long long)a.sdeg[i];
      xsum += xk[k];
    }
    long long agg;
    (void)block_excl_scan<kBlock>(xsum, &agg, sh);
    if (threadIdx.x < 64) {
      const long long ex0 = scan_lookback(desc, b, agg, &c->fault);
      if (threadIdx.x == 0) s_excl = ex0;
    }
    __syncthreads();
    long long run = s_excl;
    for (int k = 0; k < kScanItems; k++) {
      const long long i = (long long)b * kScanBlock + k * kBlock + threadIdx.x;
      long long tot;
      long long ex = block_excl_scan<kBlock>(xk[k], &tot, sh);
      if (i < total) {
        const long long s = run + ex;
        if (CUT) {
          a.scut[i] = s + xk[k];
        } else {
          a.svol[i] = s + xk[k];
          long long t0 = (s + kEdgeTile - 1) / kEdgeTile;
          long long t1 = (s + xk[k] - 1) / kEdgeTile;
          if (t1 >= a.tile_cap) { c->fault = 1; t1 = a.tile_cap - 1; }
          for (long long tt = t0; tt <= t1; tt++) a.tile_start[tt] = (int32_t)i;
        }
      }
      run += tot;
    }
    if (!CUT && b == nblk - 1 && threadIdx.x == 0) {
      c->sw_etotal = run;
      c->sw_ntiles = (int)((run + kEdgeTile - 1) / kEdgeTile);
    }
    __syncthreads();
  }
}

template <class St>
__global__ __launch_bounds__(kBlock) void k_sw_count(BatchArgs a) {
  BatchCtl* c = a.ctl;
  const long long total = c->sw_total;
  if (total <= 0) return;
  const int ntiles = (int64_t)c->sw_ntiles > a.tile_cap ? (int)a.tile_cap : c->sw_ntiles;
  const long long E = c->sw_etotal;
  const SortElem* el = a.sbuf[c->sort_flip & 1];
  __shared__ int32_t s_start[kEdgeTile + 1];
  __shared__ int64_t s_row[kEdgeTile + 1];
  __shared__ int32_t s_cnt[kEdgeTile + 1];
  __shared__ int32_t s_own[kEdgeTile + 1];
  __shared__ const VRec* s_tab[kEdgeTile + 1];
  __shared__ int32_t s_tcap[kEdgeTile + 1];
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const long long e0 = (long long)tile * kEdgeTile;
    const long long e1 = e0 + kEdgeTile < E ? e0 + kEdgeTile : E;
    const int i0 = a.tile_start[tile];
    const int i1 = tile + 1 < ntiles ? a.tile_start[tile + 1] : (int)(total - 1);
    if (i0 < 0 || i1 < i0 || i1 >= total || i1 - i0 + 1 > kEdgeTile + 1) {
      c->fault = 1;
      continue;
    }
    const int cnt = i1 - i0 + 1;
    for (int j = threadIdx.x; j < cnt; j += kBlock) {
      const long long k = i0 + j;
      const SortElem e = el[k];
      const SweepSeg& sg = a.segs[e.seg];
      s_start[j] = (int32_t)(a.svol[k] - a.sdeg[k] - e0);
      s_row[j] = a.off[e.id];
      s_own[j] = (int32_t)(k - sg.elem_off + 1);
      const Slot& S = a.slots[sg.slot];
      s_tab[j] = S.tab;
      s_tcap[j] = S.tcap;
      s_cnt[j] = 0;
    }
    __syncthreads();
    int32_t rw[kEdgesPerThread];
    int own[kEdgesPerThread];
#pragma unroll
    for (int kk = 0; kk < kEdgesPerThread; kk++) {
      const int rel = kk * kBlock + (int)threadIdx.x;
      own[kk] = -1;
      rw[kk] = 0;
      if (e0 + rel < e1) {
        int lo = 0, hi = cnt - 1;
        while (lo < hi) {
          int mid = (lo + hi + 1) >> 1;
          if (s_start[mid] <= rel) lo = mid; else hi = mid - 1;
        }
        const int32_t w = a.nbr[s_row[lo] + (rel - s_start[lo])];
        rw[kk] = St::rank_at(s_tab[lo], s_tcap[lo], w);
        own[kk] = lo;
      }
    }
#pragma unroll
    for (int kk = 0; kk < kEdgesPerThread; kk++)
      if (own[kk] >= 0 && rw[kk] > 0 && rw[kk] < s_own[own[kk]]) atomicAdd(&s_cnt[own[kk]], 1);
    __syncthreads();
    for (int j = threadIdx.x; j < cnt; j += kBlock)
      if (s_cnt[j] != 0) atomicAdd(&a.scnt[i0 + j], s_cnt[j]);
    __syncthreads();
  }
}

__device__ __forceinline__ bool b_cand_better(long long oc, long long od, long long ok,
                                              long long xc, long long xd, long long xk) {
  if (ok <= 0) return false;
  if (xk <= 0) return true;
  if (ratio_lt(oc, od, xc, xd)) return true;
  return !ratio_lt(xc, xd, oc, od) && ok < xk;
}

// One workgroup per segment: exact argmin of cut/min(vol, 2m - vol).
__global__ __launch_bounds__(kBlock) void k_sw_argmin(BatchArgs a) {
  BatchCtl* c = a.ctl;
  const int s = blockIdx.x;
  if (s >= c->sw_nseg) return;
  const SweepSeg sg = a.segs[s];
  const long long off = sg.elem_off;
  const long long bv = off > 0 ? a.svol[off - 1] : 0;
  const long long bc = off > 0 ? a.scut[off - 1] : 0;
  const long long vt = a.vol_total;
  __shared__ long long s_c[kBlock], s_d[kBlock], s_k[kBlock];
  long long mc = -1, md = 1, mk = 0;
  for (int i = threadIdx.x; i < sg.n_elem; i += kBlock) {
    const long long cut = a.scut[off + i] - bc;
    const long long vol = a.svol[off + i] - bv;
    const long long den = vol < vt - vol ? vol : vt - vol;
    if (den > 0 && b_cand_better(cut, den, i + 1, mc, md, mk)) { mc = cut; md = den; mk = i + 1; }
  }
  s_c[threadIdx.x] = mc; s_d[threadIdx.x] = md; s_k[threadIdx.x] = mk;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      const int u = threadIdx.x + o;
      if (b_cand_better(s_c[u], s_d[u], s_k[u], s_c[threadIdx.x], s_d[threadIdx.x],
                        s_k[threadIdx.x])) {
        s_c[threadIdx.x] = s_c[u];
        s_d[threadIdx.x] = s_d[u];
        s_k[threadIdx.x] = s_k[u];
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    Slot& S = a.slots[sg.slot];
    const long long k = s_k[0];
    S.kstar = k > 0 ? k : 0;
    S.best_cut = k > 0 ? s_c[0] : 0;
    S.best_den = k > 0 ? s_d[0] : 0;
    S.best_vol = k > 0 ? a.svol[off + k - 1] - bv : 0;
    S.phi = k > 0 ? (double)s_c[0] / (double)s_d[0] : 0.0;
    S.t_done = (long long)wall_clock64();
  }
}

// Dense layout: gather the nonzeros of r of every swept query by walking its
// touched list, and reset r (p and rank are reset by k_sw_reset).
__global__ __launch_bounds__(kBlock) void k_sw_finish(BatchArgs a) {
  BatchCtl* c = a.ctl;
  const int nseg = c->sw_nseg;
  const long long total = c->sw_touch_total;
  // per segment: start in the flattened touched space, its slot's touched
  // list and records, and where its r nonzeros go
  __shared__ long long s_toff[kMaxSlots];
  __shared__ const int32_t* s_tl[kMaxSlots];
  __shared__ VRec* s_tb[kMaxSlots];
  __shared__ int32_t* s_orid[kMaxSlots];
  __shared__ double* s_orval[kMaxSlots];
  __shared__ int s_cnt[kMaxSlots], s_base[kMaxSlots];
  __shared__ int s_lo;
  for (int j = threadIdx.x; j < nseg; j += kBlock) {
    const SweepSeg& sg = a.segs[j];
    const Slot& S = a.slots[sg.slot];
    s_toff[j] = sg.touch_off;
    s_tl[j] = S.touched;
    s_tb[j] = S.tab;
    s_orid[j] = sg.out_rid;
    s_orval[j] = sg.out_rval;
  }
  __syncthreads();
  // kScanBlock entries per workgroup step (a step spans at most nseg <=
  // kMaxSlots segments), four per thread with their loads issued together
  for (long long x0 = (long long)blockIdx.x * kScanBlock; x0 < total;
       x0 += (long long)gridDim.x * kScanBlock) {
    if (threadIdx.x == 0) s_lo = seg_of(s_toff, nseg, x0);
    for (int j = threadIdx.x; j < kMaxSlots; j += kBlock) s_cnt[j] = 0;
    __syncthreads();
    const int slo = s_lo;
    int sk[kScanItems];
    int32_t vk[kScanItems];
    double rv[kScanItems];
    int rk[kScanItems];
#pragma unroll
    for (int k = 0; k < kScanItems; k++) {
      const long long x = x0 + k * kBlock + threadIdx.x;
      sk[k] = -1;
      vk[k] = 0;
      if (x < total) {
        sk[k] = seg_of(s_toff, nseg, x);
        vk[k] = s_tl[sk[k]][x - s_toff[sk[k]]];
      }
    }
#pragma unroll
    for (int k = 0; k < kScanItems; k++) rv[k] = sk[k] >= 0 ? s_tb[sk[k]][vk[k]].r : 0.0;
#pragma unroll
    for (int k = 0; k < kScanItems; k++) {
      rk[k] = -1;
      if (sk[k] < 0) continue;
      s_tb[sk[k]][vk[k]].r = 0.0;
      if (rv[k] != 0.0) rk[k] = atomicAdd(&s_cnt[sk[k] - slo], 1);
    }
    __syncthreads();
    for (int j = threadIdx.x; slo + j < nseg && j < kMaxSlots; j += kBlock)
      if (s_cnt[j] > 0) s_base[j] = atomicAdd(&a.slots[a.segs[slo + j].slot].rnnz, s_cnt[j]);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kScanItems; k++) {
      if (rk[k] < 0) continue;
      const int sg = sk[k];
      const long long pos = (long long)s_base[sg - slo] + rk[k];
      const long long len = (sg + 1 < nseg ? s_toff[sg + 1] : total) - s_toff[sg];
      if (pos >= len) c->fault = 1;
      else if (s_orid[sg]) { s_orid[sg][pos] = vk[k]; s_orval[sg][pos] = rv[k]; }
    }
    __syncthreads();
  }
}

// Compact layout: gather the nonzeros of r of every swept query by scanning
// its table (the block returns to the arena afterwards, so nothing is
// reset).  Table capacities are multiples of kScanBlock records, so every
// kScanBlock-record chunk of the concatenated tables lies in one table.
// Each wave takes such a chunk (16 records per lane, in four rounds of
// coalesced loads), counts its nonzeros with ballots and reserves their
// output positions with one atomic on the slot's count; without an r output
// (PLC_QF_NO_RESIDUAL) it only counts.
__global__ __launch_bounds__(kBlock) void k_sw_gather(BatchArgs a) {
  BatchCtl* c = a.ctl;
  const int nseg = c->sw_nseg;
  constexpr int kPer = kScanBlock / 64;  // records per lane
  const long long nchunk = c->sw_touch_total / kScanBlock;
  __shared__ long long s_toff[kMaxSlots];
  for (int j = threadIdx.x; j < nseg; j += kBlock) s_toff[j] = a.segs[j].touch_off;
  __syncthreads();
  const long long nw = (long long)gridDim.x * (kBlock / 64);
  for (long long ch = (long long)blockIdx.x * (kBlock / 64) + PLC_WID; ch < nchunk; ch += nw) {
    const long long x0 = ch * kScanBlock;
    const int sgi = seg_of(s_toff, nseg, x0);
    const SweepSeg& sg = a.segs[sgi];
    Slot& S = a.slots[sg.slot];
    const VRec* tab = S.tab + (x0 - s_toff[sgi]);
    int32_t vk[kPer];
    double rk[kPer];
    int tot = 0;
#pragma unroll
    for (int k = 0; k < kPer; k++) {
      const VRec rec = tab[k * 64 + PLC_LANE];
      vk[k] = rec.deg;
      rk[k] = rec.deg != kEmptyKey ? rec.r : 0.0;
      tot += __popcll(__ballot(rk[k] != 0.0));
    }
    if (tot == 0) continue;
    int base = 0;
    if (PLC_LANE == 0) base = atomicAdd(&S.rnnz, tot);
    if (!sg.out_rid) continue;
    base = __shfl(base, 0);
#pragma unroll
    for (int k = 0; k < kPer; k++) {
      const unsigned long long m = __ballot(rk[k] != 0.0);
      if (rk[k] != 0.0) {
        const long long pos = (long long)base + __popcll(m & lanemask_lt());
        if (pos >= S.touched_cnt) c->fault = 1;
        else { sg.out_rid[pos] = vk[k]; sg.out_rval[pos] = rk[k]; }
      }
      base += __popcll(m);
    }
  }
}

// Dense layout: reset p and the sweep rank of every swept support vertex
// (after the boundary counts and the argmin no longer need them).
__global__ __launch_bounds__(kBlock) void k_sw_reset(BatchArgs a) {
  BatchCtl* c = a.ctl;
  const long long total = c->sw_total;
  const SortElem* el = a.sbuf[c->sort_flip & 1];
  for (long long k = (long long)blockIdx.x * kBlock + threadIdx.x; k < total;
       k += (long long)gridDim.x * kBlock) {
    const SortElem e = el[k];
    const Slot& S = a.slots[a.segs[e.seg].slot];
    S.tab[e.id].rank = a.hotcode[e.id];
    S.tp[e.id] = 0.0;
  }
}

// ---------------------------------------------------------------- launchers

hipError_t launch_batch_init(hipStream_t s, const BatchArgs& a) {
  int grid = (int)((a.n + kBlock - 1) / kBlock);
  if (grid > 8192) grid = 8192;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(k_b_init, dim3(grid), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_gdh_init(hipStream_t s, const BatchArgs& a, int2* gdh) {
  int grid = (int)((a.n + kBlock - 1) / kBlock);
  if (grid > 8192) grid = 8192;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(k_gdh_init, dim3(grid), dim3(kBlock), 0, s, a, gdh);
  return hipGetLastError();
}

hipError_t launch_batch_admit(hipStream_t s, const BatchArgs& a, const Admit* adm, int count,
                              bool compact) {
  if (count <= 0) return hipSuccess;
  if (compact)
    hipLaunchKernelGGL(k_b_admit<CompactState>, dim3(1), dim3(256), 0, s, a, adm, count);
  else
    hipLaunchKernelGGL(k_b_admit<DenseState>, dim3(1), dim3(256), 0, s, a, adm, count);
  return hipGetLastError();
}

hipError_t launch_batch_plan_self(hipStream_t s, const BatchArgs& a, int grid_self, bool compact) {
  hipLaunchKernelGGL(k_b_plan, dim3(1), dim3(kMaxSlots), 0, s, a);
  if (compact)
    hipLaunchKernelGGL(k_b_self<CompactState>, dim3(grid_self), dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL(k_b_self<DenseState>, dim3(grid_self), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

template <class St>
static void scatter_launch(hipStream_t s, const BatchArgs& a, int grid, hipEvent_t t0,
                           hipEvent_t t1) {
  if (t0)
    hipExtLaunchKernelGGL(k_b_scatter<St>, dim3(grid), dim3(kBlock), 0, s, t0, t1, 0, a);
  else
    hipLaunchKernelGGL(k_b_scatter<St>, dim3(grid), dim3(kBlock), 0, s, a);
}

hipError_t launch_batch_scatter(hipStream_t s, const BatchArgs& a, int grid_scatter,
                                bool compact, hipEvent_t t0, hipEvent_t t1) {
  if (compact)
    scatter_launch<CompactState>(s, a, grid_scatter, t0, t1);
  else
    scatter_launch<DenseState>(s, a, grid_scatter, t0, t1);
  return hipGetLastError();
}

hipError_t launch_batch_round_end(hipStream_t s, const BatchArgs& a) {
  hipLaunchKernelGGL(k_b_round_end, dim3(1), dim3(kMaxSlots), 0, s, a);
  return hipGetLastError();
}

template <class St>
static hipError_t sweep_kernels(hipStream_t s, const BatchArgs& a, int nseg, int64_t max_elems,
                                int grid) {
  hipLaunchKernelGGL(k_sw_keys<St>, dim3(grid), dim3(kBlock), 0, s, a);
  SortArgs sa;
  sa.buf[0] = a.sbuf[0];
  sa.buf[1] = a.sbuf[1];
  sa.count = &a.ctl->sw_total;
  sa.flip = &a.ctl->sort_flip;
  sa.done = &a.ctl->done[0];
  sa.active = nullptr;
  sa.active_value = 0;
  sa.rank = nullptr;
  hipError_t e = launch_sort(s, sa, max_elems, grid);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sw_rank<St>, dim3(grid), dim3(kBlock), 0, s, a);
  hipLaunchKernelGGL(k_sw_scan<false>, dim3(grid), dim3(kBlock), 0, s, a);
  // the count, the gathers and the reset walk many short, latency-bound
  // steps: a larger grid keeps more of them in flight
  hipLaunchKernelGGL(k_sw_count<St>, dim3(4 * grid), dim3(kBlock), 0, s, a);
  hipLaunchKernelGGL(k_sw_scan<true>, dim3(grid), dim3(kBlock), 0, s, a);
  hipLaunchKernelGGL(k_sw_argmin, dim3(nseg), dim3(kBlock), 0, s, a);
  if (St::kCompact) {
    hipLaunchKernelGGL(k_sw_gather, dim3(4 * grid), dim3(kBlock), 0, s, a);
  } else {
    hipLaunchKernelGGL(k_sw_finish, dim3(4 * grid), dim3(kBlock), 0, s, a);
    hipLaunchKernelGGL(k_sw_reset, dim3(4 * grid), dim3(kBlock), 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_batch_sweep(hipStream_t s, const BatchArgs& a, int nseg, int64_t max_elems,
                              int grid, bool compact) {
  if (nseg <= 0) return hipSuccess;
  return compact ? sweep_kernels<CompactState>(s, a, nseg, max_elems, grid)
                 : sweep_kernels<DenseState>(s, a, nseg, max_elems, grid);
}

hipError_t launch_table_clear(hipStream_t s, const ClearJob* jobs, int count, long long total,
                              int grid) {
  if (count <= 0 || count > kMaxClearJobs) return count <= 0 ? hipSuccess : hipErrorInvalidValue;
  hipLaunchKernelGGL(k_c_clear, dim3(grid), dim3(kBlock), 0, s, jobs, count, total);
  return hipGetLastError();
}

hipError_t launch_table_grow(hipStream_t s, const BatchArgs& a, const Grow* gr, int count,
                             long long total_old, long long total_list, int grid) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_c_rehash, dim3(grid), dim3(kBlock), 0, s, a, gr, count, total_old);
  hipLaunchKernelGGL(k_c_move_lists, dim3(grid), dim3(kBlock), 0, s, a, gr, count, total_list);
  hipLaunchKernelGGL(k_c_commit, dim3(1), dim3(256), 0, s, a, gr, count);
  return hipGetLastError();
}

hipError_t launch_slot_hold(hipStream_t s, const BatchArgs& a, const int32_t* holds, int count) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_slot_hold, dim3(1), dim3(256), 0, s, a, holds, count);
  return hipGetLastError();
}

}  // namespace plc
