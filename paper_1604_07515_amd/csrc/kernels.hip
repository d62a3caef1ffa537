// kernels.hip -- gfx950 kernels of the plain (one query at a time) path:
// round-synchronous PR-Nibble (Sec. 3.3) and the parallel sweep cut
// (Sec. 3.1, Theorem 1).
//
// Round t of PR-Nibble is three launches:
//   k_self    vertexMap(Frontier, UpdateSelf): snapshot rho_v = r[v], update
//             p[v] and r[v], compute the per-entry coefficient cn*rho/d(v), and
//             (single-pass decoupled look-back scan) the start of each entry's
//             edges in the round's flattened edge sequence; entries record the
//             entry index of every 1024-edge tile they start.
//   k_scatter edgeMap(G, Frontier, UpdateNgh): one workgroup per edge tile
//             (persistent grid), entries staged in LDS, coalesced neighbour
//             reads, FP64 atomic add into r[w].  The filter of the paper is
//             folded in: r only grows during a scatter, so w joins the next
//             frontier exactly when one atomic's (old, old + c) pair straddles
//             eps*d(w); that atomic appends w.  On rounds of at least the
//             binning threshold it is pass A of the binned scatter instead
//             (pairs sorted into destination bins), and on rounds over half
//             the arcs it only stamps the frontier's coefficients.
//   k_bin_apply  pass B of a binned round (LDS sums per bin, one update per
//             touched destination) or the pull form; it exits at once on the
//             other rounds.  The host leaves it out where no round can bin,
//             and in a query's first chunk behind the launches where recent
//             queries had no round large enough (k_scatter then takes the
//             atomic form whatever the round's size).
// A frontier of at most one scan block is handled by k_self alone: its last
// workgroup to arrive runs such rounds back to back (self step, scan, edge
// scatter, round close) until the frontier grows, empties or a round has
// too many edges for one workgroup; k_scatter then pushes only rounds whose
// entries were built in memory.
// Kernels read the round number and frontier size from the device control
// block and return at once when the query has finished, so rounds (and the
// sweep, guarded the same way) can be queued ahead of the host's
// termination check.
//
// The sweep: k_sweep_keys, the sort (sort.hip; its block-sort launch also
// gathers the nonzeros of r over the touched list and resets r, on the
// workgroups that hold no tile), k_vol_scan, k_cut_count, k_cut_scan (which
// also resets p and the ranks) and a one-workgroup k_sweep_finish.
//
// Arithmetic matches the paper's updates evaluated in a fixed way: the
// constants cs, cn, keep are rounded once, p[v] + cs*rho, keep*rho and
// (cn*rho)/d are each rounded separately (the library is built with
// -ffp-contract=off), and the threshold is eps*(double)d.  Only the order of
// the atomic additions into r differs from a sequential evaluation.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_util.h"
#include "plc_device.h"
#include "sort.h"

namespace plc {

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
    a.hk_r1[v] = 0.0;
    if (a.pull) a.pull[v] = PullRec{0.0, 0u, 0};
  }
  if (a.pull_epoch && blockIdx.x == 0 && threadIdx.x == 0) *a.pull_epoch = 1u;
}

__device__ __forceinline__ void reset_round_book(Ctl* c) {
  c->init_held = 0;
  c->selfed = -1;
  c->steps = 0;
  c->loop_rounds = 0;
  c->loop_pushes = 0;
  c->loop_edges = 0;
  c->bin_rounds = 0;
  c->bin_pairs = 0u;
  c->pull_rounds = 0;
  c->bin_edges = 0;
  c->t_start = (long long)wall_clock64();
  c->t_end = 0;
}

// Seed initialisation (Fig. alg:pr-nibble: r = {(x,1)}, Frontier = {x}).
__device__ void query_init_body(const PlainArgs& a, int32_t seed, int32_t rule, double alpha,
                                double eps, int32_t max_rounds, double beta) {
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
  c->beta = beta;
  c->beta_nf = 0;
  c->beta_k = 0;
  c->round = 0;
  c->cnt[0] = 1;
  c->cnt[1] = 0;
  c->ntiles = 0;
  c->etotal = 0;
  c->pushes = 0;
  c->edges = 0;
  c->support_cnt = 0;
  c->touched_cnt = 1;
  c->fault = 0;
  c->limited = 0;
  c->N = 0;
  c->sort_flip = 0;
  c->rnnz = 0;
  c->vol_total = a.vol_total;
  c->best_cut = 0;
  c->best_vol = 0;
  c->best_den = 0;
  c->kstar = 0;
  c->phi = 0.0;
  reset_round_book(c);
  a.fbuf0[0] = seed;
  a.touched[0] = seed;
  a.vr[seed].r = 1.0;
  c->status = ST_PUSH;
}

__global__ void k_query_init(PlainArgs a, int32_t seed, int32_t rule, double alpha, double eps,
                             int32_t max_rounds, double beta) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  query_init_body(a, seed, rule, alpha, eps, max_rounds, beta);
}

// The same, only after a swept query (or none since the graph was loaded);
// otherwise the previous query's state is left as it is.
__global__ void k_query_init_guarded(PlainArgs a, int32_t seed, int32_t rule, double alpha,
                                     double eps, int32_t max_rounds) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  Ctl* c = a.ctl;
  if (c->status != ST_SWEPT && c->status != ST_IDLE) {
    c->init_held = 1;
    return;
  }
  query_init_body(a, seed, rule, alpha, eps, max_rounds, 1.0);
}

// Seed-set initialisation (Sec. 3: a set S of seeds): the host has placed
// the distinct seeds in the first frontier; each gets r = 1/|S| and is
// listed as touched.  Block 0 also sets up the control block.
__global__ void k_query_init_set(PlainArgs a, int32_t nseeds, int32_t rule, double alpha,
                                 double eps, int32_t max_rounds) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
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
    c->seed = a.fbuf0[0];
    c->rule = rule;
    c->max_rounds = max_rounds;
    c->beta = 1.0;
    c->beta_nf = 0;
    c->beta_k = 0;
    c->round = 0;
    c->cnt[0] = nseeds;
    c->cnt[1] = 0;
    c->ntiles = 0;
    c->etotal = 0;
    c->pushes = 0;
    c->edges = 0;
    c->support_cnt = 0;
    c->touched_cnt = nseeds;
    c->fault = 0;
    c->limited = 0;
    c->N = 0;
    c->sort_flip = 0;
    c->rnnz = 0;
    c->vol_total = a.vol_total;
    c->best_cut = 0;
    c->best_vol = 0;
    c->best_den = 0;
    c->kstar = 0;
    c->phi = 0.0;
    reset_round_book(c);
    c->status = ST_PUSH;
  }
  const double share = 1.0 / (double)nseeds;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nseeds; i += gridDim.x * blockDim.x) {
    const int32_t v = a.fbuf0[i];
    a.touched[i] = v;
    a.vr[v].r = share;
  }
}

// ---------------------------------------------------------------- round

__device__ __forceinline__ bool push_active(const Ctl* c, int64_t ncap, int* t_out, int* nf_out) {
  if (c->status != ST_PUSH) return false;
  int t = c->round;
  int nf = c->cnt[t & 1];
  if (nf <= 0) return false;
  if ((int64_t)nf > ncap) nf = (int)ncap;
  *t_out = t;
  *nf_out = nf;
  return true;
}

// Entry i covers edges [s, s + d) of the round; record it as the first entry
// of every tile that starts inside that range.
__device__ __forceinline__ void mark_tiles(int32_t* tile_start, int64_t cap, long long s,
                                           long long d, int i, int* fault) {
  long long t0 = (s + kEdgeTile - 1) / kEdgeTile;
  long long t1 = (s + d - 1) / kEdgeTile;
  if (t1 >= cap) { *fault = 1; t1 = cap - 1; }
  for (long long tt = t0; tt <= t1; tt++) tile_start[tt] = i;
}

// Round rules sharing the round kernels.
enum : int { kModePR = 0, kModeHK = 1, kModeNB = 2 };

// HK-PR residual (Nibble vector) of vertex v at level (iteration) k: even
// levels in the state record, odd levels in hk_r1.
__device__ __forceinline__ double* hk_res(const PlainArgs& a, int k, int32_t v) {
  return (k & 1) ? &a.hk_r1[v] : &a.vr[v].r;
}

// vertexMap(Frontier, UpdateSelf) + degree scan of the frontier.
//   PR-Nibble (Figs. alg:pr-nibble / alg:pr-nibble2): p += cs rho, r =
//     keep rho (-0.0 under the optimized rule), coefficient cn rho / d.
//   HK-PR level j (Fig. alg:hkpr): p += rho; coefficient t rho / ((j+1) d),
//     or rho / d on the last level; first, the residuals of level j - 1
//     (the array level j + 1 fills) are cleared over the vertices that
//     level touched.
//   Nibble step j -> j+1 (Fig. alg:nibble): coefficient rho / (2 d), and
//     rho / 2 kept per entry for the scatter, which adds it to the vertex's
//     own next value; the same clearing as HK-PR.
template <int MODE>
__device__ __forceinline__ void self_body(const PlainArgs& a, int slot) {
  constexpr bool HK = MODE == kModeHK;
  constexpr bool LEVELS = MODE != kModePR;
  Ctl* c = a.ctl;
  int t, nf;
  if (!push_active(c, a.n, &t, &nf)) return;
  if (LEVELS) {
    if (t >= (HK ? c->hk_N : c->max_rounds)) return;  // (the host queues no more)
    if (t >= 1) {
      const int lp = (t + 2) % 3;
      const int np = c->hk_tlc[lp];
      const int32_t* Lp = a.hk_tl[lp];
      for (int i = blockIdx.x * kBlock + threadIdx.x; i < np; i += gridDim.x * kBlock)
        *hk_res(a, t + 1, Lp[i]) = 0.0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) c->hk_tlc[(t + 1) % 3] = 0;
  } else if (t >= c->max_rounds) {
    if (blockIdx.x == 0 && threadIdx.x == 0) { c->limited = 1; c->status = ST_LIMIT; }
    return;
  }
  __shared__ long long sh[kBlock / 64 + 1];
  __shared__ long long s_excl;
  __shared__ int s_tk[2];
  __shared__ int32_t s_sup[kScanBlock];
  __shared__ int32_t s_stay[LEVELS ? 1 : kScanBlock];
  __shared__ int s_nsup, s_nstay, s_base;
  ScanSite* site = &c->scan[SCAN_FRONTIER];
  scan_clear_prev(site, a.desc[SCAN_FRONTIER], a.desc_cap);
  unsigned long long* desc = a.desc[SCAN_FRONTIER] + (size_t)site->parity * a.desc_cap;
  const int32_t* F = (t & 1) ? a.fbuf1 : a.fbuf0;
  int32_t* Fn = (t & 1) ? a.fbuf0 : a.fbuf1;
  int32_t* cntn = &c->cnt[(t + 1) & 1];
  const double cs = c->cs, cn = c->cn, keep = c->keep, eps = c->eps;
  const bool opt = LEVELS || c->opt_rule != 0;
  const bool hk_last = HK && t + 1 == c->hk_N;
  const double hk_t = HK ? c->hk_t : 0.0;
  const int nblk = (nf + kScanBlock - 1) / kScanBlock;
  // a frontier of one scan block is handled by workgroup 0 alone, with no
  // ticket and no look-back (its exclusive prefix is 0; no descriptor is
  // published and the scan site is left as it was)
  const bool solo = nblk == 1;
  if (solo && blockIdx.x != 0) return;
  if (threadIdx.x == 0) { s_nsup = 0; s_nstay = 0; }
  __syncthreads();

  for (int pass = 0;; pass++) {
    int b;
    if (solo) {
      if (pass > 0) break;
      b = 0;
    } else {
      bool last;
      b = scan_ticket(site, nblk, s_tk, &last);
      if (b >= nblk) break;
    }
    // each thread takes kScanItems consecutive entries: one workgroup scan
    // of the per-thread sums, then a serial prefix inside the thread
    const int i0 = b * kScanBlock + (int)threadIdx.x * kScanItems;
    int32_t dk[kScanItems];
    long long dsum = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; k++) {
      const int i = i0 + k;
      int32_t d = 0;
      int32_t v = 0;
      bool stay = false, sup = false;
      if (i < nf) {
        v = F[i];
        double rho;
        if (LEVELS) {
          rho = *hk_res(a, t, v);
          d = a.vr[v].deg;
        } else {
          VRec rec = a.vr[v];
          rho = rec.r;
          d = rec.deg;
        }
        double pold = MODE == kModeNB ? 1.0 : a.p[v];
        if (MODE == kModeNB) {
          a.coef[i] = rho / (2.0 * (double)d);
          a.sp[i] = rho / 2.0;
        } else if (HK) {
          a.p[v] = pold + rho;
          a.coef[i] = hk_last ? rho / (double)d : (hk_t * rho) / ((double)(t + 1) * (double)d);
        } else {
          a.p[v] = pold + cs * rho;
          double nr = opt ? -0.0 : keep * rho;
          a.vr[v].r = nr;
          a.coef[i] = (cn * rho) / (double)d;
          stay = !opt && nr >= eps * (double)d;
        }
        a.rowp[i] = a.off[v];
        sup = pold == 0.0;
      }
      wave_append(stay, v, s_stay, &s_nstay);
      wave_append(sup, v, s_sup, &s_nsup);
      dk[k] = d;
      dsum += d;
    }
    long long agg;
    const long long ex = block_excl_scan<kBlock>(dsum, &agg, sh);
    if (solo) {
      if (threadIdx.x == 0) s_excl = 0;
    } else if (threadIdx.x < 64) {
      const long long ex0 = scan_lookback(desc, b, agg, &c->fault);
      if (threadIdx.x == 0) s_excl = ex0;
    }
    __syncthreads();
    long long s = s_excl + ex;
#pragma unroll
    for (int k = 0; k < kScanItems; k++) {
      const int i = i0 + k;
      if (i < nf) {
        a.estart[i] = s;
        mark_tiles(a.tile_start, a.tile_cap, s, dk[k], i, &c->fault);
      }
      s += dk[k];
    }
    if (b == nblk - 1 && threadIdx.x == 0) {
      const long long tot = s_excl + agg;
      c->etotal = tot;
      c->ntiles = (int)((tot + kEdgeTile - 1) / kEdgeTile);
      c->selfed = t;
      c->steps += 1;
      if (slot >= 0) a.work_log[2 * slot] = 1;
    }
    if (MODE != kModeNB)
      block_flush(&c->support_cnt, a.support, a.n, s_sup, &s_nsup, &s_base, &c->fault);
    if (!opt) block_flush(cntn, Fn, a.n, s_stay, &s_nstay, &s_base, &c->fault);
  }
}

// Threshold decision for one addition of c to r[w] that returned `old`
// (lanes without an addition pass valid = false): crossing appends w to the
// next frontier, first touch to the touched list (wave-ballot appends).
__device__ __forceinline__ void decide(bool valid, double old, double c, double thr, int32_t w,
                                       int32_t* s_fn, int* s_nfn, int32_t* s_tv, int* s_ntv) {
  wave_append(valid && old < thr && old + c >= thr, w, s_fn, s_nfn);
  wave_append(valid && __double_as_longlong(old) == 0, w, s_tv, s_ntv);
}

template <typename T>
__device__ __forceinline__ T ld_agent(T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_agent(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Append the n values of buf at dst[base..] (capacity cap) and, where
// mirror is set, at mirror[base..] below kScanBlock.  The caller's
// workgroup is the only writer of the list, so the base is its own count.
__device__ __forceinline__ void local_append(int32_t* dst, int64_t cap, int32_t* mirror,
                                             const int32_t* buf, int n, int base, int* fault) {
  for (int j = threadIdx.x; j < n; j += kBlock) {
    const long long slot = (long long)base + j;
    if (slot < cap) dst[slot] = buf[j]; else *fault = 1;
    if (mirror && slot < kScanBlock) mirror[slot] = buf[j];
  }
}

// Rounds with small frontiers (Figs. alg:pr-nibble / alg:pr-nibble2, the
// same updates and arithmetic as k_self + k_scatter), run back to back by
// workgroup 0 alone: the frontier (at most kScanBlock vertices) and its
// entries stay in LDS, list lengths are kept locally, and only the FP64
// additions into r go to memory as device-scope atomics.  r of the frontier
// is read and written with device-scope atomic accesses too, so that within
// the launch they are ordered with those additions.  It stops when the
// frontier empties or outgrows a scan block, when a round has more than
// kLoopEdges edges (that round's entries are then built in memory for the
// next scatter launch, exactly as k_self builds them), at the round limit, or
// after kLoopMaxRounds rounds.
__device__ void loop_rounds(const PlainArgs& a, int slot, int t, int nf) {
  Ctl* c = a.ctl;
  __shared__ int32_t s_F[2][kScanBlock];  // this round's and the next round's frontier
  __shared__ int32_t s_est[kScanBlock];   // entry i: first edge in the round's edge sequence
  __shared__ int64_t s_row[kScanBlock];   //          off[v]
  __shared__ double s_cf[kScanBlock];     //          cn rho / d(v)
  __shared__ int32_t s_fn[kLoopPass];     // crossings of one pass
  __shared__ int32_t s_tv[kLoopPass];     // first touches of one pass
  __shared__ int32_t s_sup[kScanBlock];
  __shared__ int32_t s_stay[kScanBlock];
  __shared__ long long sh[kBlock / 64 + 1];
  __shared__ int s_nfn, s_ntv, s_nsup, s_nstay;
  if (threadIdx.x == 0) {
    s_nfn = 0;
    s_ntv = 0;
    s_nsup = 0;
    s_nstay = 0;
  }
  __syncthreads();
  const double cs = c->cs, cn = c->cn, keep = c->keep, eps = c->eps;
  const bool opt = c->opt_rule != 0;
  const int max_rounds = c->max_rounds;
  const int64_t cap = a.n;
  int tcnt = c->touched_cnt, scnt = c->support_cnt;
  long long pushes = 0, edges = 0, E = 0;
  int nnext = 0, cur = 0, rounds = 0;
  bool selfed = false;
  for (int it = 0;; it++) {
    const int32_t* F = it > 0 ? s_F[cur] : (t & 1) ? a.fbuf1 : a.fbuf0;
    int32_t* Fn = (t & 1) ? a.fbuf0 : a.fbuf1;
    // vertexMap(Frontier, UpdateSelf) and the degree scan
    const int i0 = (int)threadIdx.x * kScanItems;
    int32_t dk[kScanItems];
    double ck[kScanItems];
    int64_t rk[kScanItems];
    long long dsum = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; k++) {
      const int i = i0 + k;
      int32_t d = 0;
      int32_t v = 0;
      bool stay = false, sup = false;
      ck[k] = 0.0;
      rk[k] = 0;
      if (i < nf) {
        v = F[i];
        d = a.vr[v].deg;
        double* rp = &a.vr[v].r;
        const double rho = ld_agent(rp);
        const double pold = a.p[v];
        a.p[v] = pold + cs * rho;
        const double nr = opt ? -0.0 : keep * rho;
        st_agent(rp, nr);
        ck[k] = (cn * rho) / (double)d;
        rk[k] = a.off[v];
        stay = !opt && nr >= eps * (double)d;
        sup = pold == 0.0;
      }
      wave_append(stay, v, s_stay, &s_nstay);
      wave_append(sup, v, s_sup, &s_nsup);
      dk[k] = d;
      dsum += d;
    }
    long long agg;
    const long long ex = block_excl_scan<kBlock>(dsum, &agg, sh);
    E = agg;
    const int nstay = s_nstay, nsup = s_nsup;
    local_append(a.support, cap, nullptr, s_sup, nsup, scnt, &c->fault);
    local_append(Fn, cap, s_F[cur ^ 1], s_stay, nstay, 0, &c->fault);
    scnt += nsup;
    nnext = nstay;
    if (E > kLoopEdges) {
      // too large for one workgroup: entries in memory for the scatter launch
      long long s = ex;
#pragma unroll
      for (int k = 0; k < kScanItems; k++) {
        const int i = i0 + k;
        if (i < nf) {
          a.estart[i] = s;
          a.rowp[i] = rk[k];
          a.coef[i] = ck[k];
          mark_tiles(a.tile_start, a.tile_cap, s, dk[k], i, &c->fault);
        }
        s += dk[k];
      }
      selfed = true;
      break;
    }
    {
      long long s = ex;
#pragma unroll
      for (int k = 0; k < kScanItems; k++) {
        const int i = i0 + k;
        if (i < nf) {
          s_est[i] = (int32_t)s;
          s_row[i] = rk[k];
          s_cf[i] = ck[k];
        }
        s += dk[k];
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) { s_nstay = 0; s_nsup = 0; }
    // edgeMap(G, Frontier, UpdateNgh), kLoopPass edges per pass
    constexpr int kPer = kLoopPass / kBlock;
    for (long long base = 0; base < E; base += kLoopPass) {
      int32_t w[kPer];
      double cf[kPer];
#pragma unroll
      for (int k = 0; k < kPer; k++) {
        const int rel = (int)base + k * kBlock + (int)threadIdx.x;
        w[k] = -1;
        cf[k] = 0.0;
        if (rel < E) {
          int lo = 0, hi = nf - 1;
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_est[mid] <= rel) lo = mid; else hi = mid - 1;
          }
          w[k] = a.nbr[s_row[lo] + (rel - s_est[lo])];
          cf[k] = s_cf[lo];
        }
      }
      int32_t dw[kPer];
#pragma unroll
      for (int k = 0; k < kPer; k++) dw[k] = w[k] >= 0 ? a.vr[w[k]].deg : 0;
      double old[kPer];
#pragma unroll
      for (int k = 0; k < kPer; k++) old[k] = w[k] >= 0 ? unsafeAtomicAdd(&a.vr[w[k]].r, cf[k]) : 0.0;
#pragma unroll
      for (int k = 0; k < kPer; k++)
        decide(w[k] >= 0, old[k], cf[k], eps * (double)dw[k], w[k], s_fn, &s_nfn, s_tv, &s_ntv);
      __syncthreads();
      const int nfn = s_nfn, ntv = s_ntv;
      local_append(Fn, cap, s_F[cur ^ 1], s_fn, nfn, nnext, &c->fault);
      local_append(a.touched, cap, nullptr, s_tv, ntv, tcnt, &c->fault);
      nnext += nfn;
      tcnt += ntv;
      __syncthreads();
      if (threadIdx.x == 0) { s_nfn = 0; s_ntv = 0; }
      __syncthreads();
    }
    // the round is over (the barrier orders this round's LDS appends and
    // count resets before the next round's, also when E is 0)
    __syncthreads();
    pushes += nf;
    edges += E;
    rounds += 1;
    t += 1;
    nf = nnext;
    nnext = 0;
    cur ^= 1;
    if (nf == 0 || nf > kScanBlock || t >= max_rounds || it + 1 >= kLoopMaxRounds) break;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    c->touched_cnt = tcnt;
    c->support_cnt = scnt;
    c->pushes += pushes;
    c->edges += edges;
    c->loop_rounds += rounds;
    c->loop_pushes += pushes;
    c->loop_edges += edges;
    c->steps += 1;
    if (selfed) {
      c->etotal = E;
      c->ntiles = (int)((E + kEdgeTile - 1) / kEdgeTile);
    }
    c->cnt[(t + 1) & 1] = nnext;  // stays of a round left to the scatter launch
    c->cnt[t & 1] = nf;
    c->selfed = selfed ? t : -1;
    c->round = t;
    if (slot >= 0) a.work_log[2 * slot] = 1;
  }
}

// The self launch of PR-Nibble.  A frontier of at most one scan block goes
// to loop_rounds, run by the workgroup that arrives last: the loop rewrites
// the control block, and by then every other workgroup has read the state
// it decided on (the same as the loop's) and left.
__global__ __launch_bounds__(kBlock) void k_self(PlainArgs a, int slot) {
  Ctl* c = a.ctl;
  const int32_t st = c->status;
  const int32_t t = c->round;
  int32_t nf = c->cnt[t & 1];
  if ((int64_t)nf > a.n) nf = (int32_t)a.n;
  if (st == ST_PUSH && nf > 0 && nf <= kScanBlock && t < c->max_rounds && c->beta >= 1.0) {
    __shared__ int s_last;
    if (last_block(&c->done[DONE_SELF], &s_last, false)) loop_rounds(a, slot, t, nf);
    return;
  }
  self_body<kModePR>(a, slot);
}
__global__ __launch_bounds__(kBlock) void k_hk_self(PlainArgs a) { self_body<kModeHK>(a, -1); }
__global__ __launch_bounds__(kBlock) void k_nb_self(PlainArgs a) { self_body<kModeNB>(a, -1); }

// ------------------------------------------------- binned edge scatter
//
// For a large round, one FP64 atomic per edge is bound by contention on the
// lines of high-degree destinations.  The binned form of the same edgeMap
// (Figs. alg:pr-nibble / alg:pr-nibble2, UpdateNgh) groups the round's
// (neighbour, entry) pairs by destination bin, adds each bin's contributions
// in LDS and applies one update per distinct destination:
//   pass A (in k_scatter): every chunk of kBinChunk consecutive edges is
//     sorted by bin in place (a counting sort: LDS histogram with ranks, one
//     workgroup scan) into bin_pairs[chunk], and the start of every bin's run
//     in the chunk goes to bin_T (bin-major).  No global atomics.
//   pass B (k_bin_apply): one item per bin, or per slice of the chunks for a
//     bin whose expected share of the round's edges exceeds kBinQ.  The item
//     gathers its runs, adds every contribution into an LDS array over the
//     bin's vertex range (first touches listed), then updates each touched
//     destination once: a plain read-modify-write of r when the item owns the
//     whole bin (no other workgroup writes those records in this launch), a
//     device-scope atomic when the bin is split.  The filter is folded in as
//     in the atomic scatter: r only grows, so w joins the next frontier when
//     its single update (old, old + sum) straddles eps d(w).
// The sum of a destination's contributions is formed in another order than
// in a sequence of atomics; that is the only difference.

// LDS of the scatter launch: the atomic scatter's arrays or pass A's, which
// never run in the same launch.
struct ScatterLds {
  int32_t start[kEdgeTile + 1];
  int64_t row[kEdgeTile + 1];
  double coef[kEdgeTile + 1];
  int32_t fn[kEdgeTile];
  int32_t tv[kEdgeTile];
  int nfn, ntv, base, last;
};
struct BinSortLds {
  int32_t start[kEdgeTile + 1];
  int64_t row[kEdgeTile + 1];
  int hist[kMaxBins + kBlock];
  int sh[kBlock / 64 + 1];
};
union ScatterShared {
  ScatterLds at;
  BinSortLds bs;
};

__device__ __forceinline__ bool pull_round(const PlainArgs& a, long long E) {
  return a.pull != nullptr && a.nbins > 0 && E >= a.bin_emin && E >= a.pull_emin;
}
__device__ __forceinline__ bool bin_round(const PlainArgs& a, long long E) {
  return a.nbins > 0 && E >= a.bin_emin && E <= (long long)a.bin_cmax * kBinChunk &&
         !pull_round(a, E);
}

// Exclusive scan over the workgroup of one int per thread; sh holds
// kBlock/64 + 1 slots.  Every thread must call it.
__device__ __forceinline__ int block_excl_scan_int(int x, int* total, int* sh) {
  int inc = x;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(inc, o);
    if ((int)PLC_LANE >= o) inc += y;
  }
  if (PLC_LANE == 63) sh[PLC_WID] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int w = 0; w < kBlock / 64; w++) {
      const int v = sh[w];
      sh[w] = acc;
      acc += v;
    }
    sh[kBlock / 64] = acc;
  }
  __syncthreads();
  const int ex = inc - x + sh[PLC_WID];
  *total = sh[kBlock / 64];
  __syncthreads();
  return ex;
}

// Pass A, run by the scatter launch in place of the atomic scatter.
// Workgroups take chunks in turn; a chunk's kBinChunkTiles tiles are staged
// one at a time (entries in LDS, a binary search per edge as in the atomic
// scatter).  The chunk's pairs stay in registers until the histogram scan.
__device__ void bin_sort_chunks(const PlainArgs& a, int nf, BinSortLds& L) {
  Ctl* c = a.ctl;
  int32_t* const s_start = L.start;
  int64_t* const s_row = L.row;
  int* const s_hist = L.hist;
  int* const sh = L.sh;
  constexpr int kPer = kBinChunk / kBlock;           // edges per thread per chunk
  constexpr int kBinsPT = kMaxBins / kBlock;         // bins per thread in the scan
  const int nb = a.nbins;
  const long long E = c->etotal;
  const int ntiles = (int64_t)c->ntiles > a.tile_cap ? (int)a.tile_cap : c->ntiles;
  const int C = (int)((E + kBinChunk - 1) / kBinChunk);
  for (int ch = blockIdx.x; ch < C; ch += gridDim.x) {
    for (int b = threadIdx.x; b < nb; b += kBlock) s_hist[b] = 0;
    __syncthreads();
    int32_t w[kPer], ie[kPer], bk[kPer];  // bk: bin << 16 | rank within the chunk's bin
#pragma unroll
    for (int tt = 0; tt < kBinChunkTiles; tt++) {
      const int tile = ch * kBinChunkTiles + tt;
      const long long e0 = (long long)tile * kEdgeTile;
      const long long e1 = e0 + kEdgeTile < E ? e0 + kEdgeTile : E;
      int cnt = 0, i0 = 0;
      if (tile < ntiles) {
        i0 = a.tile_start[tile];
        const int i1 = tile + 1 < ntiles ? a.tile_start[tile + 1] : nf - 1;
        cnt = i1 - i0 + 1;
        if (i0 < 0 || i1 < i0 || i1 >= nf || cnt > kEdgeTile + 1) {
          c->fault = 1;  // inconsistent tile map: the tile is skipped, the fault reported
          cnt = 0;
        }
        for (int j = threadIdx.x; j < cnt; j += kBlock) {
          s_start[j] = (int32_t)(a.estart[i0 + j] - e0);
          s_row[j] = a.rowp[i0 + j];
        }
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < kEdgesPerThread; k++) {
        const int rel = k * kBlock + (int)threadIdx.x;
        const int x = tt * kEdgesPerThread + k;
        w[x] = -1;
        ie[x] = 0;
        if (cnt > 0 && e0 + rel < e1) {
          int lo = 0, hi = cnt - 1;
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_start[mid] <= rel) lo = mid; else hi = mid - 1;
          }
          w[x] = a.nbr[s_row[lo] + (rel - s_start[lo])];
          ie[x] = i0 + lo;
        }
      }
#pragma unroll
      for (int k = 0; k < kEdgesPerThread; k++) {
        const int x = tt * kEdgesPerThread + k;
        bk[x] = 0;
        if (w[x] >= 0) {
          const int b = a.bin_of_blk[w[x] / kBinGran];
          bk[x] = (b << 16) | atomicAdd(&s_hist[b], 1);
        }
      }
      __syncthreads();  // before the next tile's entries are staged
    }
    // run starts: exclusive prefix of the histogram (kBinsPT bins per thread)
    int loc[kBinsPT];
    int tsum = 0;
#pragma unroll
    for (int k = 0; k < kBinsPT; k++) {
      const int b = (int)threadIdx.x * kBinsPT + k;
      loc[k] = b < nb ? s_hist[b] : 0;
      tsum += loc[k];
    }
    int total;
    int ex = block_excl_scan_int(tsum, &total, sh);
#pragma unroll
    for (int k = 0; k < kBinsPT; k++) {
      const int b = (int)threadIdx.x * kBinsPT + k;
      if (b <= nb) {
        s_hist[b] = ex;
        a.bin_T[(size_t)b * a.bin_cmax + ch] = ex;
      }
      ex += loc[k];
    }
    __syncthreads();
    int2* out = a.bin_pairs + (size_t)ch * kBinChunk;
#pragma unroll
    for (int x = 0; x < kPer; x++) {
      if (w[x] >= 0) out[s_hist[bk[x] >> 16] + (bk[x] & 0xffff)] = make_int2(w[x], ie[x]);
    }
    __syncthreads();
  }
}

// Pass B of a binned round, or the pull form of a round that covers at
// least half the graph's arcs, then the round's close.  Exits at once when
// the round was neither (k_scatter then closed it).
//   Pass B: each item gathers its bin's runs of (neighbour, entry) pairs
//   from pass A and adds the entries' coefficients into an LDS array over
//   the bin's vertices.
//   Pull: each item walks a slice of its bin's own vertices' arcs (CSR rows
//   in order) and adds the coefficient of every neighbour whose pull record
//   carries this round's epoch (the frontier), with no pairs and no pass A.
// Then every touched destination gets one update (plain when the item owns
// the whole bin, atomic otherwise), on which its threshold crossing and
// first touch are decided.
__global__ __launch_bounds__(kBlock) void k_bin_apply(PlainArgs a, int slot) {
  Ctl* c = a.ctl;
  int t, nf;
  if (!push_active(c, a.n, &t, &nf)) return;
  if (t >= c->max_rounds || c->selfed != t) return;
  const long long E = c->etotal;
  const bool pull = pull_round(a, E);
  if (!pull && !bin_round(a, E)) return;
  __shared__ double acc[kBinWidth];          // the item's sums, zero between items
  __shared__ int32_t s_list[kBinWidth];      // first touches of the item (offsets in the bin)
  __shared__ int s_items[kMaxBins + 1];      // first item of each bin
  // pass B: start of the item's run in each chunk, and the exclusive prefix
  // of the run lengths; pull: the bin's row offsets from its first arc
  __shared__ int s_runs[2 * kBinItemChunks + 1];
  static_assert(2 * kBinItemChunks + 1 >= kBinWidth + 1, "a bin's row offsets fit");
  int* const s_rs = s_runs;
  int* const s_rp = s_runs + kBinItemChunks;
  __shared__ int sh[kBlock / 64 + 1];
  __shared__ int s_nl, s_fb, s_tb, s_last;
  constexpr int kBinsPT = kMaxBins / kBlock;
  constexpr int kRunsPT = kBinItemChunks / kBlock;
  constexpr int kListPT = kBinWidth / kBlock;
  static_assert(kListPT <= 32, "flush masks are 32 bits");
  static_assert(kBinWidth < 65536, "the flush packs two counts in one int");
  const int nb = a.nbins;
  const int C = (int)((E + kBinChunk - 1) / kBinChunk);
  const double eps = c->eps;
  const unsigned pull_ep = pull ? *a.pull_epoch : 0u;
  int32_t* Fn = (t & 1) ? a.fbuf0 : a.fbuf1;
  int32_t* cntn = &c->cnt[(t + 1) & 1];
  for (int j = threadIdx.x; j < kBinWidth; j += kBlock) acc[j] = 0.0;
  // items per bin: the bin's expected share of the round's edges (E vol_b /
  // 2m) over kBinQ, at least enough that an item spans <= kBinItemChunks
  // chunks, at most one per chunk (pull: the bin's arcs vol_b over kBinQ);
  // every workgroup computes the same table
  {
    const int smin = (C + kBinItemChunks - 1) / kBinItemChunks;
    int loc[kBinsPT];
    int tsum = 0;
#pragma unroll
    for (int k = 0; k < kBinsPT; k++) {
      const int b = (int)threadIdx.x * kBinsPT + k;
      int it = 0;
      if (b < nb) {
        const double expect =
            pull ? (double)a.bin_vol[b] : (double)E * (double)a.bin_vol[b] / (double)a.vol_total;
        it = (int)ceil(expect / (double)kBinQ);
        if (!pull) {
          it = it > smin ? it : smin;
          it = it < C ? it : C;
        }
        it = it > 1 ? it : 1;
      }
      loc[k] = it;
      tsum += it;
    }
    int total;
    int ex = block_excl_scan_int(tsum, &total, sh);
#pragma unroll
    for (int k = 0; k < kBinsPT; k++) {
      const int b = (int)threadIdx.x * kBinsPT + k;
      if (b < nb) s_items[b] = ex;
      ex += loc[k];
    }
    if (threadIdx.x == 0) {
      s_items[nb] = total;
      s_nl = 0;
    }
    __syncthreads();
  }
  const int items = s_items[nb];
  for (int it = blockIdx.x; it < items; it += gridDim.x) {
    int lo = 0, hi = nb - 1;  // the bin: last b with s_items[b] <= it
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (s_items[mid] <= it) lo = mid; else hi = mid - 1;
    }
    const int b = lo;
    const int S = s_items[b + 1] - s_items[b];
    const int sl = it - s_items[b];
    const int vlo = a.bin_lo[b];
    const int W = a.bin_lo[b + 1] - vlo;
    const bool own = S == 1;
    if (pull) {
      // the slice of the bin's arcs: rows vlo .. vlo + Wn (the last bin may
      // end past n), arcs A0 .. A1 of the CSR
      const int Wn = (int)((int64_t)vlo + W < a.n ? W : a.n - vlo);
      const long long A0 = a.off[vlo], A1 = a.off[vlo + Wn];
      const long long j0 = A0 + (A1 - A0) * sl / S, j1 = A0 + (A1 - A0) * (sl + 1) / S;
      for (int r = threadIdx.x; r <= Wn; r += kBlock) s_runs[r] = (int)(a.off[vlo + r] - A0);
      __syncthreads();
      constexpr int kU = 4;
      for (long long e0 = j0; e0 < j1; e0 += kBlock * kU) {
        int32_t u[kU];
#pragma unroll
        for (int q = 0; q < kU; q++) {
          const long long e = e0 + q * kBlock + (int)threadIdx.x;
          u[q] = e < j1 ? a.nbr[e] : -1;
        }
        double cf[kU];
#pragma unroll
        for (int q = 0; q < kU; q++) {
          cf[q] = 0.0;
          if (u[q] >= 0) {
            const PullRec pr = a.pull[u[q]];
            if (pr.stamp == pull_ep) cf[q] = pr.coef;
          }
        }
#pragma unroll
        for (int q = 0; q < kU; q++) {
          bool first = false;
          int jl = 0;
          if (cf[q] != 0.0) {
            // the row holding arc e: the last row whose first arc is <= e
            const int rel = (int)(e0 + q * kBlock + (int)threadIdx.x - A0);
            int l2 = 0, h2 = Wn - 1;
            while (l2 < h2) {
              const int mid = (l2 + h2 + 1) >> 1;
              if (s_runs[mid] <= rel) l2 = mid; else h2 = mid - 1;
            }
            jl = l2;
            first = atomicAdd(&acc[jl], cf[q]) == 0.0;
          }
          wave_append(first, jl, s_list, &s_nl);
        }
      }
    } else {
      const int c0 = (int)((long long)sl * C / S), c1 = (int)((long long)(sl + 1) * C / S);
      const int nc = c1 - c0;
      // the item's runs
      int rl[kRunsPT];
      int lsum = 0;
#pragma unroll
      for (int k = 0; k < kRunsPT; k++) {
        const int q = (int)threadIdx.x * kRunsPT + k;
        rl[k] = 0;
        if (q < nc) {
          const int st = a.bin_T[(size_t)b * a.bin_cmax + c0 + q];
          const int en = a.bin_T[(size_t)(b + 1) * a.bin_cmax + c0 + q];
          s_rs[q] = (c0 + q) * kBinChunk + st;
          rl[k] = en - st;
          if (rl[k] < 0 || en > kBinChunk) { c->fault = 1; rl[k] = 0; }
        }
        lsum += rl[k];
      }
      int L;
      int ex = block_excl_scan_int(lsum, &L, sh);
#pragma unroll
      for (int k = 0; k < kRunsPT; k++) {
        const int q = (int)threadIdx.x * kRunsPT + k;
        if (q < nc) s_rp[q] = ex;
        ex += rl[k];
      }
      __syncthreads();
      // add every contribution into the LDS array; the first toucher of an
      // offset lists it
      constexpr int kU = 4;
      for (int j0 = 0; j0 < L; j0 += kBlock * kU) {
        int2 pr[kU];
#pragma unroll
        for (int u = 0; u < kU; u++) {
          const int j = j0 + u * kBlock + (int)threadIdx.x;
          pr[u] = make_int2(-1, 0);
          if (j < L) {
            int l2 = 0, h2 = nc - 1;
            while (l2 < h2) {
              const int mid = (l2 + h2 + 1) >> 1;
              if (s_rp[mid] <= j) l2 = mid; else h2 = mid - 1;
            }
            pr[u] = a.bin_pairs[s_rs[l2] + (j - s_rp[l2])];
          }
        }
        double cf[kU];
#pragma unroll
        for (int u = 0; u < kU; u++) cf[u] = pr[u].x >= 0 && pr[u].y < nf ? a.coef[pr[u].y] : 0.0;
#pragma unroll
        for (int u = 0; u < kU; u++) {
          const int jl = pr[u].x - vlo;
          bool first = false;
          if (pr[u].x >= 0) {
            // (contributions are positive, so exactly one addition per touched
            // offset returns 0; an impossible zero one is not listed)
            if (jl >= 0 && jl < W) first = atomicAdd(&acc[jl], cf[u]) == 0.0 && cf[u] != 0.0;
            else c->fault = 1;
          }
          wave_append(first, jl, s_list, &s_nl);
        }
      }
    }
    __syncthreads();
    // one update per touched destination
    const int nl = s_nl;
    unsigned fm = 0, tm = 0;
    int nfl = 0, ntl = 0;
    int32_t jv[kListPT];
    double xv[kListPT];
#pragma unroll
    for (int m = 0; m < kListPT; m++) {
      const int k = m * kBlock + (int)threadIdx.x;
      jv[m] = -1;
      xv[m] = 0.0;
      if (k < nl) {
        jv[m] = s_list[k];
        xv[m] = acc[jv[m]];
        acc[jv[m]] = 0.0;
      }
    }
#pragma unroll
    for (int m = 0; m < kListPT; m++) {
      if (jv[m] < 0) continue;
      const int32_t w = vlo + jv[m];
      double old, thr;
      if (own) {
        const VRec rec = a.vr[w];
        old = rec.r;
        a.vr[w].r = old + xv[m];
        thr = eps * (double)rec.deg;
      } else {
        thr = eps * (double)a.vr[w].deg;
        old = unsafeAtomicAdd(&a.vr[w].r, xv[m]);
      }
      if (old < thr && old + xv[m] >= thr) { fm |= 1u << m; nfl++; }
      if (__double_as_longlong(old) == 0) { tm |= 1u << m; ntl++; }
    }
    // both counts in one scan (each total is at most kBinWidth < 2^16)
    int both;
    const int bex = block_excl_scan_int(nfl | (ntl << 16), &both, sh);
    const int fex = bex & 0xffff, tex = bex >> 16;
    const int NF = both & 0xffff, NT = both >> 16;
    if (threadIdx.x == 0) {
      s_fb = NF > 0 ? atomicAdd(cntn, NF) : 0;
      s_tb = NT > 0 ? atomicAdd(&c->touched_cnt, NT) : 0;
      s_nl = 0;
    }
    __syncthreads();
    long long pf = (long long)s_fb + fex, pt = (long long)s_tb + tex;
#pragma unroll
    for (int m = 0; m < kListPT; m++) {
      if (jv[m] < 0) continue;
      const int32_t w = vlo + jv[m];
      if (fm >> m & 1u) {
        if (pf < a.n) Fn[pf] = w; else c->fault = 1;
        pf++;
      }
      if (tm >> m & 1u) {
        if (pt < a.n) a.touched[pt] = w; else c->fault = 1;
        pt++;
      }
    }
    __syncthreads();
  }
  if (last_block(&c->done[DONE_BIN], &s_last, false)) {
    if (threadIdx.x == 0) {
      c->pushes += nf;
      c->edges += E;
      c->bin_rounds += 1;
      if (pull) c->pull_rounds += 1;
      c->bin_edges += E;
      c->cnt[t & 1] = 0;
      c->round = t + 1;
      if (a.pull_epoch) *a.pull_epoch += 1u;
      if (slot >= 0) a.work_log[2 * slot + 1] = 1;
    }
  }
}

// edgeMap(G, Frontier, UpdateNgh) with the filter folded in.  Each
// workgroup takes a contiguous range of edge tiles; every edge is one
// device-scope FP64 atomic.  (Combining the contributions to the
// highest-degree destinations in LDS, as the batched scatter does, measured
// slower here: one query's round spreads over few workgroups, and the
// per-workgroup clear and flush cost more than the contention they save.)
//   PR-Nibble: into r, threshold eps d(w), first touches to the touched list.
//   HK-PR level j: into the level-(j+1) residuals, threshold
//     ((e^-t eps) d(w)) / (2 N psi_{j+1}), first touches to level j+1's list;
//     on the last level into p (UpdateNghLast), first touches of p to the
//     support list, no frontier.
//   Nibble step j -> j+1: into vector j+1, threshold eps d(w), first touches
//     to list j+1; each entry's own rho / 2 is added by the workgroup whose
//     tile holds the entry's first edge.
template <int MODE>
__device__ __forceinline__ void scatter_body(const PlainArgs& a, int slot, ScatterShared& sm,
                                             int pair = -1, bool apply = true) {
  constexpr bool HK = MODE == kModeHK;
  constexpr bool LEVELS = MODE != kModePR;
  Ctl* c = a.ctl;
  int t, nf;
  if (!push_active(c, a.n, &t, &nf)) return;
  if (HK ? t >= c->hk_N : t >= c->max_rounds) return;
  if (c->selfed != t) return;  // no entries built for this round (a self loop stopped before it)
  // which launch pairs of a first chunk carry rounds that could bin or pull
  // (the host queues k_bin_apply behind those pairs only); without
  // k_bin_apply behind it the round takes the atomic form
  if (MODE == kModePR && pair >= 0 && blockIdx.x == 0 && threadIdx.x == 0 &&
      (pull_round(a, c->etotal) || bin_round(a, c->etotal)))
    c->bin_pairs |= 1u << pair;
  if (MODE == kModePR && !apply) {
    // (falls through to the atomic form)
  } else if (MODE == kModePR && pull_round(a, c->etotal)) {
    // a pull round: the frontier's coefficients, stamped with the round's
    // epoch, for k_bin_apply to pull (which also closes the round)
    const unsigned ep = *a.pull_epoch;
    const int32_t* F = (t & 1) ? a.fbuf1 : a.fbuf0;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < nf; i += gridDim.x * kBlock)
      a.pull[F[i]] = PullRec{a.coef[i], ep, 0};
    return;
  } else if (MODE == kModePR && bin_round(a, c->etotal)) {
    bin_sort_chunks(a, nf, sm.bs);  // pass A; k_bin_apply adds and closes the round
    return;
  }
  int32_t* const s_start = sm.at.start;
  int64_t* const s_row = sm.at.row;
  double* const s_coef = sm.at.coef;
  int32_t* const s_fn = sm.at.fn;
  int32_t* const s_tv = sm.at.tv;
  int& s_nfn = sm.at.nfn;
  int& s_ntv = sm.at.ntv;
  int& s_base = sm.at.base;
  int& s_last = sm.at.last;
  const int ntiles = (int64_t)c->ntiles > a.tile_cap ? (int)a.tile_cap : c->ntiles;
  const long long E = c->etotal;
  const bool hk_last = HK && t + 1 == c->hk_N;
  const double eps = HK ? c->hk_A : c->eps;                   // threshold numerator factor
  const int32_t* Fc = (t & 1) ? a.fbuf1 : a.fbuf0;            // this round's frontier
  const double den = HK && !hk_last ? a.hk_B[t + 1] : 1.0;    // threshold denominator
  int32_t* Fn = (t & 1) ? a.fbuf0 : a.fbuf1;
  int32_t* cntn = &c->cnt[(t + 1) & 1];
  // where first touches go
  int32_t* tv_list = LEVELS ? (hk_last ? a.support : a.hk_tl[(t + 1) % 3]) : a.touched;
  int32_t* tv_cnt =
      LEVELS ? (hk_last ? &c->support_cnt : &c->hk_tlc[(t + 1) % 3]) : &c->touched_cnt;
  const int per = (ntiles + gridDim.x - 1) / gridDim.x;
  const int tb = blockIdx.x * per;
  const int te = tb + per < ntiles ? tb + per : ntiles;
  // workgroups without tiles (large grids, small rounds) leave at once; the
  // round is closed by the last of the `busy` ones (at least workgroup 0)
  const int busy = per > 0 ? (ntiles + per - 1) / per : 1;
  if ((int)blockIdx.x >= busy) return;
  if (threadIdx.x == 0) { s_nfn = 0; s_ntv = 0; }
  __syncthreads();

  for (int tile = tb; tile < te; tile++) {
    const long long e0 = (long long)tile * kEdgeTile;
    const long long e1 = e0 + kEdgeTile < E ? e0 + kEdgeTile : E;
    const int i0 = a.tile_start[tile];
    const int i1 = tile + 1 < ntiles ? a.tile_start[tile + 1] : nf - 1;
    if (i0 < 0 || i1 < i0 || i1 >= nf || i1 - i0 + 1 > kEdgeTile + 1) {
      c->fault = 1;  // inconsistent tile map: skip the tile, report a fault
      continue;
    }
    const int cnt = i1 - i0 + 1;
    for (int j = threadIdx.x; j < cnt; j += kBlock) {
      s_start[j] = (int32_t)(a.estart[i0 + j] - e0);
      s_row[j] = a.rowp[i0 + j];
      s_coef[j] = a.coef[i0 + j];
    }
    __syncthreads();
    // Four independent edges per thread: all neighbour loads, then all
    // degree loads and atomics, then the decisions, so latencies overlap.
    int32_t w[kEdgesPerThread];
    double cf[kEdgesPerThread];
#pragma unroll
    for (int k = 0; k < kEdgesPerThread; k++) {
      const int rel = k * kBlock + (int)threadIdx.x;
      w[k] = -1;
      cf[k] = 0.0;
      if (e0 + rel < e1) {
        int lo = 0, hi = cnt - 1;
        while (lo < hi) {
          int mid = (lo + hi + 1) >> 1;
          if (s_start[mid] <= rel) lo = mid; else hi = mid - 1;
        }
        w[k] = a.nbr[s_row[lo] + (rel - s_start[lo])];
        cf[k] = s_coef[lo];
      }
    }
    int32_t dw[kEdgesPerThread];
#pragma unroll
    for (int k = 0; k < kEdgesPerThread; k++) dw[k] = w[k] >= 0 && !hk_last ? a.vr[w[k]].deg : 0;
    double old[kEdgesPerThread];
#pragma unroll
    for (int k = 0; k < kEdgesPerThread; k++) {
      double* dst = nullptr;
      if (w[k] >= 0) dst = !LEVELS ? &a.vr[w[k]].r : hk_last ? &a.p[w[k]] : hk_res(a, t + 1, w[k]);
      old[k] = dst ? unsafeAtomicAdd(dst, cf[k]) : 0.0;
    }
#pragma unroll
    for (int k = 0; k < kEdgesPerThread; k++) {
      if (hk_last)
        wave_append(w[k] >= 0 && __double_as_longlong(old[k]) == 0, w[k], s_tv, &s_ntv);
      else
        decide(w[k] >= 0, old[k], cf[k], (eps * (double)dw[k]) / den, w[k], s_fn, &s_nfn, s_tv,
               &s_ntv);
    }
    if (!hk_last) block_flush(cntn, Fn, a.n, s_fn, &s_nfn, &s_base, &c->fault);
    block_flush(tv_cnt, tv_list, a.n, s_tv, &s_ntv, &s_base, &c->fault);
    if (MODE == kModeNB) {
      // the kept halves of the entries whose first edge is in this tile
      for (int jj = threadIdx.x; jj < cnt; jj += kBlock) {
        const int st = s_start[jj];
        if (st < 0 || e0 + st >= e1) continue;
        const int i = i0 + jj;
        const int32_t v = Fc[i];
        const double h = a.sp[i];
        const double o = unsafeAtomicAdd(hk_res(a, t + 1, v), h);
        decide(true, o, h, eps * (double)a.vr[v].deg, v, s_fn, &s_nfn, s_tv, &s_ntv);
      }
      block_flush(cntn, Fn, a.n, s_fn, &s_nfn, &s_base, &c->fault);
      block_flush(tv_cnt, tv_list, a.n, s_tv, &s_ntv, &s_base, &c->fault);
    }
  }
  if (last_block_of(&c->done[DONE_SCATTER], &s_last, false, (unsigned)busy)) {
    if (threadIdx.x == 0) {
      c->pushes += nf;
      c->edges += E;
      c->cnt[t & 1] = 0;
      c->round = t + 1;
      if (a.pull_epoch) *a.pull_epoch += 1u;
      if (slot >= 0) a.work_log[2 * slot + 1] = 1;
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_scatter(PlainArgs a, int slot, int pair, int apply) {
  __shared__ ScatterShared sm;
  scatter_body<kModePR>(a, slot, sm, pair, apply != 0);
}
__global__ __launch_bounds__(kBlock) void k_hk_scatter(PlainArgs a) {
  __shared__ ScatterShared sm;
  scatter_body<kModeHK>(a, -1, sm);
}
__global__ __launch_bounds__(kBlock) void k_nb_scatter(PlainArgs a) {
  __shared__ ScatterShared sm;
  scatter_body<kModeNB>(a, -1, sm);
}

// HK-PR initialisation (Fig. alg:hkpr: r = {(x, 1)}, Frontier = {x},
// j = 0); level 0 touched only x.
__global__ void k_hk_init(PlainArgs a, int32_t x, int32_t N, double t, double A) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  Ctl* c = a.ctl;
  c->cs = 0.0;
  c->cn = 0.0;
  c->keep = 0.0;
  c->eps = 0.0;
  c->seed = x;
  c->rule = -1;
  c->max_rounds = N;
  c->opt_rule = 1;
  c->round = 0;
  c->cnt[0] = 1;
  c->cnt[1] = 0;
  c->ntiles = 0;
  c->etotal = 0;
  c->pushes = 0;
  c->edges = 0;
  c->support_cnt = 0;
  c->touched_cnt = 0;  // no residual is reported: the sweep gathers none
  c->fault = 0;
  c->limited = 0;
  c->N = 0;
  c->sort_flip = 0;
  c->rnnz = 0;
  c->vol_total = a.vol_total;
  c->best_cut = 0;
  c->best_vol = 0;
  c->best_den = 0;
  c->kstar = 0;
  c->phi = 0.0;
  reset_round_book(c);
  c->hk_N = N;
  c->hk_t = t;
  c->hk_A = A;
  c->hk_tlc[0] = 1;
  c->hk_tlc[1] = 0;
  c->hk_tlc[2] = 0;
  a.hk_tl[0][0] = x;
  a.fbuf0[0] = x;
  a.vr[x].r = 1.0;
  c->status = ST_PUSH;
}

// Nibble initialisation (Fig. alg:nibble: p = {(x, 1)}, Frontier = {x});
// vector 0 is the seed's indicator, its support list holds x.
__global__ void k_nb_init(PlainArgs a, int32_t x, double eps, int32_t T) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  Ctl* c = a.ctl;
  c->cs = 0.0;
  c->cn = 0.0;
  c->keep = 0.0;
  c->eps = eps;
  c->seed = x;
  c->rule = -2;
  c->max_rounds = T;
  c->opt_rule = 1;
  c->round = 0;
  c->cnt[0] = 1;
  c->cnt[1] = 0;
  c->ntiles = 0;
  c->etotal = 0;
  c->pushes = 0;
  c->edges = 0;
  c->support_cnt = 0;
  c->touched_cnt = 0;
  c->fault = 0;
  c->limited = 0;
  c->N = 0;
  c->sort_flip = 0;
  c->rnnz = 0;
  c->vol_total = a.vol_total;
  c->best_cut = 0;
  c->best_vol = 0;
  c->best_den = 0;
  c->kstar = 0;
  c->phi = 0.0;
  reset_round_book(c);
  c->hk_N = 0;
  c->hk_tlc[0] = 1;
  c->hk_tlc[1] = 0;
  c->hk_tlc[2] = 0;
  a.hk_tl[0][0] = x;
  a.fbuf0[0] = x;
  a.vr[x].r = 1.0;
  c->status = ST_PUSH;
}

// End of Nibble after J steps, returning vector R (J, or J - 1 when step J
// left an empty frontier): p and the support list take vector R over the
// vertices it touched, and both vector arrays are cleared (vector J over
// list J, vector J - 1 over list J - 1: every earlier one was cleared by
// the self kernel two steps later; each entry of vector R is read and
// cleared by the same thread).  The frontier count is zeroed so that the
// sweep may start.
__global__ __launch_bounds__(kBlock) void k_nb_finish(PlainArgs a, int32_t R, int32_t J) {
  Ctl* c = a.ctl;
  for (int q = 0; q < 2; q++) {
    const int lv = J - q;
    if (lv < 0) continue;
    const int li = lv % 3;
    const int cnt = c->hk_tlc[li];
    const int32_t* L = a.hk_tl[li];
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < cnt; i += gridDim.x * kBlock) {
      const int32_t v = L[i];
      double* x = hk_res(a, lv, v);
      if (lv == R) {
        a.p[v] = *x;
        a.support[i] = v;
      }
      *x = 0.0;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    c->support_cnt = c->hk_tlc[R % 3];
    c->cnt[J & 1] = 0;
  }
}

// After the last HK-PR level: residuals can remain only on the vertices the
// last two levels touched (every earlier level was cleared by the self
// kernel two levels later); clear both arrays there.
__global__ __launch_bounds__(kBlock) void k_hk_clear(PlainArgs a) {
  Ctl* c = a.ctl;
  const int J = c->round;
  for (int q = 0; q < 2; q++) {
    const int lv = J - q;
    if (lv < 0) continue;
    const int li = lv % 3;
    const int cnt = c->hk_tlc[li];
    const int32_t* L = a.hk_tl[li];
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < cnt; i += gridDim.x * kBlock) {
      const int32_t v = L[i];
      a.vr[v].r = 0.0;
      a.hk_r1[v] = 0.0;
    }
  }
}

// ---------------------------------------------------------------- beta variant
// PR-Nibble pushing the top beta fraction of the active set by r/d per round
// (end of Sec. 3.3).  The frontier holds the whole active set; before the
// round it is ranked with the sweep's sort (keys: bit-inverted r/d, ties by
// ascending id) and the top k = ceil(beta |F|) move to its front as the
// round's frontier; after the round the other |F| - k, still at or above
// their thresholds (their r only grew), join the next frontier.

// Sort keys of the active set (count in N; 0 when the push has ended).
__global__ __launch_bounds__(kBlock) void k_beta_keys(PlainArgs a) {
  Ctl* c = a.ctl;
  int t, nf;
  if (!push_active(c, a.n, &t, &nf) || t >= c->max_rounds) {
    if (blockIdx.x == 0 && threadIdx.x == 0) { c->N = 0; c->beta_nf = 0; }
    return;
  }
  const int32_t* F = (t & 1) ? a.fbuf1 : a.fbuf0;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < nf; i += gridDim.x * kBlock) {
    const int32_t v = F[i];
    const VRec rec = a.vr[v];
    SortElem e;
    e.key = ~(unsigned long long)__double_as_longlong(rec.r / (double)rec.deg);
    e.id = v;
    e.seg = 0;
    a.sbuf[0][i] = e;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    c->N = nf;
    c->sort_flip = 0;
    c->beta_nf = nf;
  }
}

// Ranked active set back into the frontier buffer; the round's frontier is
// its first k entries.
__global__ __launch_bounds__(kBlock) void k_beta_select(PlainArgs a) {
  Ctl* c = a.ctl;
  const int nf = c->beta_nf;
  if (nf <= 0) return;
  const int t = c->round;
  int32_t* F = (t & 1) ? a.fbuf1 : a.fbuf0;
  const SortElem* el = a.sbuf[c->sort_flip & 1];
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < nf; i += gridDim.x * kBlock) F[i] = el[i].id;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    long long k = (long long)ceil(c->beta * (double)nf);
    if (k < 1) k = 1;
    if (k > nf) k = nf;
    c->beta_k = (int32_t)k;
    c->cnt[t & 1] = (int32_t)k;
  }
}

// After the round: the unpushed part of the ranked set joins the next
// frontier (one counter atomic per workgroup step).
__global__ __launch_bounds__(kBlock) void k_beta_carry(PlainArgs a) {
  Ctl* c = a.ctl;
  const int nf = c->beta_nf, k = c->beta_k;
  if (nf <= k) return;
  const int t = c->round;              // the round just closed was t - 1
  const int32_t* F = ((t - 1) & 1) ? a.fbuf1 : a.fbuf0;
  int32_t* Fn = (t & 1) ? a.fbuf1 : a.fbuf0;
  __shared__ int s_base;
  for (int i0 = k + blockIdx.x * kBlock; i0 < nf; i0 += gridDim.x * kBlock) {
    const int m = nf - i0 < kBlock ? nf - i0 : kBlock;
    if (threadIdx.x == 0) s_base = atomicAdd(&c->cnt[t & 1], m);
    __syncthreads();
    if ((int)threadIdx.x < m) {
      const long long slot = (long long)s_base + threadIdx.x;
      if (slot < a.n) Fn[slot] = F[i0 + threadIdx.x]; else c->fault = 1;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- sweep

// The sweep may start once the frontier is empty (or the watchdog fired).
__device__ __forceinline__ bool sweep_ready(const Ctl* c) {
  if (c->status == ST_LIMIT) return true;
  return c->status == ST_PUSH && c->cnt[c->round & 1] == 0;
}

// Sort keys: non-increasing p/d is ascending order of the bit-inverted IEEE
// pattern of the positive ratio; equal ratios order by ascending id.
// The sweep sequence is queued for supports of at most `bound` vertices (it
// sets the sort's launches); a larger support leaves the query unswept, for
// a sweep queued with a larger bound.
__global__ __launch_bounds__(kBlock) void k_sweep_keys(PlainArgs a, long long bound) {
  Ctl* c = a.ctl;
  if (!sweep_ready(c) || (long long)c->support_cnt > bound) return;
  __shared__ int s_last;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    SweepOut o;
    o.ids = a.sid;
    o.p = a.sp;
    o.rid = a.rid;
    o.rval = a.rval;
    o.rcap = a.n;
    o.pad = 0;
    c->out = o;
  }
  const int N = (int64_t)c->support_cnt > a.n ? (int)a.n : c->support_cnt;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < N; i += gridDim.x * kBlock) {
    int32_t v = a.support[i];
    double ratio = a.p[v] / (double)a.vr[v].deg;
    SortElem e;
    e.key = ~(unsigned long long)__double_as_longlong(ratio);
    e.id = v;
    e.seg = 0;
    a.sbuf[0][i] = e;
  }
  if (last_block(&c->done[DONE_KEYS], &s_last, false)) {
    if (threadIdx.x == 0) {
      c->N = N;
      c->sort_flip = 0;
      c->status = ST_SWEEPING;
    }
  }
}

// Rank map (rank[v_k] = k, outside = 0) with per-position degree, p and id,
// and the inclusive volume prefix vol(S_k) with the edge-tile map over the
// support's edges in sweep order (the offsets of the Z array in Theorem 1's
// proof).
__global__ __launch_bounds__(kBlock) void k_vol_scan(PlainArgs a) {
  Ctl* c = a.ctl;
  if (c->status != ST_SWEEPING) return;
  const int N = c->N;
  if (N <= 0) return;
  const SortElem* el = a.sbuf[c->sort_flip & 1];
  int32_t* const out_ids = c->out.ids;
  double* const out_p = c->out.p;
  __shared__ long long sh[kBlock / 64 + 1];
  __shared__ long long s_excl;
  __shared__ int s_tk[2];
  ScanSite* site = &c->scan[SCAN_VOL];
  scan_clear_prev(site, a.desc[SCAN_VOL], a.desc_cap);
  unsigned long long* desc = a.desc[SCAN_VOL] + (size_t)site->parity * a.desc_cap;
  const int nblk = (N + kScanBlock - 1) / kScanBlock;
  for (;;) {
    bool last;
    int b = scan_ticket(site, nblk, s_tk, &last);
    if (b >= nblk) break;
    // kScanItems consecutive positions per thread (see k_self)
    const int i0 = b * kScanBlock + (int)threadIdx.x * kScanItems;
    int32_t dk[kScanItems];
    long long dsum = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; k++) {
      const int i = i0 + k;
      dk[k] = 0;
      if (i < N) {
        const int32_t v = el[i].id;
        a.vr[v].rank = i + 1;
        dk[k] = a.vr[v].deg;
        a.sdeg[i] = dk[k];
        out_p[i] = a.p[v];
        out_ids[i] = v;
        a.scnt[i] = 0;
      }
      dsum += dk[k];
    }
    long long agg;
    const long long ex = block_excl_scan<kBlock>(dsum, &agg, sh);
    if (threadIdx.x < 64) {
      const long long ex0 = scan_lookback(desc, b, agg, &c->fault);
      if (threadIdx.x == 0) s_excl = ex0;
    }
    __syncthreads();
    long long s = s_excl + ex;
#pragma unroll
    for (int k = 0; k < kScanItems; k++) {
      const int i = i0 + k;
      if (i < N) {
        a.svol[i] = s + dk[k];
        mark_tiles(a.tile_start, a.tile_cap, s, dk[k], i, &c->fault);
      }
      s += dk[k];
    }
    if (b == nblk - 1 && threadIdx.x == 0) {
      const long long base = s_excl + agg;
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
  const int32_t* const sid = c->out.ids;
  const int ntiles = (int64_t)c->ntiles > a.tile_cap ? (int)a.tile_cap : c->ntiles;
  const long long E = c->etotal;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const long long e0 = (long long)tile * kEdgeTile;
    const long long e1 = e0 + kEdgeTile < E ? e0 + kEdgeTile : E;
    const int i0 = a.tile_start[tile];
    const int i1 = tile + 1 < ntiles ? a.tile_start[tile + 1] : N - 1;
    if (i0 < 0 || i1 < i0 || i1 >= N || i1 - i0 + 1 > kEdgeTile + 1) {
      c->fault = 1;
      continue;
    }
    const int cnt = i1 - i0 + 1;
    for (int j = threadIdx.x; j < cnt; j += kBlock) {
      int k = i0 + j;
      s_start[j] = (int32_t)(a.svol[k] - a.sdeg[k] - e0);
      s_row[j] = a.off[sid[k]];
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
        int32_t w = a.nbr[s_row[lo] + (rel - s_start[lo])];
        rw[kk] = a.vr[w].rank;
        own[kk] = lo;
      }
    }
#pragma unroll
    for (int kk = 0; kk < kEdgesPerThread; kk++) {
      if (own[kk] >= 0 && rw[kk] > 0 && rw[kk] < i0 + own[kk] + 1) atomicAdd(&s_cnt[own[kk]], 1);
    }
    __syncthreads();
    for (int j = threadIdx.x; j < cnt; j += kBlock)
      if (s_cnt[j] != 0) atomicAdd(&a.scnt[i0 + j], s_cnt[j]);
    __syncthreads();
  }
}

// Candidate order for the best prefix: smaller cut/den (exact), then smaller k.
__device__ __forceinline__ bool cand_better(long long oc, long long od, long long ok, long long xc,
                                            long long xd, long long xk) {
  if (ok <= 0) return false;
  if (xk <= 0) return true;
  if (ratio_lt(oc, od, xc, xd)) return true;
  return !ratio_lt(xc, xd, oc, od) && ok < xk;
}

__device__ void block_argmin(long long* s_bc, long long* s_bd, long long* s_bk) {
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      const int u = threadIdx.x + o;
      if (cand_better(s_bc[u], s_bd[u], s_bk[u], s_bc[threadIdx.x], s_bd[threadIdx.x],
                      s_bk[threadIdx.x])) {
        s_bc[threadIdx.x] = s_bc[u];
        s_bd[threadIdx.x] = s_bd[u];
        s_bk[threadIdx.x] = s_bk[u];
      }
    }
    __syncthreads();
  }
}

// Inclusive prefix of the boundary deltas gives |boundary(S_k)|; with vol_k
// the conductance of every prefix follows.  Each block publishes its best
// prefix (smallest cut/den by exact comparison, first k on ties, den = 0
// excluded); k_sweep_finish reduces the candidates.
__global__ __launch_bounds__(kBlock) void k_cut_scan(PlainArgs a) {
  Ctl* c = a.ctl;
  if (c->status != ST_SWEEPING) return;
  const int N = c->N;
  if (N <= 0) return;
  __shared__ long long sh[kBlock / 64 + 1];
  __shared__ long long s_excl;
  __shared__ int s_tk[2];
  __shared__ long long s_bc[kBlock], s_bd[kBlock], s_bk[kBlock];
  ScanSite* site = &c->scan[SCAN_CUT];
  scan_clear_prev(site, a.desc[SCAN_CUT], a.desc_cap);
  unsigned long long* desc = a.desc[SCAN_CUT] + (size_t)site->parity * a.desc_cap;
  const int nblk = (N + kScanBlock - 1) / kScanBlock;
  const long long vt = c->vol_total;
  for (;;) {
    bool last;
    int b = scan_ticket(site, nblk, s_tk, &last);
    if (b >= nblk) break;
    // kScanItems consecutive positions per thread (see k_self)
    const int i0 = b * kScanBlock + (int)threadIdx.x * kScanItems;
    long long dk[kScanItems];
    long long dsum = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; k++) {
      const int i = i0 + k;
      dk[k] = i < N ? (long long)a.sdeg[i] - 2ll * a.scnt[i] : 0;
      dsum += dk[k];
    }
    long long agg;
    const long long ex = block_excl_scan<kBlock>(dsum, &agg, sh);
    if (threadIdx.x < 64) {
      const long long ex0 = scan_lookback(desc, b, agg, &c->fault);
      if (threadIdx.x == 0) s_excl = ex0;
    }
    __syncthreads();
    long long cut = s_excl + ex;
    long long mc = -1, md = 1, mk = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; k++) {
      const int i = i0 + k;
      cut += dk[k];
      if (i < N) {
        const long long vol = a.svol[i];
        const long long den = vol < vt - vol ? vol : vt - vol;
        if (den > 0 && (mk <= 0 || ratio_lt(cut, den, mc, md))) { mc = cut; md = den; mk = i + 1; }
      }
    }
    s_bc[threadIdx.x] = mc; s_bd[threadIdx.x] = md; s_bk[threadIdx.x] = mk;
    __syncthreads();
    block_argmin(s_bc, s_bd, s_bk);
    if (threadIdx.x == 0) {
      a.bbest[3 * b] = s_bc[0];
      a.bbest[3 * b + 1] = s_bd[0];
      a.bbest[3 * b + 2] = s_bk[0];
    }
    __syncthreads();
  }
  // p and the sweep rank of every support vertex are read by no later
  // kernel (k_vol_scan read p, k_cut_count the rank): reset them
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < N; i += gridDim.x * kBlock) {
    const int32_t v = a.support[i];
    a.vr[v].rank = 0;
    a.p[v] = 0.0;
  }
}

// Reduce the per-block candidates of k_cut_scan (one workgroup).
__device__ void cut_final(const PlainArgs& a, Ctl* c, int N) {
  const int nblk = (N + kScanBlock - 1) / kScanBlock;
  __shared__ long long s_bc[kBlock], s_bd[kBlock], s_bk[kBlock];
  long long mc = -1, md = 1, mk = 0;
  for (int j = threadIdx.x; j < nblk; j += kBlock) {
    long long jc = a.bbest[3 * j], jd = a.bbest[3 * j + 1], jk = a.bbest[3 * j + 2];
    if (cand_better(jc, jd, jk, mc, md, mk)) { mc = jc; md = jd; mk = jk; }
  }
  s_bc[threadIdx.x] = mc; s_bd[threadIdx.x] = md; s_bk[threadIdx.x] = mk;
  __syncthreads();
  block_argmin(s_bc, s_bd, s_bk);
  if (threadIdx.x == 0) {
    long long bk = s_bk[0];
    c->kstar = bk > 0 ? bk : 0;
    c->best_cut = bk > 0 ? s_bc[0] : 0;
    c->best_den = bk > 0 ? s_bd[0] : 0;
    c->best_vol = bk > 0 ? a.svol[bk - 1] : 0;
    c->phi = bk > 0 ? (double)s_bc[0] / (double)s_bd[0] : 0.0;
  }
}

// One workgroup reduces k_cut_scan's per-block candidates to the best
// prefix and marks the sweep finished.  The query's dense state is reset by
// then: r of every touched vertex by the block sort's side job, p and the
// sweep rank of every support vertex by k_cut_scan.
__global__ __launch_bounds__(kBlock) void k_sweep_finish(PlainArgs a) {
  Ctl* c = a.ctl;
  if (c->status != ST_SWEEPING) return;
  if (c->N > 0) cut_final(a, c, c->N);
  if (threadIdx.x == 0) {
    c->t_end = (long long)wall_clock64();
    c->status = ST_SWEPT;
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
                             double alpha, double eps, int32_t max_rounds, double beta) {
  hipLaunchKernelGGL(k_query_init, dim3(1), dim3(64), 0, s, a, seed, rule, alpha, eps,
                     max_rounds, beta);
  return hipGetLastError();
}

hipError_t launch_query_init_guarded(hipStream_t s, const PlainArgs& a, int32_t seed,
                                     int32_t rule, double alpha, double eps, int32_t max_rounds) {
  hipLaunchKernelGGL(k_query_init_guarded, dim3(1), dim3(64), 0, s, a, seed, rule, alpha, eps,
                     max_rounds);
  return hipGetLastError();
}

hipError_t launch_query_init_set(hipStream_t s, const PlainArgs& a, int32_t nseeds, int32_t rule,
                                 double alpha, double eps, int32_t max_rounds) {
  int grid = (nseeds + kBlock - 1) / kBlock;
  if (grid > 1024) grid = 1024;
  hipLaunchKernelGGL(k_query_init_set, dim3(grid), dim3(kBlock), 0, s, a, nseeds, rule, alpha, eps,
                     max_rounds);
  return hipGetLastError();
}

hipError_t launch_beta_pre(hipStream_t s, const PlainArgs& a, int grid, int64_t max_count) {
  hipLaunchKernelGGL(k_beta_keys, dim3(grid), dim3(kBlock), 0, s, a);
  SortArgs sa;
  sa.buf[0] = a.sbuf[0];
  sa.buf[1] = a.sbuf[1];
  sa.count = &a.ctl->N;
  sa.flip = &a.ctl->sort_flip;
  sa.done = &a.ctl->done[DONE_SORT];
  sa.active = nullptr;
  sa.active_value = 0;
  sa.rank = nullptr;
  hipError_t e = launch_sort(s, sa, max_count < a.n ? max_count : a.n, grid);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_beta_select, dim3(grid), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_beta_post(hipStream_t s, const PlainArgs& a, int grid) {
  hipLaunchKernelGGL(k_beta_carry, dim3(grid), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_hk_init(hipStream_t s, const PlainArgs& a, int32_t x, int32_t N, double t,
                          double A) {
  hipLaunchKernelGGL(k_hk_init, dim3(1), dim3(64), 0, s, a, x, N, t, A);
  return hipGetLastError();
}

hipError_t launch_hk_level(hipStream_t s, const PlainArgs& a, int grid_self, int grid_scatter) {
  hipLaunchKernelGGL(k_hk_self, dim3(grid_self), dim3(kBlock), 0, s, a);
  hipLaunchKernelGGL(k_hk_scatter, dim3(grid_scatter), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_nb_init(hipStream_t s, const PlainArgs& a, int32_t x, double eps, int32_t T) {
  hipLaunchKernelGGL(k_nb_init, dim3(1), dim3(64), 0, s, a, x, eps, T);
  return hipGetLastError();
}

hipError_t launch_nb_step(hipStream_t s, const PlainArgs& a, int grid_self, int grid_scatter) {
  hipLaunchKernelGGL(k_nb_self, dim3(grid_self), dim3(kBlock), 0, s, a);
  hipLaunchKernelGGL(k_nb_scatter, dim3(grid_scatter), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_nb_finish(hipStream_t s, const PlainArgs& a, int32_t R, int32_t J, int grid) {
  hipLaunchKernelGGL(k_nb_finish, dim3(grid), dim3(kBlock), 0, s, a, R, J);
  return hipGetLastError();
}

hipError_t launch_hk_clear(hipStream_t s, const PlainArgs& a, int grid) {
  hipLaunchKernelGGL(k_hk_clear, dim3(grid), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_self(hipStream_t s, const PlainArgs& a, int grid, hipEvent_t t0, hipEvent_t t1,
                       int slot) {
  if (slot >= kMaxChunk) return hipErrorInvalidValue;
  if (t0)
    hipExtLaunchKernelGGL(k_self, dim3(grid), dim3(kBlock), 0, s, t0, t1, 0, a, slot);
  else
    hipLaunchKernelGGL(k_self, dim3(grid), dim3(kBlock), 0, s, a, slot);
  return hipGetLastError();
}

hipError_t launch_scatter(hipStream_t s, const PlainArgs& a, int grid, hipEvent_t t0,
                          hipEvent_t t1, int slot, int grid_bin, int pair, bool apply_wanted) {
  if (slot >= kMaxChunk || pair >= 32) return hipErrorInvalidValue;
  // k_bin_apply only where a round can be binned or pulled (an empty
  // launch still costs a dispatch every round)
  const bool apply = apply_wanted && bins_possible(a);
  const int ap = apply ? 1 : 0;
  if (t0) {
    hipExtLaunchKernelGGL(k_scatter, dim3(grid), dim3(kBlock), 0, s, t0, apply ? nullptr : t1, 0,
                          a, slot, pair, ap);
    if (apply)
      hipExtLaunchKernelGGL(k_bin_apply, dim3(grid_bin), dim3(kBlock), 0, s, nullptr, t1, 0, a,
                            slot);
  } else {
    hipLaunchKernelGGL(k_scatter, dim3(grid), dim3(kBlock), 0, s, a, slot, pair, ap);
    if (apply) hipLaunchKernelGGL(k_bin_apply, dim3(grid_bin), dim3(kBlock), 0, s, a, slot);
  }
  return hipGetLastError();
}

// A finished query's results, from the sweep's buffers into its result
// block: the support in sweep order with p, and the nonzeros of r.
__global__ __launch_bounds__(kBlock) void k_copy_result(PlainArgs a, int32_t* ids, double* p,
                                                        int32_t* rid, double* rval, int N, int R) {
  const int stride = gridDim.x * kBlock;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < N; i += stride) {
    ids[i] = a.sid[i];
    p[i] = a.sp[i];
  }
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < R; i += stride) {
    rid[i] = a.rid[i];
    rval[i] = a.rval[i];
  }
}

hipError_t launch_copy_result(hipStream_t s, const PlainArgs& a, int32_t* ids, double* p,
                              int32_t* rid, double* rval, int N, int R, int grid) {
  if (N < 0 || R < 0 || N > a.n || R > a.n) return hipErrorInvalidValue;
  if (N == 0 && R == 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_result, dim3(grid), dim3(kBlock), 0, s, a, ids, p, rid, rval, N, R);
  return hipGetLastError();
}

// Several results' parts into one destination (the host's pinned staging
// memory): one workgroup per part at a time, 16-byte words where both ends
// allow it.
__global__ __launch_bounds__(kBlock) void k_gather_results(const GatherJob* jobs, int njobs,
                                                           uint32_t* dst) {
  for (int j = blockIdx.x; j < njobs; j += gridDim.x) {
    const GatherJob J = jobs[j];
    const uint32_t* src = J.src;
    uint32_t* out = dst + J.dst_off;
    const uint64_t nw = J.words;
    const bool wide = ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(out)) & 15) == 0;
    const uint64_t n4 = wide ? nw / 4 : 0;
    for (uint64_t i = threadIdx.x; i < n4; i += kBlock)
      reinterpret_cast<uint4*>(out)[i] = reinterpret_cast<const uint4*>(src)[i];
    for (uint64_t i = 4 * n4 + threadIdx.x; i < nw; i += kBlock) out[i] = src[i];
  }
}

hipError_t launch_gather_results(hipStream_t s, const GatherJob* jobs, int njobs, uint32_t* dst) {
  if (njobs <= 0) return hipSuccess;
  const int grid = njobs < 1024 ? njobs : 1024;
  hipLaunchKernelGGL(k_gather_results, dim3(grid), dim3(kBlock), 0, s, jobs, njobs, dst);
  return hipGetLastError();
}

hipError_t launch_sweep(hipStream_t s, const PlainArgs& a, int grid, int64_t max_count) {
  hipLaunchKernelGGL(k_sweep_keys, dim3(grid), dim3(kBlock), 0, s, a, (long long)max_count);
  SortArgs sa;
  sa.buf[0] = a.sbuf[0];
  sa.buf[1] = a.sbuf[1];
  sa.count = &a.ctl->N;
  sa.flip = &a.ctl->sort_flip;
  sa.done = &a.ctl->done[DONE_SORT];
  sa.active = &a.ctl->status;
  sa.active_value = ST_SWEEPING;
  // the volume prefix is written only after the sort: its words hold the
  // small-count path's rank accumulators meanwhile
  sa.rank = reinterpret_cast<unsigned long long*>(a.svol);
  // the block sort's workgroups without a tile gather the nonzeros of r over
  // the touched list into the result buffers and reset r (no later sweep
  // kernel reads r)
  static_assert(sizeof(VRec) % sizeof(double) == 0, "r read with a stride of whole records");
  sa.side_ids = a.touched;
  sa.side_count = &a.ctl->touched_cnt;
  sa.side_val = &a.vr[0].r;
  sa.side_stride = (int)(sizeof(VRec) / sizeof(double));
  sa.side_out_id = a.rid;
  sa.side_out_val = a.rval;
  sa.side_out_cnt = &a.ctl->rnnz;
  sa.side_out_cap = a.n;
  sa.side_fault = &a.ctl->fault;
  hipError_t e = launch_sort(s, sa, max_count < a.n ? max_count : a.n, grid);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_vol_scan, dim3(grid), dim3(kBlock), 0, s, a);
  // the count walks many short, latency-bound steps: a larger grid keeps
  // each workgroup to about one
  hipLaunchKernelGGL(k_cut_count, dim3(4 * grid), dim3(kBlock), 0, s, a);
  hipLaunchKernelGGL(k_cut_scan, dim3(grid), dim3(kBlock), 0, s, a);
  hipLaunchKernelGGL(k_sweep_finish, dim3(1), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

}  // namespace plc
