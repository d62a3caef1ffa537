// plc.cpp -- host side of libplc: the C ABI declared in include/plc.h.
//
// A context owns a view of the caller's device arena, the caller's stream and
// a pinned host mirror of the device control block.  plc_run drives the plain
// path: per query it queues the seed initialisation, a chunk of (self,
// scatter) launch pairs (launches past the end of the push exit at once) and
// the sweep sequence for the largest recent support (it runs only if the
// push has ended within that bound), then reads the control block back; an
// unfinished push gets short further chunks, and a larger support the sweep
// for its own bound, each with a read-back.  Within one plc_run call the
// next query's guarded initialisation and first chunk are queued behind the
// running query's first read-back (they stand aside on the device while the
// running query is unfinished), so the GPU works while the host reads back.  Results are copied
// device-to-device into an exact-size arena block, and the dense per-vertex
// state is reset through the touched list.  The batch engine (plc_batch_reserve and after)
// runs many queries per launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstddef>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <set>
#include <thread>
#include <vector>

#include "../../include/plc.h"
#include "arena.h"
#include "batch_device.h"
#include "plc_device.h"

using plc::Arena;
using plc::Ctl;
using plc::PlainArgs;

namespace {

struct Result {
  plc_result_info info{};
  void* block = nullptr;
  int32_t* ids = nullptr;
  double* p = nullptr;
  int32_t* rid = nullptr;
  double* rval = nullptr;
};

struct EventPair {
  hipEvent_t a = nullptr, b = nullptr;
};

// A launch sequence recorded once as a HIP graph (on the context's capture
// stream) and replayed with one hipGraphLaunch on the caller's stream.  The
// fields below exec say what it was recorded for.  Graphs carry no event
// nodes: while timing is on, kernels are launched directly instead.
struct Captured {
  hipGraphExec_t exec = nullptr;
  int gs = -1, gc = -1, gw = -1, rounds = -1;
  long long emin = 0;  // plain rounds: the binning threshold the graph's arguments carry
  uint32_t mask = ~0u;  // plain first chunks: pairs followed by k_bin_apply (bit i: pair i)
  bool matches(int s, int c, int w, int r, long long e = 0, uint32_t m = ~0u) const {
    return exec && gs == s && gc == c && gw == w && rounds == r && emin == e && mask == m;
  }
};

static void captured_free(Captured& c) {
  if (c.exec) (void)hipGraphExecDestroy(c.exec);
  c = Captured{};
}

struct KTime {
  int64_t launches = 0;
  double ms = 0;
  int64_t units = 0;
  int64_t entries = 0;
};

enum { HS_FREE = 0, HS_RUN = 1, HS_PUSHED = 2, HS_SWEEP = 3 };

struct SweepHdr {
  int32_t nseg;
  int32_t total;
  long long touch_total;
};

// Host side of a graph's batch engine.
struct BatchEngine {
  int B = 0;
  plc::BatchArgs args{};
  std::vector<void*> blocks;
  plc::Slot* slots_h = nullptr;      // pinned mirror of the slot array
  plc::SweepSeg* segs_h = nullptr;   // pinned sweep plan
  plc::Admit* adm_h = nullptr;       // pinned admission list
  plc::Admit* adm_d = nullptr;       // device admission list
  plc::BatchCtl* ctl_h = nullptr;    // pinned mirror of the control block
  SweepHdr* hdr_h = nullptr;         // pinned sweep header
  std::vector<int> state;            // HS_*
  std::vector<uint64_t> qid;
  std::vector<int> qbucket;          // compact: hint bucket of the slot's query
  std::vector<uint32_t> qflags;      // flags of the slot's query
  std::vector<Result> sweeping;      // result blocks filled by the sweep in flight
  std::deque<std::pair<uint64_t, plc_query>> queue;
  size_t bytes = 0;
  Captured round_g;                  // one round: plan, self, scatter, round end
  bool compact = false;              // PLC_STATE_COMPACT
  // dense layout: the slots' lists, slices of q*n (frontiers: (2q+k)*n)
  int32_t* d_fbuf = nullptr;
  int32_t* d_support = nullptr;
  int32_t* d_touched = nullptr;
  // compact layout: per slot, the running query's block and table capacity
  std::vector<void*> qblock;
  std::vector<int64_t> qcap;
  std::vector<int32_t> qgrows;       // growths of the slot's table
  std::vector<int64_t> qbound;       // touched bound of the slot's query
  std::vector<int> hold;             // hold flag last sent to the device
  std::vector<char> fresh;           // admitted this step: slots_h not read back yet
  plc::Grow* grow_h = nullptr;       // pinned grow records
  plc::Grow* grow_d = nullptr;
  int32_t* holds_h = nullptr;        // pinned hold updates
  int32_t* holds_d = nullptr;
  plc::ClearJob* clear_h = nullptr;  // pinned table clears of one step (2B)
  plc::ClearJob* clear_d = nullptr;
  // compact layout: running mean of the final touched count of finished
  // queries, per quarter decade of the work-bound scale 1/(alpha' eps); a
  // new query's first table is sized for it (fewer growth steps)
  std::map<int, double> touched_hint;
};

static int hint_bucket(const plc_query& q) {
  const double ap = q.rule == PLC_RULE_OPT ? 2.0 * q.alpha / (1.0 + q.alpha) : q.alpha;
  return (int)std::floor(4.0 * std::log10(1.0 / (ap * q.eps)));
}

}  // namespace

struct plc_graph {
  plc_ctx* ctx = nullptr;
  int64_t n = 0, arcs = 0, maxdeg = 0;
  size_t bytes = 0;
  std::vector<void*> blocks;
  std::vector<int32_t> deg;  // host copy of degrees, for query validation
  std::vector<int32_t> hotcode_h;  // staging for the hot codes at load
  PlainArgs args{};
  // launch shapes (workgroups per launch); 0 = context default
  int plain_self = 0, plain_scatter = 0, plain_sweep = 0;
  int batch_self = 0, batch_scatter = 0, batch_sweep = 0;
  BatchEngine* batch = nullptr;
  std::map<int, Captured> chunk_g;  // plain path: R rounds of (self, scatter), by R
  // plain path: a query's first chunk of R rounds, by (R << 32 | mask); its
  // pairs queue k_bin_apply as the mask says and report rounds that could
  // bin (a mask that comes back finds its graph still recorded)
  std::map<uint64_t, Captured> first_g;
  std::map<int64_t, Captured> sweep_g;  // plain path: the sweep, by sort bound (power of 2)
};

struct plc_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  Arena arena;
  plc_options opt{};
  Ctl* ctl_host = nullptr;  // pinned
  // plc_result_copy_many: pinned, device-mapped staging (jobs, then data),
  // grown as needed
  char* stage_h = nullptr;
  char* stage_d = nullptr;
  size_t stage_bytes = 0;
  std::map<uint64_t, Result> results;
  std::map<uint64_t, plc_graph*> inflight;  // submitted to a batch engine, not finished
  uint64_t next_id = 1;
  bool broken = false;
  std::set<plc_graph*> graphs;
  int num_cu = 256;
  int grid_self = 256, grid_scatter = 1024, grid_sweep = 512, grid_bin = 1024;
  double clock_ns = 10.0;         // nanoseconds per tick of the kernels' constant-rate clock
  uint32_t cur_flags = 0;         // plain path: flags of the running query
  int32_t cur_pipe = 0;           // plain path: plc_result_info.pipelined of the running query
  std::deque<int> round_hist;  // plain path: working self launches of the last queries
  std::deque<int> support_hist;  // plain path: support sizes of the last queries
  // plain path: Ctl::bin_pairs of the last queries whose first chunk reported
  // them (the pairs of a first chunk whose rounds could bin or pull)
  std::deque<uint32_t> pair_hist;
  std::chrono::steady_clock::time_point q_t0;  // plain path: start of the running query
  std::chrono::steady_clock::time_point next_t0;  // plain path: start of the queued next query
  hipEvent_t rb_event = nullptr;  // plain path: recorded after the running query's read-back
  std::vector<int32_t> work_log_h = std::vector<int32_t>(2 * plc::kMaxChunk);
  bool use_graphs = false;            // replay captured graphs (PLC_LAUNCH_GRAPH)
  hipStream_t cap_stream = nullptr;   // private stream that graphs are recorded on
  bool timing = false;
  std::vector<EventPair> ev_scatter, ev_self;
  EventPair ev_sweep;
  KTime t_scatter, t_self, t_sweep;
};

#define HIPCHK(ctx, expr)                       \
  do {                                          \
    hipError_t e_ = (expr);                     \
    if (e_ != hipSuccess) {                     \
      (ctx)->broken = true;                     \
      return PLC_E_HIP;                         \
    }                                           \
  } while (0)

extern "C" const char* plc_status_str(plc_status s) {
  switch (s) {
    case PLC_OK: return "ok";
    case PLC_E_INVALID: return "invalid argument";
    case PLC_E_NOMEM: return "arena exhausted";
    case PLC_E_BUSY: return "busy";
    case PLC_E_NOTREADY: return "not ready";
    case PLC_E_NOTFOUND: return "not found";
    case PLC_E_LIMIT: return "round limit reached";
    case PLC_E_HIP: return "HIP runtime error";
    default: return "unknown status";
  }
}

extern "C" plc_status plc_init(plc_ctx** out, int32_t device, void* dev_arena, size_t arena_bytes,
                               void* hip_stream, const plc_options* opt) {
  if (!out || !dev_arena || arena_bytes < 4096) return PLC_E_INVALID;
  if (reinterpret_cast<uintptr_t>(dev_arena) % Arena::kAlign) return PLC_E_INVALID;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return PLC_E_INVALID;
  if (hipSetDevice(device) != hipSuccess) return PLC_E_HIP;
  plc_ctx* c = new (std::nothrow) plc_ctx();
  if (!c) return PLC_E_NOMEM;
  c->device = device;
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->arena.reset(dev_arena, arena_bytes);
  if (opt) c->opt = *opt;
  if (c->opt.max_rounds <= 0) c->opt.max_rounds = 1 << 20;
  if (c->opt.batch_slots <= 0 || c->opt.batch_slots > 1024) c->opt.batch_slots = 256;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
    c->num_cu = prop.multiProcessorCount;
  c->grid_self = c->num_cu;
  c->grid_scatter = 4 * c->num_cu;
  c->grid_sweep = 2 * c->num_cu;
  c->grid_bin = 4 * c->num_cu;
  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) == hipSuccess && khz > 0)
    c->clock_ns = 1e6 / (double)khz;
  if (hipHostMalloc(reinterpret_cast<void**>(&c->ctl_host), sizeof(Ctl), hipHostMallocDefault) !=
      hipSuccess) {
    delete c;
    return PLC_E_HIP;
  }
  std::memset(c->ctl_host, 0, sizeof(Ctl));
  // The caller's stream may be the null stream, which cannot be captured, so
  // graphs are recorded on a stream of our own and replayed on the caller's.
  if (c->opt.launch_mode == PLC_LAUNCH_GRAPH &&
      hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) == hipSuccess)
    c->use_graphs = true;
  *out = c;
  return PLC_OK;
}

static void batch_free(plc_ctx* ctx, plc_graph* g);

static void graph_captures_free(plc_graph* g) {
  for (auto& kv : g->chunk_g) captured_free(kv.second);
  g->chunk_g.clear();
  for (auto& kv : g->first_g) captured_free(kv.second);
  g->first_g.clear();
  for (auto& kv : g->sweep_g) captured_free(kv.second);
  g->sweep_g.clear();
}

static void free_events(plc_ctx* c) {
  for (auto& e : c->ev_scatter) { (void)hipEventDestroy(e.a); (void)hipEventDestroy(e.b); }
  for (auto& e : c->ev_self) { (void)hipEventDestroy(e.a); (void)hipEventDestroy(e.b); }
  c->ev_scatter.clear();
  c->ev_self.clear();
  if (c->ev_sweep.a) { (void)hipEventDestroy(c->ev_sweep.a); (void)hipEventDestroy(c->ev_sweep.b); }
  c->ev_sweep = EventPair{};
  if (c->rb_event) (void)hipEventDestroy(c->rb_event);
  c->rb_event = nullptr;
}

extern "C" plc_status plc_destroy(plc_ctx* ctx) {
  if (!ctx) return PLC_E_INVALID;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  for (plc_graph* g : ctx->graphs) {
    batch_free(ctx, g);
    graph_captures_free(g);
    delete g;
  }
  free_events(ctx);
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  if (ctx->ctl_host) (void)hipHostFree(ctx->ctl_host);
  if (ctx->stage_h) (void)hipHostFree(ctx->stage_h);
  delete ctx;
  return PLC_OK;
}

// ---------------------------------------------------------------- graphs

static bool host_validate(int64_t n, const std::vector<int64_t>& off, const int32_t* nbr) {
  unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::atomic<bool> ok{true};
  std::vector<std::thread> th;
  for (unsigned t = 0; t < nt; t++) {
    th.emplace_back([&, t]() {
      for (int64_t v = t; v < n && ok.load(std::memory_order_relaxed); v += nt) {
        for (int64_t e = off[v]; e < off[v + 1]; e++) {
          int64_t w = nbr[e];
          if (w < 0 || w >= n || w == v || (e > off[v] && nbr[e - 1] >= w)) { ok = false; break; }
          // symmetric: v must appear in w's sorted row
          const int32_t* lo = nbr + off[w];
          const int32_t* hi = nbr + off[w + 1];
          const int32_t* it = std::lower_bound(lo, hi, (int32_t)v);
          if (it == hi || *it != v) { ok = false; break; }
        }
      }
    });
  }
  for (auto& x : th) x.join();
  return ok.load();
}

static void graph_release_blocks(plc_ctx* ctx, plc_graph* g) {
  for (void* b : g->blocks) ctx->arena.release(b);
  g->blocks.clear();
}

extern "C" plc_status plc_graph_load(plc_ctx* ctx, int64_t n, int64_t num_arcs,
                                     const void* offsets, int32_t offsets_bits,
                                     const int32_t* nbrs, uint32_t flags, plc_graph** out) {
  if (!ctx || !out || !offsets || n <= 0 || num_arcs < 0) return PLC_E_INVALID;
  if (ctx->broken) return PLC_E_HIP;
  if (offsets_bits != 32 && offsets_bits != 64) return PLC_E_INVALID;
  if (num_arcs > 0 && !nbrs) return PLC_E_INVALID;
  if (n >= (int64_t)INT32_MAX || num_arcs >= (int64_t)1 << 40) return PLC_E_INVALID;
  (void)hipSetDevice(ctx->device);

  std::vector<int64_t> off((size_t)n + 1);
  if (offsets_bits == 64) {
    std::memcpy(off.data(), offsets, sizeof(int64_t) * ((size_t)n + 1));
  } else {
    const int32_t* o32 = static_cast<const int32_t*>(offsets);
    for (int64_t i = 0; i <= n; i++) off[i] = o32[i];
  }
  if (off[0] != 0 || off[n] != num_arcs) return PLC_E_INVALID;
  int64_t maxdeg = 0;
  std::vector<int32_t> deg((size_t)n);
  for (int64_t v = 0; v < n; v++) {
    int64_t d = off[v + 1] - off[v];
    if (d < 0 || d >= INT32_MAX) return PLC_E_INVALID;
    deg[v] = (int32_t)d;
    maxdeg = std::max(maxdeg, d);
  }
  // Neighbour ids index per-vertex arrays on the device: always range-checked.
  {
    bool ok = true;
    for (int64_t e = 0; e < num_arcs; e++) {
      uint32_t w = (uint32_t)nbrs[e];
      ok &= w < (uint64_t)n;
    }
    if (!ok) return PLC_E_INVALID;
  }
  if ((flags & PLC_GRAPH_VALIDATE) && !host_validate(n, off, nbrs)) return PLC_E_INVALID;

  plc_graph* g = new (std::nothrow) plc_graph();
  if (!g) return PLC_E_NOMEM;
  g->ctx = ctx;
  g->n = n;
  g->arcs = num_arcs;
  g->maxdeg = maxdeg;
  g->deg.swap(deg);

  bool nomem = false;
  auto take = [&](size_t bytes) -> void* {
    void* p = ctx->arena.alloc(bytes);
    if (!p) { nomem = true; return nullptr; }
    g->blocks.push_back(p);
    g->bytes += (bytes + Arena::kAlign - 1) & ~(Arena::kAlign - 1);
    return p;
  };
  const size_t N = (size_t)n;
  const size_t nscan = N / plc::kScanBlock + 2;
  const size_t ntile = (size_t)num_arcs / plc::kEdgeTile + 2;
  PlainArgs& a = g->args;
  a.n = n;
  a.vol_total = num_arcs;
  a.off = static_cast<int64_t*>(take(8 * (N + 1)));
  a.nbr = static_cast<int32_t*>(take(4 * std::max<size_t>((size_t)num_arcs, 1)));
  a.vr = static_cast<plc::VRec*>(take(sizeof(plc::VRec) * N));
  a.p = static_cast<double*>(take(8 * N));
  a.ctl = static_cast<Ctl*>(take(sizeof(Ctl)));
  a.fbuf0 = static_cast<int32_t*>(take(4 * N));
  a.fbuf1 = static_cast<int32_t*>(take(4 * N));
  a.coef = static_cast<double*>(take(8 * N));
  a.estart = static_cast<int64_t*>(take(8 * N));
  a.rowp = static_cast<int64_t*>(take(8 * N));
  a.tile_start = static_cast<int32_t*>(take(4 * ntile));
  a.tile_cap = (int64_t)ntile;
  a.desc_cap = (int32_t)nscan;
  for (int s = 0; s < plc::NUM_SCANS; s++)
    a.desc[s] = static_cast<unsigned long long*>(take(2 * 8 * nscan));
  a.support = static_cast<int32_t*>(take(4 * N));
  a.touched = static_cast<int32_t*>(take(4 * N));
  a.sbuf[0] = static_cast<plc::SortElem*>(take(sizeof(plc::SortElem) * N));
  a.sbuf[1] = static_cast<plc::SortElem*>(take(sizeof(plc::SortElem) * N));
  a.sdeg = static_cast<int32_t*>(take(4 * N));
  a.svol = static_cast<int64_t*>(take(8 * N));
  a.scnt = static_cast<int32_t*>(take(4 * N));
  a.sp = static_cast<double*>(take(8 * N));
  a.sid = static_cast<int32_t*>(take(4 * N));
  a.rid = static_cast<int32_t*>(take(4 * N));
  a.rval = static_cast<double*>(take(8 * N));
  a.bbest = static_cast<long long*>(take(24 * nscan));
  int32_t* hot_ids = static_cast<int32_t*>(take(4 * (size_t)plc::kHot));
  int32_t* hotcode = static_cast<int32_t*>(take(4 * N));
  a.hot_ids = hot_ids;
  a.hotcode = hotcode;
  a.hk_r1 = static_cast<double*>(take(8 * N));
  a.hk_tl[0] = a.touched;
  a.hk_tl[1] = static_cast<int32_t*>(take(4 * N));
  a.hk_tl[2] = static_cast<int32_t*>(take(4 * N));
  a.hk_B = static_cast<double*>(take(8 * (size_t)(plc::kHkMaxLevels + 1)));
  a.work_log = static_cast<int32_t*>(take(4 * 2 * (size_t)plc::kMaxChunk));
  // Destination bins of the binned scatter: whole kBinGran-vertex blocks, at
  // most kBinWidth vertices and about 1/1024 of the volume each (the volume
  // target doubles until fewer than kMaxBins bins result); off for graphs of
  // more than kBinMaxVertices vertices or when the context turned it off.
  std::vector<int32_t> bin_of_blk, bin_lo;
  std::vector<long long> bin_vol;
  const int64_t nblk = (n + plc::kBinGran - 1) / plc::kBinGran;
  const bool bins_on = ctx->opt.bin_min_edges >= 0 &&
                       n <= plc::kBinMaxVertices;
  static_assert(plc::kBinMaxVertices / plc::kBinWidth <= plc::kMaxBins * 3 / 4,
                "the width bound alone leaves room for the volume bins");
  if (bins_on) {
    long long vt = std::max<long long>(1, num_arcs / 1024);
    for (;;) {
      bin_of_blk.assign((size_t)nblk, 0);
      bin_lo.clear();
      bin_vol.clear();
      long long cw = 0, cv = 0;
      for (int64_t k = 0; k < nblk; k++) {
        const int64_t v0 = k * plc::kBinGran, v1 = std::min<int64_t>(n, v0 + plc::kBinGran);
        const long long vol = (long long)(off[v1] - off[v0]);
        if (bin_lo.empty() || cw + plc::kBinGran > plc::kBinWidth || (cw > 0 && cv + vol > vt)) {
          bin_lo.push_back((int32_t)v0);
          bin_vol.push_back(0);
          cw = 0;
          cv = 0;
        }
        bin_of_blk[(size_t)k] = (int32_t)bin_lo.size() - 1;
        cw += plc::kBinGran;
        cv += vol;
        bin_vol.back() += vol;
      }
      bin_lo.push_back((int32_t)std::min<int64_t>((int64_t)INT32_MAX, nblk * plc::kBinGran));
      if ((int)bin_vol.size() < plc::kMaxBins) break;
      vt *= 2;
    }
    const int nb = (int)bin_vol.size();
    const int64_t emax = std::min<int64_t>(std::max<int64_t>(num_arcs, 1), plc::kBinEmax);
    a.bin_cmax = (int32_t)((emax + plc::kBinChunk - 1) / plc::kBinChunk);
    a.bin_of_blk = static_cast<int32_t*>(take(4 * (size_t)nblk));
    a.bin_lo = static_cast<int32_t*>(take(4 * (size_t)(nb + 1)));
    a.bin_vol = static_cast<long long*>(take(8 * (size_t)nb));
    a.bin_T = static_cast<int32_t*>(take(4 * (size_t)(nb + 1) * (size_t)a.bin_cmax));
    a.bin_pairs = static_cast<int2*>(take(8 * (size_t)a.bin_cmax * plc::kBinChunk));
    a.nbins = nb;
    a.bin_emin = ctx->opt.bin_min_edges > 0 ? ctx->opt.bin_min_edges : plc::kBinEmin;
    // the pull form for rounds over at least half the arcs (records cleared
    // by the graph init kernel)
    a.pull = static_cast<plc::PullRec*>(take(sizeof(plc::PullRec) * (size_t)n));
    a.pull_epoch = static_cast<unsigned*>(take(256));
    a.pull_emin = std::max<long long>(1, (num_arcs + 1) / 2);
  } else {
    a.nbins = 0;
    a.bin_cmax = 0;
    a.bin_emin = 0;
    a.pull = nullptr;
    a.pull_epoch = nullptr;
    a.pull_emin = 0;
  }
  if (nomem) {
    graph_release_blocks(ctx, g);
    delete g;
    return PLC_E_NOMEM;
  }
  hipStream_t s = ctx->stream;
  auto fail = [&]() {
    ctx->broken = true;
    graph_release_blocks(ctx, g);
    delete g;
    return PLC_E_HIP;
  };
  if (hipMemcpyAsync((void*)a.off, off.data(), 8 * (N + 1), hipMemcpyHostToDevice, s) != hipSuccess)
    return fail();
  if (num_arcs > 0 &&
      hipMemcpyAsync((void*)a.nbr, nbrs, 4 * (size_t)num_arcs, hipMemcpyHostToDevice, s) !=
          hipSuccess)
    return fail();
  // Hot destinations: the kHot highest-degree vertices (degree >= 32, ties by
  // id).  Their hot index lives in the idle rank field of the state record.
  {
    std::vector<int32_t> order(N);
    for (size_t v = 0; v < N; v++) order[v] = (int32_t)v;
    const size_t H = std::min<size_t>(N, (size_t)plc::kHot);
    auto by_deg = [&](int32_t x, int32_t y) {
      return g->deg[x] != g->deg[y] ? g->deg[x] > g->deg[y] : x < y;
    };
    std::partial_sort(order.begin(), order.begin() + H, order.end(), by_deg);
    g->hotcode_h.assign(N, 0);
    std::vector<int32_t> ids(plc::kHot, 0);
    for (size_t j = 0; j < H && g->deg[order[j]] >= 32; j++) {
      ids[j] = order[j];
      g->hotcode_h[order[j]] = -(int32_t)(j + 1);
    }
    if (hipMemcpyAsync(hot_ids, ids.data(), 4 * (size_t)plc::kHot, hipMemcpyHostToDevice, s) !=
            hipSuccess ||
        hipMemcpyAsync(hotcode, g->hotcode_h.data(), 4 * N, hipMemcpyHostToDevice, s) != hipSuccess)
      return fail();
    if (hipStreamSynchronize(s) != hipSuccess) return fail();
    g->hotcode_h.clear();
    g->hotcode_h.shrink_to_fit();
  }
  if (a.nbins > 0 &&
      (hipMemcpyAsync((void*)a.bin_of_blk, bin_of_blk.data(), 4 * bin_of_blk.size(),
                      hipMemcpyHostToDevice, s) != hipSuccess ||
       hipMemcpyAsync((void*)a.bin_lo, bin_lo.data(), 4 * bin_lo.size(), hipMemcpyHostToDevice,
                      s) != hipSuccess ||
       hipMemcpyAsync((void*)a.bin_vol, bin_vol.data(), 8 * bin_vol.size(),
                      hipMemcpyHostToDevice, s) != hipSuccess))
    return fail();
  if (hipMemsetAsync(a.ctl, 0, sizeof(Ctl), s) != hipSuccess) return fail();
  for (int k = 0; k < plc::NUM_SCANS; k++)
    if (hipMemsetAsync(a.desc[k], 0, 2 * 8 * nscan, s) != hipSuccess) return fail();
  if (plc::launch_graph_init(s, a) != hipSuccess) return fail();
  if (hipStreamSynchronize(s) != hipSuccess) return fail();
  ctx->graphs.insert(g);
  *out = g;
  return PLC_OK;
}

extern "C" plc_status plc_graph_free(plc_ctx* ctx, plc_graph* g) {
  if (!ctx || !g || !ctx->graphs.count(g)) return PLC_E_INVALID;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  batch_free(ctx, g);
  graph_captures_free(g);
  graph_release_blocks(ctx, g);
  ctx->graphs.erase(g);
  delete g;
  return PLC_OK;
}

extern "C" plc_status plc_graph_info_get(const plc_graph* g, plc_graph_info* out) {
  if (!g || !out) return PLC_E_INVALID;
  out->n = g->n;
  out->arcs = g->arcs;
  out->max_degree = g->maxdeg;
  out->bytes = (int64_t)g->bytes;
  return PLC_OK;
}

// ---------------------------------------------------------------- queries

static bool query_ok(const plc_graph* g, const plc_query& q) {
  if (q.seed < 0 || q.seed >= g->n) return false;
  if (g->deg[q.seed] < 1) return false;
  if (!(q.alpha > 0.0 && q.alpha < 1.0)) return false;
  if (!std::isfinite(q.eps) || !(q.eps >= 1e-250)) return false;
  if (q.rule != PLC_RULE_OPT && q.rule != PLC_RULE_ORIG) return false;
  if ((q.flags & ~PLC_QF_ALL) != 0u) return false;
  return true;
}

static hipError_t ev_pair(EventPair& e) {
  if (e.a) return hipSuccess;
  hipError_t r = hipEventCreate(&e.a);
  if (r != hipSuccess) return r;
  return hipEventCreate(&e.b);
}

static int shape(int tuned, int dflt) { return tuned > 0 ? tuned : dflt; }

// Record body(stream) into c.exec.  On failure the context stops using graphs
// (direct launches run the same kernels) and false is returned.
template <class F>
static bool capture(plc_ctx* ctx, Captured& c, F&& body) {
  hipStream_t cs = ctx->cap_stream;
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed);
  if (e == hipSuccess) {
    const hipError_t eb = body(cs);
    hipGraph_t graph = nullptr;
    const hipError_t ee = hipStreamEndCapture(cs, &graph);
    e = eb != hipSuccess ? eb : ee;
    if (e == hipSuccess) e = hipGraphInstantiate(&c.exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    c.exec = nullptr;
    captured_free(c);
    ctx->use_graphs = false;
    return false;
  }
  return true;
}

// The launch pairs of a first chunk that queue k_bin_apply: those whose
// rounds could bin or pull in any of the last queries (all of them until a
// query has reported, or when the context fixed the binning threshold;
// pairs from 32 on always queue it).  Binned rounds sit
// at the same few pairs from query to query (those of the largest frontiers),
// and k_bin_apply exits at once after every other round at the cost of a
// dispatch; a round at a pair without it takes the atomic form and reports
// itself, so the next first chunks queue k_bin_apply there.
constexpr size_t kFirstGraphs = 64;  // first-chunk graphs kept per graph

static uint32_t first_chunk_mask(const plc_ctx* ctx) {
  // (only with the binning threshold left to the library: a threshold the
  // caller fixed bins every round of that size)
  if (ctx->opt.bin_min_edges != 0 || ctx->pair_hist.empty()) return ~0u;
  uint32_t m = 0;
  for (uint32_t b : ctx->pair_hist) m |= b;
  return m;
}

// Graph of R plain rounds (self, scatter).  first: a query's first chunk,
// whose pair i reports in Ctl::bin_pairs a round that could bin or pull and
// queues k_bin_apply only where bit i of first_chunk_mask is set (always
// from pair 32 on).
static Captured* plain_chunk_graph(plc_ctx* ctx, plc_graph* g, int R, bool first = false) {
  const int gs = shape(g->plain_self, ctx->grid_self);
  const int gc = shape(g->plain_scatter, ctx->grid_scatter);
  const uint32_t mask = first ? first_chunk_mask(ctx) : ~0u;
  const uint64_t key = ((uint64_t)R << 32) | mask;
  if (first && g->first_g.size() >= kFirstGraphs && !g->first_g.count(key)) {
    for (auto& kv : g->first_g) captured_free(kv.second);  // bound the recorded masks
    g->first_g.clear();
  }
  Captured& c = first ? g->first_g[key] : g->chunk_g[R];
  if (c.matches(gs, gc, 0, R, g->args.bin_emin, mask)) return &c;
  captured_free(c);
  c.gs = gs;
  c.gc = gc;
  c.gw = 0;
  c.rounds = R;
  c.emin = g->args.bin_emin;
  c.mask = mask;
  const PlainArgs& a = g->args;
  const bool ok = capture(ctx, c, [&](hipStream_t cs) -> hipError_t {
    hipError_t r;
    for (int i = 0; i < R; i++) {
      const bool tracked = first && i < 32;
      const bool apply = !tracked || ((mask >> i) & 1u);
      if ((r = plc::launch_self(cs, a, gs)) != hipSuccess) return r;
      if ((r = plc::launch_scatter(cs, a, gc, nullptr, nullptr, -1, ctx->grid_bin,
                                   tracked ? i : -1, apply)) != hipSuccess)
        return r;
    }
    return hipSuccess;
  });
  return ok ? &c : nullptr;
}

// Graph of the plain sweep sequence for supports of at most max_count
// vertices (a power of 2: it sets the sort's launches, one rank merge up to
// 65536 elements, merge passes above).
static Captured* plain_sweep_graph(plc_ctx* ctx, plc_graph* g, int64_t max_count) {
  const int gw = shape(g->plain_sweep, ctx->grid_sweep);
  Captured& c = g->sweep_g[max_count];
  if (c.matches(0, 0, gw, 0)) return &c;
  captured_free(c);
  c.gs = 0;
  c.gc = 0;
  c.gw = gw;
  c.rounds = 0;
  const PlainArgs& a = g->args;
  const bool ok = capture(ctx, c, [&](hipStream_t cs) -> hipError_t {
    return plc::launch_sweep(cs, a, gw, max_count);
  });
  return ok ? &c : nullptr;
}

// Queue `rounds` rounds as direct launches; with timing on, each kernel
// carries start and stop events on its own dispatch timestamps
// (ctx->ev_self[i], ctx->ev_scatter[i] for round i of the chunk) and marks
// a.work_log[2i] / [2i + 1] when it did work.  first: a query's first chunk,
// with the same k_bin_apply launches and reports as its graph (so the timed
// launches are the ones the graphs replay).

static hipError_t queue_rounds(plc_ctx* ctx, const plc_graph* g, int rounds, bool beta,
                               bool first = false) {
  const PlainArgs& a = g->args;
  hipStream_t s = ctx->stream;
  const int gs = shape(g->plain_self, ctx->grid_self);
  const int gc = shape(g->plain_scatter, ctx->grid_scatter);
  const int gw = shape(g->plain_sweep, ctx->grid_sweep);
  const uint32_t mask = first && !beta ? first_chunk_mask(ctx) : ~0u;
  for (int i = 0; i < rounds; i++) {
    hipError_t r;
    const bool tracked = first && !beta && i < 32;
    const int pair = tracked ? i : -1;
    const bool apply = !tracked || ((mask >> i) & 1u);
    if (beta && (r = plc::launch_beta_pre(s, a, gw, g->n)) != hipSuccess) return r;
    if (ctx->timing) {
      size_t k = (size_t)i;
      while (ctx->ev_self.size() <= k) ctx->ev_self.emplace_back();
      while (ctx->ev_scatter.size() <= k) ctx->ev_scatter.emplace_back();
      if ((r = ev_pair(ctx->ev_self[k])) != hipSuccess) return r;
      if ((r = ev_pair(ctx->ev_scatter[k])) != hipSuccess) return r;
      if ((r = plc::launch_self(s, a, gs, ctx->ev_self[k].a, ctx->ev_self[k].b, i)) != hipSuccess)
        return r;
      if ((r = plc::launch_scatter(s, a, gc, ctx->ev_scatter[k].a, ctx->ev_scatter[k].b, i,
                                   ctx->grid_bin, pair, apply)) != hipSuccess)
        return r;
    } else {
      if ((r = plc::launch_self(s, a, gs)) != hipSuccess) return r;
      if ((r = plc::launch_scatter(s, a, gc, nullptr, nullptr, -1, ctx->grid_bin, pair,
                                   apply)) != hipSuccess)
        return r;
    }
    if (beta && (r = plc::launch_beta_post(s, a, gw)) != hipSuccess) return r;
  }
  return hipSuccess;
}

static plc_status sweep_and_record(plc_ctx* ctx, plc_graph* g, uint64_t* id_out,
                                   plc_result_info* info_out);
static plc_status record_result(plc_ctx* ctx, plc_graph* g, uint64_t* id_out,
                                plc_result_info* info_out);
static hipError_t queue_sweep(plc_ctx* ctx, plc_graph* g, int64_t bound);

// One plain query: from q.seed, or, with set non-null, from the nset
// distinct seeds in set (q.seed is then ignored).
// Push: chunks of (self, scatter) launch pairs, each followed by a
// read-back of the control block.  A self launch may run several small
// rounds, and pairs queued past the end of the push exit at once but still
// cost a dispatch each, so the first chunk is the upper quartile of the
// last queries' counts of working self launches and later chunks are short.
static int first_chunk(const plc_ctx* ctx) {
  int chunk = 16;
  if (!ctx->round_hist.empty()) {
    std::vector<int> hs(ctx->round_hist.begin(), ctx->round_hist.end());
    std::sort(hs.begin(), hs.end());
    chunk = hs[(3 * hs.size()) / 4];
  }
  return std::max(2, std::min(plc::kMaxChunk, chunk));
}

// Queue query q's guarded initialisation and first chunk behind the running
// query's read-back, so that the GPU works on it while the host takes that
// read-back.  Returns the chunk's pair count (0: nothing queued, -1: error).
static int prelaunch(plc_ctx* ctx, plc_graph* g, const plc_query& q) {
  if (!ctx->use_graphs || ctx->timing) return 0;
  const int R = first_chunk(ctx);
  Captured* cg = plain_chunk_graph(ctx, g, R, true);
  if (!cg) return 0;
  hipStream_t s = ctx->stream;
  if (plc::launch_query_init_guarded(s, g->args, q.seed, (int32_t)q.rule, q.alpha, q.eps,
                                     ctx->opt.max_rounds) != hipSuccess ||
      hipGraphLaunch(cg->exec, s) != hipSuccess) {
    ctx->broken = true;
    return -1;
  }
  return R;
}

// One plain query: from q.seed, or, with set non-null, from the nset
// distinct seeds in set (q.seed is then ignored).  pre > 0: its guarded
// initialisation and first chunk of pre pairs are already queued.  next
// (may be null): the following query, queued behind this one's first
// read-back; *next_pre receives its chunk (0 when it must start afresh).
static plc_status run_one(plc_ctx* ctx, plc_graph* g, const plc_query& q, uint64_t* id_out,
                          plc_result_info* info_out, const int32_t* set = nullptr,
                          int32_t nset = 0, double beta = 1.0, int pre = 0,
                          const plc_query* next = nullptr, int* next_pre = nullptr,
                          int pipe_in = 0, int* next_pipe = nullptr) {
  ctx->q_t0 = pre > 0 ? ctx->next_t0 : std::chrono::steady_clock::now();
  ctx->cur_flags = q.flags;
  ctx->cur_pipe = pipe_in;
  if (next_pre) *next_pre = 0;
  if (next_pipe) *next_pipe = 0;
  hipStream_t s = ctx->stream;
  const PlainArgs& a = g->args;
  if (pre > 0) {
    // (queued by the previous query's run)
  } else if (set) {
    HIPCHK(ctx, hipMemcpyAsync(a.fbuf0, set, 4 * (size_t)nset, hipMemcpyHostToDevice, s));
    HIPCHK(ctx, plc::launch_query_init_set(s, a, nset, (int32_t)q.rule, q.alpha, q.eps,
                                           ctx->opt.max_rounds));
  } else {
    HIPCHK(ctx, plc::launch_query_init(s, a, q.seed, (int32_t)q.rule, q.alpha, q.eps,
                                       ctx->opt.max_rounds, beta));
  }
  const bool use_beta = beta < 1.0;
  int queued = 0;
  int chunk = pre > 0 ? pre : first_chunk(ctx);
  // Each chunk is followed by the sweep, queued for the largest recent
  // support (its kernels exit at once unless the push has ended with a
  // support within that bound), so a typical query needs one read-back.
  int64_t spec_bound = 0;
  if (!ctx->timing && !use_beta && !ctx->support_hist.empty()) {
    spec_bound = 1024;
    const int64_t mx = *std::max_element(ctx->support_hist.begin(), ctx->support_hist.end());
    while (spec_bound < mx) spec_bound <<= 1;
  }
  bool swept = false;
  bool reports = pre > 0;  // the first chunk reports Ctl::bin_pairs
  Ctl& h = *ctx->ctl_host;
  for (bool first = true;; first = false) {
    const int R = chunk;
    if (!(first && pre > 0)) {
      // while timing is on, rounds are launched directly (graphs carry no
      // events) (the beta variant's rounds are launched directly too)
      Captured* cg = ctx->use_graphs && !ctx->timing && !use_beta
                         ? plain_chunk_graph(ctx, g, R, first)
                         : nullptr;
      if (first && !use_beta) reports = true;  // graph or direct launches, both tracked
      if (ctx->timing) HIPCHK(ctx, hipMemsetAsync(a.work_log, 0, 4 * 2 * (size_t)R, s));
      if (cg)
        HIPCHK(ctx, hipGraphLaunch(cg->exec, s));
      else
        HIPCHK(ctx, queue_rounds(ctx, g, R, use_beta, first));
    }
    if (spec_bound) HIPCHK(ctx, queue_sweep(ctx, g, spec_bound));
    const EventPair* ev_s = ctx->ev_self.data();
    const EventPair* ev_c = ctx->ev_scatter.data();
    HIPCHK(ctx, hipMemcpyAsync(&h, a.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    if (ctx->timing)
      HIPCHK(ctx, hipMemcpyAsync(ctx->work_log_h.data(), a.work_log, 4 * 2 * (size_t)R,
                                 hipMemcpyDeviceToHost, s));
    int held = 0;  // pairs of the next query's chunk queued behind this read-back
    if (first && next && spec_bound && !set && !use_beta) {
      if (!ctx->rb_event &&
          hipEventCreateWithFlags(&ctx->rb_event, hipEventDisableTiming) != hipSuccess)
        ctx->rb_event = nullptr;
      if (ctx->rb_event) {
        HIPCHK(ctx, hipEventRecord(ctx->rb_event, s));
        held = prelaunch(ctx, g, *next);
        if (held < 0) return PLC_E_HIP;
      }
    }
    if (held > 0)
      HIPCHK(ctx, hipEventSynchronize(ctx->rb_event));
    else
      HIPCHK(ctx, hipStreamSynchronize(s));
    if (held > 0) {
      if (h.status == plc::ST_SWEPT) {
        // the next query started behind this one: its time counts from here,
        // when this one is known to be done
        if (next_pre) *next_pre = held;
        if (next_pipe) *next_pipe = 1;
        ctx->next_t0 = std::chrono::steady_clock::now();
      } else {
        // its initialisation stood aside and the chunk continued this query's
        // push: wait for it and read the state again; the next query starts
        // afresh later
        HIPCHK(ctx, hipMemcpyAsync(&h, a.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
        HIPCHK(ctx, hipStreamSynchronize(s));
        if (!h.init_held) {  // unexpected: the guard let a query start over this one
          ctx->broken = true;
          return PLC_E_HIP;
        }
        if (next_pipe) *next_pipe = 2;
        queued += held;
      }
    }
    if (ctx->timing) {
      // only the launches that did work count (pairs past the end of the
      // push, and scatters after a self launch that ran the rounds itself,
      // exit at once)
      float ms = 0;
      for (int i = 0; i < R; i++) {
        if (ctx->work_log_h[2 * i + 1]) {
          HIPCHK(ctx, hipEventElapsedTime(&ms, ev_c[i].a, ev_c[i].b));
          ctx->t_scatter.ms += ms;
          ctx->t_scatter.launches++;
        }
        if (ctx->work_log_h[2 * i]) {
          HIPCHK(ctx, hipEventElapsedTime(&ms, ev_s[i].a, ev_s[i].b));
          ctx->t_self.ms += ms;
          ctx->t_self.launches++;
        }
      }
    }
    queued += R;
    if (h.status == plc::ST_SWEPT) { swept = true; break; }  // pushed and swept
    if (h.status == plc::ST_LIMIT) break;  // watchdog: sweep the partial p
    if (h.status != plc::ST_PUSH || h.fault) {  // unexpected state: device-side fault
      ctx->broken = true;
      return PLC_E_HIP;
    }
    if (h.cnt[h.round & 1] == 0) break;     // next frontier empty: the push is done
    chunk = std::max(2, std::min(64, queued / 3));
  }
  ctx->round_hist.push_back(h.steps);
  if (ctx->round_hist.size() > 16) ctx->round_hist.pop_front();
  ctx->support_hist.push_back(swept ? h.N : h.support_cnt);
  if (ctx->support_hist.size() > 16) ctx->support_hist.pop_front();
  if (reports) {
    ctx->pair_hist.push_back(h.bin_pairs);
    if (ctx->pair_hist.size() > 16) ctx->pair_hist.pop_front();
  }
  if (swept) return record_result(ctx, g, id_out, info_out);
  return sweep_and_record(ctx, g, id_out, info_out);
}

// Queue the plain sweep for supports of at most `bound` vertices (a power
// of 2: it sets the sort's launches); with timing on, between the context's
// sweep events.
static hipError_t queue_sweep(plc_ctx* ctx, plc_graph* g, int64_t bound) {
  hipStream_t s = ctx->stream;
  Captured* sg = ctx->use_graphs && !ctx->timing ? plain_sweep_graph(ctx, g, bound) : nullptr;
  if (sg) return hipGraphLaunch(sg->exec, s);
  hipError_t r;
  if (ctx->timing) {
    if ((r = ev_pair(ctx->ev_sweep)) != hipSuccess) return r;
    if ((r = hipEventRecord(ctx->ev_sweep.a, s)) != hipSuccess) return r;
  }
  r = plc::launch_sweep(s, g->args, shape(g->plain_sweep, ctx->grid_sweep), bound);
  if (r != hipSuccess) return r;
  if (ctx->timing) return hipEventRecord(ctx->ev_sweep.b, s);
  return hipSuccess;
}

// After a plain push (the control block read back into ctx->ctl_host):
// run the sweep, then record the result.
static plc_status sweep_and_record(plc_ctx* ctx, plc_graph* g, uint64_t* id_out,
                                   plc_result_info* info_out) {
  hipStream_t s = ctx->stream;
  const PlainArgs& a = g->args;
  Ctl& h = *ctx->ctl_host;
  int64_t bound = 1024;
  while (bound < h.support_cnt) bound <<= 1;
  HIPCHK(ctx, queue_sweep(ctx, g, bound));
  HIPCHK(ctx, hipMemcpyAsync(&h, a.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
  HIPCHK(ctx, hipStreamSynchronize(s));
  return record_result(ctx, g, id_out, info_out);
}

// After a plain sweep (the control block read back into ctx->ctl_host):
// take the result block, sized from the sweep's counts (support N, nonzeros
// of r), queue the copy of the results into it and record the result.
// Without room for the block the query reports PLC_E_NOMEM.
static plc_status record_result(plc_ctx* ctx, plc_graph* g, uint64_t* id_out,
                                plc_result_info* info_out) {
  hipStream_t s = ctx->stream;
  const PlainArgs& a = g->args;
  Ctl& h = *ctx->ctl_host;
  if (h.status != plc::ST_SWEPT || h.fault || h.N < 0 || h.N > g->n || h.rnnz < 0 ||
      h.rnnz > g->n) {  // unexpected state: device-side fault
    ctx->broken = true;
    return PLC_E_HIP;
  }
  const size_t N = (size_t)h.N;
  const size_t R = (ctx->cur_flags & PLC_QF_NO_RESIDUAL) ? 0 : (size_t)h.rnnz;
  const size_t off_p = (4 * N + 255) & ~(size_t)255;
  const size_t off_rid = off_p + ((8 * N + 255) & ~(size_t)255);
  const size_t off_rval = off_rid + ((4 * R + 255) & ~(size_t)255);
  Result res;
  res.block = ctx->arena.alloc(off_rval + 8 * R);
  if (res.block) {
    char* b = static_cast<char*>(res.block);
    res.ids = reinterpret_cast<int32_t*>(b);
    res.p = reinterpret_cast<double*>(b + off_p);
    res.rid = reinterpret_cast<int32_t*>(b + off_rid);
    res.rval = reinterpret_cast<double*>(b + off_rval);
    HIPCHK(ctx, plc::launch_copy_result(s, a, res.ids, res.p, res.rid, res.rval, (int)N, (int)R,
                                        shape(g->plain_sweep, ctx->grid_sweep)));
    if (ctx->cur_flags & PLC_QF_NO_RESIDUAL) {
      res.rid = nullptr;
      res.rval = nullptr;
    }
  }
  if (ctx->timing) {
    float ms = 0;
    // rounds run inside a self launch are not the scatter kernel's work
    ctx->t_scatter.units += h.edges - h.loop_edges;
    ctx->t_scatter.entries += h.pushes - h.loop_pushes;
    ctx->t_self.units += h.pushes;
    ctx->t_self.entries += h.pushes;
    HIPCHK(ctx, hipEventElapsedTime(&ms, ctx->ev_sweep.a, ctx->ev_sweep.b));
    ctx->t_sweep.ms += ms;
    ctx->t_sweep.launches++;
    ctx->t_sweep.units += h.etotal;
    ctx->t_sweep.entries += h.N;
  }

  plc_result_info& info = res.info;
  info.status = h.limited ? PLC_E_LIMIT : PLC_OK;
  info.rounds = h.round;
  info.pushes = h.pushes;
  info.edges = h.edges;
  info.support = h.N;
  info.kstar = h.kstar;
  info.cut = h.best_cut;
  info.vol = h.best_vol;
  info.phi = h.phi;
  info.r_nnz = h.rnnz;
  info.launches = h.steps;
  info.loop_rounds = h.loop_rounds;
  info.loop_edges = h.loop_edges;
  info.host_ns = std::chrono::duration_cast<std::chrono::nanoseconds>(
                     std::chrono::steady_clock::now() - ctx->q_t0).count();
  info.device_ns = h.t_end > h.t_start ? (int64_t)((double)(h.t_end - h.t_start) * ctx->clock_ns) : 0;
  info.bin_rounds = h.bin_rounds;
  info.pull_rounds = h.pull_rounds;
  info.bin_edges = h.bin_edges;
  info.flags = ctx->cur_flags;
  info.pipelined = ctx->cur_pipe;
  plc_status st = PLC_OK;
  if (!res.block) {
    info.status = PLC_E_NOMEM;
    st = PLC_E_NOMEM;
  }
  uint64_t id = ctx->next_id++;
  ctx->results[id] = res;
  if (id_out) *id_out = id;
  if (info_out) *info_out = info;
  return st;
}

extern "C" plc_status plc_run(plc_ctx* ctx, plc_graph* g, const plc_query* q, int32_t count,
                              uint64_t* ids, plc_result_info* infos) {
  if (!ctx || !g || !ctx->graphs.count(g) || (count > 0 && !q) || count < 0) return PLC_E_INVALID;
  if (ctx->broken) return PLC_E_HIP;
  (void)hipSetDevice(ctx->device);
  plc_status first = PLC_OK;
  int pre = 0;   // the current query's queued first chunk (see run_one)
  int pipe = 0;  // the current query's plc_result_info.pipelined
  for (int32_t i = 0; i < count; i++) {
    if (!query_ok(g, q[i])) {
      if (ids) ids[i] = 0;
      if (infos) {
        std::memset(&infos[i], 0, sizeof(plc_result_info));
        infos[i].status = PLC_E_INVALID;
      }
      if (first == PLC_OK) first = PLC_E_INVALID;
      continue;
    }
    // the next query (when valid) is queued behind this one's first read-back
    const plc_query* nq = i + 1 < count && query_ok(g, q[i + 1]) ? &q[i + 1] : nullptr;
    int next_pre = 0, next_pipe = 0;
    plc_status st = run_one(ctx, g, q[i], ids ? &ids[i] : nullptr, infos ? &infos[i] : nullptr,
                            nullptr, 0, 1.0, pre, nq, &next_pre, pipe, &next_pipe);
    pre = next_pre;
    pipe = next_pipe;
    if (st == PLC_E_HIP) return st;
    if (st != PLC_OK && first == PLC_OK) first = st;
  }
  if (hipStreamSynchronize(ctx->stream) != hipSuccess) {
    ctx->broken = true;
    return PLC_E_HIP;
  }
  return first;
}

extern "C" plc_status plc_run_set(plc_ctx* ctx, plc_graph* g, const int32_t* seeds,
                                  int32_t nseeds, double alpha, double eps, int32_t rule,
                                  uint64_t* id, plc_result_info* info) {
  if (!ctx || !g || !ctx->graphs.count(g) || !seeds || nseeds < 1) return PLC_E_INVALID;
  if (ctx->broken) return PLC_E_HIP;
  plc_query q{};
  q.seed = seeds[0];
  q.alpha = alpha;
  q.eps = eps;
  q.rule = rule;
  std::vector<int32_t> set(seeds, seeds + nseeds);
  for (int32_t v : set) {
    q.seed = v;
    if (!query_ok(g, q)) return PLC_E_INVALID;
  }
  std::sort(set.begin(), set.end());
  set.erase(std::unique(set.begin(), set.end()), set.end());
  (void)hipSetDevice(ctx->device);
  plc_status st = run_one(ctx, g, q, id, info, set.data(), (int32_t)set.size());
  if (st == PLC_E_HIP) return st;
  if (hipStreamSynchronize(ctx->stream) != hipSuccess) {
    ctx->broken = true;
    return PLC_E_HIP;
  }
  return st;
}

// psi_k = sum_{m=0}^{N-k} k!/(m+k)! t^m (Sec. 3.4), term by term:
// term_0 = 1, term_m = term_{m-1} * t / (k + m).
static double hk_psi(int32_t N, int32_t k, double t) {
  double term = 1.0, s = 1.0;
  for (int32_t m = 1; m <= N - k; m++) {
    term = term * t / (double)(k + m);
    s += term;
  }
  return s;
}

extern "C" plc_status plc_run_hkpr(plc_ctx* ctx, plc_graph* g, int32_t seed, int32_t N,
                                   double eps, double t, uint64_t* id, plc_result_info* info) {
  if (!ctx || !g || !ctx->graphs.count(g)) return PLC_E_INVALID;
  if (seed < 0 || seed >= g->n || g->deg[seed] < 1) return PLC_E_INVALID;
  if (N < 1 || N > plc::kHkMaxLevels) return PLC_E_INVALID;
  if (!std::isfinite(eps) || !(eps > 0.0) || !std::isfinite(t) || !(t > 0.0))
    return PLC_E_INVALID;
  if (ctx->broken) return PLC_E_HIP;
  (void)hipSetDevice(ctx->device);
  ctx->q_t0 = std::chrono::steady_clock::now();
  ctx->cur_flags = 0;
  ctx->cur_pipe = 0;
  hipStream_t s = ctx->stream;
  const PlainArgs& a = g->args;
  // threshold of level k: ((e^-t eps) d(w)) / B_k with B_k = 2 N psi_k
  std::vector<double> B(N + 1);
  for (int32_t k = 0; k <= N; k++) B[k] = 2.0 * (double)N * hk_psi(N, k, t);
  HIPCHK(ctx, hipMemcpyAsync(a.hk_B, B.data(), sizeof(double) * (N + 1), hipMemcpyHostToDevice,
                             s));
  HIPCHK(ctx, plc::launch_hk_init(s, a, seed, N, t, std::exp(-t) * eps));
  // at most N levels; levels past an empty frontier exit at once
  // (HK-PR levels and Nibble steps reach far larger frontiers than the
  // PR-Nibble sample the shape was tuned on: at least CU/2 workgroups)
  const int gs = std::max(shape(g->plain_self, ctx->grid_self), ctx->num_cu / 2);
  const int gc = shape(g->plain_scatter, ctx->grid_scatter);
  for (int32_t j = 0; j < N; j++) HIPCHK(ctx, plc::launch_hk_level(s, a, gs, gc));
  HIPCHK(ctx, plc::launch_hk_clear(s, a, shape(g->plain_sweep, ctx->grid_sweep)));
  Ctl& h = *ctx->ctl_host;
  HIPCHK(ctx, hipMemcpyAsync(&h, a.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
  HIPCHK(ctx, hipStreamSynchronize(s));
  if (h.status != plc::ST_PUSH || h.cnt[h.round & 1] != 0 || h.fault) {
    ctx->broken = true;
    return PLC_E_HIP;
  }
  plc_status st = sweep_and_record(ctx, g, id, info);
  if (st == PLC_E_HIP) return st;
  if (hipStreamSynchronize(s) != hipSuccess) {
    ctx->broken = true;
    return PLC_E_HIP;
  }
  return st;
}

extern "C" plc_status plc_run_beta(plc_ctx* ctx, plc_graph* g, const plc_query* q, double beta,
                                   uint64_t* id, plc_result_info* info) {
  if (!ctx || !g || !ctx->graphs.count(g) || !q) return PLC_E_INVALID;
  if (!query_ok(g, *q) || !(beta > 0.0 && beta <= 1.0)) return PLC_E_INVALID;
  if (ctx->broken) return PLC_E_HIP;
  (void)hipSetDevice(ctx->device);
  plc_status st = run_one(ctx, g, *q, id, info, nullptr, 0, beta);
  if (st == PLC_E_HIP) return st;
  if (hipStreamSynchronize(ctx->stream) != hipSuccess) {
    ctx->broken = true;
    return PLC_E_HIP;
  }
  return st;
}

extern "C" plc_status plc_run_nibble(plc_ctx* ctx, plc_graph* g, int32_t seed, double eps,
                                     int32_t T, uint64_t* id, plc_result_info* info) {
  if (!ctx || !g || !ctx->graphs.count(g)) return PLC_E_INVALID;
  if (seed < 0 || seed >= g->n || g->deg[seed] < 1) return PLC_E_INVALID;
  if (T < 0 || T > plc::kNbMaxSteps || !std::isfinite(eps) || !(eps > 0.0)) return PLC_E_INVALID;
  if (ctx->broken) return PLC_E_HIP;
  (void)hipSetDevice(ctx->device);
  ctx->q_t0 = std::chrono::steady_clock::now();
  ctx->cur_flags = 0;
  ctx->cur_pipe = 0;
  hipStream_t s = ctx->stream;
  const PlainArgs& a = g->args;
  HIPCHK(ctx, plc::launch_nb_init(s, a, seed, eps, T));
  // (HK-PR levels and Nibble steps reach far larger frontiers than the
  // PR-Nibble sample the shape was tuned on: at least CU/2 workgroups)
  const int gs = std::max(shape(g->plain_self, ctx->grid_self), ctx->num_cu / 2);
  const int gc = shape(g->plain_scatter, ctx->grid_scatter);
  for (int32_t j = 0; j < T; j++) HIPCHK(ctx, plc::launch_nb_step(s, a, gs, gc));
  Ctl& h = *ctx->ctl_host;
  HIPCHK(ctx, hipMemcpyAsync(&h, a.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
  HIPCHK(ctx, hipStreamSynchronize(s));
  if (h.status != plc::ST_PUSH || h.fault || h.round < 0 || h.round > T) {
    ctx->broken = true;
    return PLC_E_HIP;
  }
  // the returned vector: the last step's, unless that step's frontier was
  // empty, then the one before it
  const int32_t J = h.round;
  const int32_t R = h.cnt[J & 1] > 0 ? J : J - 1;
  HIPCHK(ctx, plc::launch_nb_finish(s, a, R, J, shape(g->plain_sweep, ctx->grid_sweep)));
  h.support_cnt = h.hk_tlc[R % 3];
  h.touched_cnt = 0;
  plc_status st = sweep_and_record(ctx, g, id, info);
  if (st == PLC_E_HIP) return st;
  if (hipStreamSynchronize(s) != hipSuccess) {
    ctx->broken = true;
    return PLC_E_HIP;
  }
  return st;
}

extern "C" plc_status plc_result_info_get(plc_ctx* ctx, uint64_t id, plc_result_info* out) {
  if (!ctx || !out) return PLC_E_INVALID;
  auto it = ctx->results.find(id);
  if (it == ctx->results.end()) return ctx->inflight.count(id) ? PLC_E_NOTREADY : PLC_E_NOTFOUND;
  *out = it->second.info;
  return PLC_OK;
}

extern "C" plc_status plc_result_copy(plc_ctx* ctx, uint64_t id, int32_t* sweep_ids,
                                      double* sweep_p, int32_t* r_ids, double* r_vals) {
  if (!ctx) return PLC_E_INVALID;
  if (ctx->broken) return PLC_E_HIP;
  auto it = ctx->results.find(id);
  if (it == ctx->results.end()) return PLC_E_NOTFOUND;
  Result& r = it->second;
  if (!r.block) return PLC_E_NOMEM;
  (void)hipSetDevice(ctx->device);
  hipStream_t s = ctx->stream;
  // (a query run with PLC_QF_NO_RESIDUAL keeps no r vector)
  size_t N = (size_t)r.info.support, R = r.rid ? (size_t)r.info.r_nnz : 0;
  if (sweep_ids && N) HIPCHK(ctx, hipMemcpyAsync(sweep_ids, r.ids, 4 * N, hipMemcpyDeviceToHost, s));
  if (sweep_p && N) HIPCHK(ctx, hipMemcpyAsync(sweep_p, r.p, 8 * N, hipMemcpyDeviceToHost, s));
  if (r_ids && R) HIPCHK(ctx, hipMemcpyAsync(r_ids, r.rid, 4 * R, hipMemcpyDeviceToHost, s));
  if (r_vals && R) HIPCHK(ctx, hipMemcpyAsync(r_vals, r.rval, 8 * R, hipMemcpyDeviceToHost, s));
  HIPCHK(ctx, hipStreamSynchronize(s));
  return PLC_OK;
}

extern "C" plc_status plc_result_copy_many(plc_ctx* ctx, int32_t count, const uint64_t* ids,
                                           int32_t* const* sweep_ids, double* const* sweep_p,
                                           int32_t* const* r_ids, double* const* r_vals) {
  if (!ctx || count < 0 || (count > 0 && !ids)) return PLC_E_INVALID;
  if (ctx->broken) return PLC_E_HIP;
  if (count == 0) return PLC_OK;
  // the parts to copy: (source, bytes, host destination); data offsets in
  // the staging memory 16-byte aligned
  struct Part {
    const void* src;
    size_t bytes;
    void* dst;
    size_t off;
  };
  std::vector<Part> parts;
  parts.reserve(4 * (size_t)count);
  size_t data = 0;
  for (int32_t i = 0; i < count; i++) {
    auto it = ctx->results.find(ids[i]);
    if (it == ctx->results.end()) return PLC_E_NOTFOUND;
    const Result& r = it->second;
    if (!r.block) return PLC_E_NOMEM;
    const size_t N = (size_t)r.info.support, R = r.rid ? (size_t)r.info.r_nnz : 0;
    auto add = [&](const void* src, size_t bytes, void* dst) {
      if (!dst || !bytes) return;
      parts.push_back(Part{src, bytes, dst, data});
      data += (bytes + 15) & ~(size_t)15;
    };
    add(r.ids, 4 * N, sweep_ids ? sweep_ids[i] : nullptr);
    add(r.p, 8 * N, sweep_p ? sweep_p[i] : nullptr);
    add(r.rid, 4 * R, r_ids ? r_ids[i] : nullptr);
    add(r.rval, 8 * R, r_vals ? r_vals[i] : nullptr);
  }
  if (parts.empty()) return PLC_OK;
  (void)hipSetDevice(ctx->device);
  hipStream_t s = ctx->stream;
  const size_t jobs_bytes = (sizeof(plc::GatherJob) * parts.size() + 255) & ~(size_t)255;
  const size_t need = jobs_bytes + data;
  if (need > ctx->stage_bytes) {
    // (the stream is idle here: every earlier call ended with a wait)
    size_t cap = std::max<size_t>(ctx->stage_bytes, (size_t)1 << 20);
    while (cap < need) cap <<= 1;
    if (ctx->stage_h) (void)hipHostFree(ctx->stage_h);
    ctx->stage_h = nullptr;
    ctx->stage_d = nullptr;
    ctx->stage_bytes = 0;
    void* h = nullptr;
    void* d = nullptr;
    if (hipHostMalloc(&h, cap, hipHostMallocMapped) != hipSuccess) {
      (void)hipGetLastError();
      return PLC_E_NOMEM;
    }
    if (hipHostGetDevicePointer(&d, h, 0) != hipSuccess) {
      (void)hipGetLastError();
      (void)hipHostFree(h);
      return PLC_E_HIP;
    }
    ctx->stage_h = static_cast<char*>(h);
    ctx->stage_d = static_cast<char*>(d);
    ctx->stage_bytes = cap;
  }
  plc::GatherJob* jobs = reinterpret_cast<plc::GatherJob*>(ctx->stage_h);
  for (size_t k = 0; k < parts.size(); k++)
    jobs[k] = plc::GatherJob{static_cast<const uint32_t*>(parts[k].src), parts[k].off / 4,
                             parts[k].bytes / 4};
  HIPCHK(ctx, plc::launch_gather_results(
                  s, reinterpret_cast<const plc::GatherJob*>(ctx->stage_d), (int)parts.size(),
                  reinterpret_cast<uint32_t*>(ctx->stage_d + jobs_bytes)));
  HIPCHK(ctx, hipStreamSynchronize(s));
  for (const Part& pt : parts) std::memcpy(pt.dst, ctx->stage_h + jobs_bytes + pt.off, pt.bytes);
  return PLC_OK;
}

extern "C" plc_status plc_release(plc_ctx* ctx, uint64_t id) {
  if (!ctx) return PLC_E_INVALID;
  auto it = ctx->results.find(id);
  if (it == ctx->results.end()) return PLC_E_NOTFOUND;
  // The block may still be the target of the queued result copy, but every
  // later user of arena memory is queued on the same stream, behind it, so
  // it returns to the arena at once (no wait).
  if (it->second.block) ctx->arena.release(it->second.block);
  ctx->results.erase(it);
  return PLC_OK;
}

extern "C" plc_status plc_arena_free_bytes(plc_ctx* ctx, size_t* total, size_t* largest) {
  if (!ctx) return PLC_E_INVALID;
  if (total) *total = ctx->arena.free_bytes();
  if (largest) *largest = ctx->arena.largest_free();
  return PLC_OK;
}

extern "C" plc_status plc_timing_enable(plc_ctx* ctx, int32_t on) {
  if (!ctx) return PLC_E_INVALID;
  ctx->timing = on != 0;
  ctx->t_scatter = KTime{};
  ctx->t_self = KTime{};
  ctx->t_sweep = KTime{};
  return PLC_OK;
}

static void put_time(const KTime& k, plc_kernel_time* o) {
  if (!o) return;
  o->launches = k.launches;
  o->ms = k.ms;
  o->units = k.units;
  o->entries = k.entries;
}

extern "C" plc_status plc_timing_get(plc_ctx* ctx, plc_kernel_time* scatter, plc_kernel_time* self,
                                     plc_kernel_time* sweep) {
  if (!ctx) return PLC_E_INVALID;
  put_time(ctx->t_scatter, scatter);
  put_time(ctx->t_self, self);
  put_time(ctx->t_sweep, sweep);
  return PLC_OK;
}

// ---------------------------------------------------------------- batched path

static double now_ms() {
  return std::chrono::duration<double, std::milli>(
             std::chrono::steady_clock::now().time_since_epoch()).count();
}

static void batch_free(plc_ctx* ctx, plc_graph* g) {
  BatchEngine* E = g->batch;
  if (!E) return;
  for (void* b : E->blocks) ctx->arena.release(b);
  for (auto& r : E->sweeping)
    if (r.block) ctx->arena.release(r.block);
  for (int q = 0; q < E->B; q++)
    if (E->state[q] != HS_FREE) ctx->inflight.erase(E->qid[q]);
  for (auto& pq : E->queue) ctx->inflight.erase(pq.first);
  if (E->slots_h) (void)hipHostFree(E->slots_h);
  if (E->segs_h) (void)hipHostFree(E->segs_h);
  if (E->adm_h) (void)hipHostFree(E->adm_h);
  if (E->ctl_h) (void)hipHostFree(E->ctl_h);
  if (E->hdr_h) (void)hipHostFree(E->hdr_h);
  if (E->grow_h) (void)hipHostFree(E->grow_h);
  if (E->holds_h) (void)hipHostFree(E->holds_h);
  if (E->clear_h) (void)hipHostFree(E->clear_h);
  for (void* b : E->qblock)
    if (b) ctx->arena.release(b);
  captured_free(E->round_g);
  delete E;
  g->batch = nullptr;
}

// Round-buffer and sweep-buffer capacities (entries, edges, sort elements).
// A single query never exceeds them (frontier <= n, edges <= 2m, support <= n),
// so every step makes progress.
static void batch_caps(const plc_graph* g, int B, int64_t* nf_cap, int64_t* e_cap,
                       int64_t* s_cap) {
  const int64_t n = g->n, arcs = std::max<int64_t>(g->arcs, 1);
  *nf_cap = std::min<int64_t>(std::max<int64_t>(2 * n, 1 << 22), (int64_t)B * n);
  *nf_cap = std::max<int64_t>(*nf_cap, n);
  *nf_cap = std::min<int64_t>(*nf_cap, INT32_MAX / 2);
  *e_cap = std::max<int64_t>(2 * arcs, 1 << 26);
  *s_cap = std::max<int64_t>(std::min<int64_t>(2 * n, (int64_t)B * n), n);
  *s_cap = std::min<int64_t>(*s_cap, INT32_MAX / 2);
}

static size_t batch_fixed_bytes(const plc_graph* g, int B) {
  int64_t nf_cap, e_cap, s_cap;
  batch_caps(g, B, &nf_cap, &e_cap, &s_cap);
  const int64_t tile_cap = e_cap / plc::kEdgeTile + 2;
  const int64_t desc_cap = std::max(nf_cap, s_cap) / plc::kScanBlock + 2;
  size_t b = 0;
  b += 28 * (size_t)nf_cap + 4 * (size_t)tile_cap + 3 * 16 * (size_t)desc_cap;
  b += (2 * sizeof(plc::SortElem) + 4 + 8 + 4 + 8) * (size_t)s_cap;
  b += (sizeof(plc::Slot) + sizeof(plc::SweepSeg) + sizeof(plc::Admit) + sizeof(plc::Grow) +
        2 * sizeof(plc::ClearJob) + 12) * (size_t)B;
  b += 8 * (size_t)g->n + 64 * 1024;  // compact: graph-wide {d, hot code}
  return b;
}

// Compact layout.  A table's capacity is a multiple of kScanBlock records
// (the r gather scans tables in kScanBlock chunks) sized so that before a
// round at most half of it is occupied and the round's worst case
// (occupancy + one new key per edge of the frontier, "worst") stays within
// 3/4 of it: linear probing then stays short even in the rounds that add
// nearly as many new keys as they have edges (the first rounds of a query),
// and a table never fills.  A query block holds the records (16 B), p (8 B)
// and four lists of 3/4 cap vertex ids (12 B): 36 B per record.
static int64_t table_cap_for(const plc_graph* g, int64_t occupied, int64_t worst) {
  occupied = std::min<int64_t>(std::max<int64_t>(occupied, 1), g->n);
  worst = std::min<int64_t>(std::max<int64_t>(worst, occupied), g->n);
  const int64_t need = std::max<int64_t>(2 * occupied, (4 * worst + 2) / 3);
  return (need + plc::kScanBlock - 1) / plc::kScanBlock * plc::kScanBlock;
}
static bool table_needs_growth(int64_t cap, int64_t occupied, int64_t worst) {
  return 2 * occupied > cap || 4 * worst > 3 * cap;
}
static size_t table_block_bytes(int64_t cap) { return 36 * (size_t)cap; }
static int64_t table_list_cap(int64_t cap) { return cap / 4 * 3; }
// growth: at least twice the current capacity (few rehashes), but never
// beyond the table that the query's touched bound needs
static int64_t table_grown_cap(const plc_graph* g, int64_t cap, int64_t occupied, int64_t worst,
                               int64_t bound) {
  return std::max<int64_t>(table_cap_for(g, occupied, worst),
                           std::min<int64_t>(2 * cap, table_cap_for(g, bound, bound)));
}
// Touched bound of a query (the push's work bound, Sec. 3.3): every push but
// the seed's moves at least alpha' eps d(v) of the unit mass into p, so at
// most 1 + d(seed) + 1/(alpha' eps) vertices are touched (and at most n).
static int64_t touched_bound(const plc_graph* g, const plc_query& q) {
  const double ap = q.rule == PLC_RULE_OPT ? 2.0 * q.alpha / (1.0 + q.alpha) : q.alpha;
  const double b = 1.0 + (double)g->deg[q.seed] + std::floor(1.0 / (ap * q.eps));
  return (int64_t)std::min(b, (double)g->n);
}

// Arena kept free for result blocks when tables are taken (admission) or
// grown (half of it).
static size_t result_headroom(const plc_ctx* ctx) {
  return std::max<size_t>((size_t)64 << 20, ctx->arena.capacity() / 32);
}

static size_t batch_slot_bytes(const plc_graph* g) {
  return (sizeof(plc::VRec) + 8 + 8 + 4 + 4) * (size_t)g->n;  // vr, p, 2 frontiers, support, touched
}

static plc_status batch_create(plc_ctx* ctx, plc_graph* g, int B) {
  BatchEngine* E = new (std::nothrow) BatchEngine();
  if (!E) return PLC_E_NOMEM;
  g->batch = E;
  E->B = B;
  int64_t nf_cap, e_cap, s_cap;
  batch_caps(g, B, &nf_cap, &e_cap, &s_cap);
  const int64_t tile_cap = e_cap / plc::kEdgeTile + 2;
  const int64_t desc_cap = std::max(nf_cap, s_cap) / plc::kScanBlock + 2;
  const size_t n = (size_t)g->n;
  bool nomem = false;
  auto take = [&](size_t bytes) -> void* {
    void* p = ctx->arena.alloc(bytes);
    if (!p) { nomem = true; return nullptr; }
    E->blocks.push_back(p);
    E->bytes += (bytes + Arena::kAlign - 1) & ~(Arena::kAlign - 1);
    return p;
  };
  plc::BatchArgs& a = E->args;
  a.n = g->n;
  a.vol_total = g->arcs;
  a.off = g->args.off;
  a.nbr = g->args.nbr;
  a.hot_ids = g->args.hot_ids;
  a.hotcode = g->args.hotcode;
  a.B = B;
  E->compact = ctx->opt.batch_state == PLC_STATE_COMPACT;
  a.slots = static_cast<plc::Slot*>(take(sizeof(plc::Slot) * B));
  if (E->compact) {
    a.vr = nullptr;
    a.p = nullptr;
    a.gdh = static_cast<int2*>(take(8 * n));
  } else {
    a.vr = static_cast<plc::VRec*>(take(sizeof(plc::VRec) * n * B));
    a.p = static_cast<double*>(take(8 * n * B));
    E->d_fbuf = static_cast<int32_t*>(take(4 * 2 * n * B));
    E->d_support = static_cast<int32_t*>(take(4 * n * B));
    E->d_touched = static_cast<int32_t*>(take(4 * n * B));
    a.gdh = nullptr;
  }
  E->grow_d = static_cast<plc::Grow*>(take(sizeof(plc::Grow) * B));
  E->holds_d = static_cast<int32_t*>(take(4 * (size_t)B));
  E->clear_d = static_cast<plc::ClearJob*>(take(sizeof(plc::ClearJob) * 2 * (size_t)B));
  a.ctl = static_cast<plc::BatchCtl*>(take(sizeof(plc::BatchCtl)));
  a.fprefix = static_cast<int32_t*>(take(4 * ((size_t)B + 1)));
  a.eslot = static_cast<int32_t*>(take(4 * (size_t)nf_cap));
  a.coef = static_cast<double*>(take(8 * (size_t)nf_cap));
  a.estart = static_cast<int64_t*>(take(8 * (size_t)nf_cap));
  a.rowp = static_cast<int64_t*>(take(8 * (size_t)nf_cap));
  a.nf_cap = (int32_t)nf_cap;
  a.e_cap = e_cap;
  a.tile_start = static_cast<int32_t*>(take(4 * (size_t)tile_cap));
  a.tile_cap = tile_cap;
  a.desc_cap = (int32_t)desc_cap;
  for (int k = 0; k < plc::BNUM_SCANS; k++)
    a.desc[k] = static_cast<unsigned long long*>(take(2 * 8 * (size_t)desc_cap));
  a.segs = static_cast<plc::SweepSeg*>(take(sizeof(plc::SweepSeg) * B));
  a.sbuf[0] = static_cast<plc::SortElem*>(take(sizeof(plc::SortElem) * (size_t)s_cap));
  a.sbuf[1] = static_cast<plc::SortElem*>(take(sizeof(plc::SortElem) * (size_t)s_cap));
  a.sdeg = static_cast<int32_t*>(take(4 * (size_t)s_cap));
  a.svol = static_cast<int64_t*>(take(8 * (size_t)s_cap));
  a.scnt = static_cast<int32_t*>(take(4 * (size_t)s_cap));
  a.scut = static_cast<int64_t*>(take(8 * (size_t)s_cap));
  a.s_cap = s_cap;
  E->adm_d = static_cast<plc::Admit*>(take(sizeof(plc::Admit) * B));
  if (nomem) {
    batch_free(ctx, g);
    return PLC_E_NOMEM;
  }
  E->state.assign(B, HS_FREE);
  E->qid.assign(B, 0);
  E->qblock.assign(B, nullptr);
  E->qbucket.assign(B, 0);
  E->qflags.assign(B, 0u);
  E->qcap.assign(B, 0);
  E->qgrows.assign(B, 0);
  E->qbound.assign(B, 0);
  E->hold.assign(B, 0);
  E->fresh.assign(B, 0);
  if (hipHostMalloc(reinterpret_cast<void**>(&E->slots_h), sizeof(plc::Slot) * B,
                    hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&E->segs_h), sizeof(plc::SweepSeg) * B,
                    hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&E->adm_h), sizeof(plc::Admit) * B,
                    hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&E->ctl_h), sizeof(plc::BatchCtl),
                    hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&E->hdr_h), sizeof(SweepHdr),
                    hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&E->grow_h), sizeof(plc::Grow) * B,
                    hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&E->holds_h), 4 * (size_t)B,
                    hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&E->clear_h), sizeof(plc::ClearJob) * 2 * (size_t)B,
                    hipHostMallocDefault) != hipSuccess) {
    batch_free(ctx, g);
    ctx->broken = true;
    return PLC_E_HIP;
  }
  hipStream_t s = ctx->stream;
  HIPCHK(ctx, hipMemsetAsync(a.slots, 0, sizeof(plc::Slot) * B, s));
  HIPCHK(ctx, hipMemsetAsync(a.ctl, 0, sizeof(plc::BatchCtl), s));
  for (int k = 0; k < plc::BNUM_SCANS; k++)
    HIPCHK(ctx, hipMemsetAsync(a.desc[k], 0, 2 * 8 * (size_t)desc_cap, s));
  if (E->compact)
    HIPCHK(ctx, plc::launch_gdh_init(s, a, const_cast<int2*>(a.gdh)));
  else
    HIPCHK(ctx, plc::launch_batch_init(s, a));
  HIPCHK(ctx, hipStreamSynchronize(s));
  return PLC_OK;
}

extern "C" plc_status plc_batch_reserve(plc_ctx* ctx, plc_graph* g, int32_t slots,
                                        int32_t* granted) {
  if (slots <= 0 && ctx) slots = ctx->opt.batch_slots;
  if (!ctx || !g || !ctx->graphs.count(g) || slots < 1 || slots > 1024) return PLC_E_INVALID;
  if (ctx->broken) return PLC_E_HIP;
  (void)hipSetDevice(ctx->device);
  if (hipStreamSynchronize(ctx->stream) != hipSuccess) {
    ctx->broken = true;
    return PLC_E_HIP;
  }
  batch_free(ctx, g);
  // Largest slot count that fits the free arena (one block per array),
  // keeping headroom for the result blocks of finished queries.
  int B = slots;
  const size_t per = ctx->opt.batch_state == PLC_STATE_COMPACT ? 0 : batch_slot_bytes(g);
  const size_t free_now = ctx->arena.free_bytes();
  const size_t headroom = std::max<size_t>((size_t)64 << 20, free_now / 16);
  const size_t budget = free_now > headroom ? free_now - headroom : 0;
  while (B > 0) {
    size_t need = batch_fixed_bytes(g, B) + per * (size_t)B;
    if (need <= budget) break;
    B--;
  }
  while (B > 0) {
    plc_status st = batch_create(ctx, g, B);
    if (st == PLC_OK) break;
    if (st != PLC_E_NOMEM) return st;
    B = B * 3 / 4;  // fragmentation: retry smaller
  }
  if (granted) *granted = B;
  return B > 0 ? PLC_OK : PLC_E_NOMEM;
}

extern "C" plc_status plc_submit(plc_ctx* ctx, plc_graph* g, const plc_query* q, int32_t count,
                                 uint64_t* ids) {
  if (!ctx || !g || !ctx->graphs.count(g) || count < 0 || (count > 0 && !q)) return PLC_E_INVALID;
  if (ctx->broken) return PLC_E_HIP;
  if (!g->batch) return PLC_E_INVALID;
  plc_status first = PLC_OK;
  for (int32_t i = 0; i < count; i++) {
    if (!query_ok(g, q[i])) {
      if (ids) ids[i] = 0;
      if (first == PLC_OK) first = PLC_E_INVALID;
      continue;
    }
    uint64_t id = ctx->next_id++;
    g->batch->queue.emplace_back(id, q[i]);
    ctx->inflight[id] = g;
    if (ids) ids[i] = id;
  }
  return first;
}

// Graph of one batched round: plan, self, scatter, round end.
static Captured* batch_round_graph(plc_ctx* ctx, plc_graph* g) {
  const int gs = shape(g->batch_self, ctx->grid_self);
  const int gc = shape(g->batch_scatter, ctx->grid_scatter);
  Captured& c = g->batch->round_g;
  if (c.matches(gs, gc, 0, 1)) return &c;
  captured_free(c);
  c.gs = gs;
  c.gc = gc;
  c.gw = 0;
  c.rounds = 1;
  const plc::BatchArgs& a = g->batch->args;
  const bool compact = g->batch->compact;
  const bool ok = capture(ctx, c, [&](hipStream_t cs) -> hipError_t {
    hipError_t r;
    if ((r = plc::launch_batch_plan_self(cs, a, gs, compact)) != hipSuccess) return r;
    if ((r = plc::launch_batch_scatter(cs, a, gc, compact)) != hipSuccess) return r;
    return plc::launch_batch_round_end(cs, a);
  });
  return ok ? &c : nullptr;
}

constexpr int kBatchChain = 4;  // rounds per read-back, dense throughput mode

// One global step.  defer_sweep: while other queries are still pushing and
// none waits for a slot, leave finished queries unswept so that they are
// swept together later (fewer, larger sweeps: throughput mode).
static plc_status batch_step(plc_ctx* ctx, plc_graph* g, int32_t* in_flight, uint64_t* done_ids,
                             int32_t done_cap, int32_t* n_done, bool defer_sweep) {
  BatchEngine& E = *g->batch;
  plc::BatchArgs& a = E.args;
  hipStream_t s = ctx->stream;
  // 1. admission into free slots, in submission order (compact layout: while
  // the arena holds the query's first table and the result headroom)
  const int64_t n = g->n;
  int nadm = 0, njobs = 0;
  long long clear_total = 0;
  for (int q = 0; q < E.B && !E.queue.empty(); q++) {
    if (E.state[q] != HS_FREE) continue;
    const uint64_t id = E.queue.front().first;
    const plc_query qq = E.queue.front().second;
    plc::Admit& ad = E.adm_h[nadm];
    if (E.compact) {
      int64_t expect = 1;
      const int64_t bound = touched_bound(g, qq);
      auto hint = E.touched_hint.find(hint_bucket(qq));
      // never above this query's own touched bound (plc_query_bytes_estimate)
      if (hint != E.touched_hint.end())
        expect = (int64_t)std::min(hint->second, (double)bound);
      E.qbound[q] = bound;
      // the hinted size if the arena has room for it, else the seed's first
      // round only (the table then grows like any other)
      const int64_t first = table_cap_for(g, 1, 1 + (int64_t)g->deg[qq.seed]);
      int64_t cap = table_cap_for(g, expect, std::max<int64_t>(expect, 1 + g->deg[qq.seed]));
      void* blk = nullptr;
      for (;;) {
        const size_t bytes = table_block_bytes(cap);
        if (ctx->arena.free_bytes() >= bytes + result_headroom(ctx)) blk = ctx->arena.alloc(bytes);
        if (blk || cap == first) break;
        cap = first;
      }
      if (!blk) break;
      char* b = static_cast<char*>(blk);
      const int64_t L = table_list_cap(cap);
      ad.tab = reinterpret_cast<plc::VRec*>(b);
      ad.tp = reinterpret_cast<double*>(b + 16 * cap);
      int32_t* lists = reinterpret_cast<int32_t*>(b + 24 * cap);
      ad.fb0 = lists;
      ad.fb1 = lists + L;
      ad.support = lists + 2 * L;
      ad.touched = lists + 3 * L;
      ad.tcap = (int32_t)cap;
      ad.list_cap = (int32_t)L;
      plc::ClearJob& J = E.clear_h[njobs++];
      J.tab = ad.tab;
      J.tp = ad.tp;
      J.cap = cap;
      J.off = clear_total;
      clear_total += cap;
      E.qblock[q] = blk;
      E.qcap[q] = cap;
      E.qgrows[q] = 0;
      E.qbucket[q] = hint_bucket(qq);
    } else {
      ad.tab = a.vr + (int64_t)q * n;
      ad.tp = a.p + (int64_t)q * n;
      ad.fb0 = E.d_fbuf + 2 * (int64_t)q * n;
      ad.fb1 = E.d_fbuf + (2 * (int64_t)q + 1) * n;
      ad.support = E.d_support + (int64_t)q * n;
      ad.touched = E.d_touched + (int64_t)q * n;
      ad.tcap = 0;
      ad.list_cap = (int32_t)n;
    }
    E.queue.pop_front();
    nadm++;
    E.qflags[q] = qq.flags;
    ad.slot = q;
    ad.seed = qq.seed;
    ad.rule = (int32_t)qq.rule;
    ad.max_rounds = ctx->opt.max_rounds;
    ad.alpha = qq.alpha;
    ad.eps = qq.eps;
    ad.seed_deg = g->deg[qq.seed];
    ad.pad = 0;
    E.state[q] = HS_RUN;
    E.qid[q] = id;
    E.fresh[q] = 1;
    E.hold[q] = 0;
  }
  // 1b. compact layout: grow every table that this round could fill past
  // half (new keys this round <= the frontier's edge count); a query whose
  // table cannot grow now sits the round out
  int nfail = 0, ngrow = 0;
  long long total_old = 0, total_list = 0;
  std::vector<void*> old_blocks;
  if (E.compact) {
    int nhold = 0;
    for (int q = 0; q < E.B; q++) {
      if (E.state[q] != HS_RUN || E.fresh[q]) continue;
      const plc::Slot& S = E.slots_h[q];
      if (S.status != plc::SL_PUSH) continue;
      const int64_t occ = S.touched_cnt;
      const int64_t worst = std::min<int64_t>(E.qbound[q], occ + S.edge_next[S.par]);
      if (!table_needs_growth(E.qcap[q], occ, worst)) {
        if (E.hold[q]) {
          E.holds_h[nhold++] = q;
          E.hold[q] = 0;
        }
        continue;
      }
      const int64_t cap = table_grown_cap(g, E.qcap[q], occ, worst, E.qbound[q]);
      const size_t bytes = table_block_bytes(cap);
      void* blk = ctx->arena.free_bytes() >= bytes + result_headroom(ctx) / 2
                      ? ctx->arena.alloc(bytes) : nullptr;
      if (!blk) {
        if (!E.hold[q]) {
          E.holds_h[nhold++] = q | (1 << 16);
          E.hold[q] = 1;
        }
        continue;
      }
      char* b = static_cast<char*>(blk);
      const int64_t L = table_list_cap(cap);
      plc::Grow& G = E.grow_h[ngrow++];
      G.slot = q;
      G.old_cap = (int32_t)E.qcap[q];
      G.new_cap = (int32_t)cap;
      G.list_cap = (int32_t)L;
      G.rec_off = total_old;
      G.list_off = total_list;
      G.par = S.par;
      G.n_front = S.cnt[S.par];
      G.n_sup = S.support_cnt;
      G.n_touch = S.touched_cnt;
      total_list += (long long)G.n_front + G.n_sup + G.n_touch;
      G.tab = reinterpret_cast<plc::VRec*>(b);
      G.tp = reinterpret_cast<double*>(b + 16 * cap);
      int32_t* lists = reinterpret_cast<int32_t*>(b + 24 * cap);
      G.fb0 = lists;
      G.fb1 = lists + L;
      G.support = lists + 2 * L;
      G.touched = lists + 3 * L;
      plc::ClearJob& J = E.clear_h[njobs++];
      J.tab = G.tab;
      J.tp = G.tp;
      J.cap = cap;
      J.off = clear_total;
      clear_total += cap;
      total_old += E.qcap[q];
      old_blocks.push_back(E.qblock[q]);
      E.qblock[q] = blk;
      E.qcap[q] = cap;
      E.qgrows[q]++;
      E.hold[q] = 0;  // k_c_move_lists clears the device flag
    }
    if (nhold > 0) {
      HIPCHK(ctx, hipMemcpyAsync(E.holds_d, E.holds_h, 4 * (size_t)nhold, hipMemcpyHostToDevice,
                                 s));
      HIPCHK(ctx, plc::launch_slot_hold(s, a, E.holds_d, nhold));
    }
    // Every running query held and none left to sweep or admitted: nothing
    // would ever free memory, so the held query that needs the most fails.
    bool progress = false, held = false;
    for (int q = 0; q < E.B; q++) {
      if (E.state[q] == HS_PUSHED || (E.state[q] == HS_RUN && !E.hold[q])) progress = true;
      held |= E.state[q] == HS_RUN && E.hold[q];
    }
    if (!held && !progress && nadm == 0 && !E.queue.empty()) {
      bool busy = false;
      for (int q = 0; q < E.B; q++) busy |= E.state[q] != HS_FREE;
      if (!busy) {
        // nothing runs and the first queued query's table does not fit
        const uint64_t id = E.queue.front().first;
        E.queue.pop_front();
        Result res;
        res.info.status = PLC_E_NOMEM;
        ctx->results[id] = res;
        ctx->inflight.erase(id);
        if (done_ids && nfail < done_cap) done_ids[nfail] = id;
        nfail++;
      }
    }
    if (held && !progress) {
      int worst = -1;
      int64_t wneed = -1;
      for (int q = 0; q < E.B; q++) {
        if (E.state[q] != HS_RUN || !E.hold[q]) continue;
        const plc::Slot& S = E.slots_h[q];
        const int64_t need = (int64_t)S.touched_cnt + S.edge_next[S.par];
        if (need > wneed) { wneed = need; worst = q; }
      }
      const plc::Slot& S = E.slots_h[worst];
      Result res;
      res.info.status = PLC_E_NOMEM;
      res.info.rounds = S.rounds;
      res.info.pushes = S.pushes;
      res.info.edges = S.edges;
      const uint64_t id = E.qid[worst];
      ctx->results[id] = res;
      ctx->inflight.erase(id);
      if (done_ids && nfail < done_cap) done_ids[nfail] = id;
      nfail++;
      ctx->arena.release(E.qblock[worst]);  // the device slot stays held until re-admitted
      E.qblock[worst] = nullptr;
      E.qcap[worst] = 0;
      E.state[worst] = HS_FREE;
      E.qid[worst] = 0;
    }
  }
  // 1c. clear new tables, admit, move grown tables (in this order)
  const int gw = shape(g->batch_sweep, ctx->grid_sweep);
  if (njobs > 0) {
    HIPCHK(ctx, hipMemcpyAsync(E.clear_d, E.clear_h, sizeof(plc::ClearJob) * njobs,
                               hipMemcpyHostToDevice, s));
    HIPCHK(ctx, plc::launch_table_clear(s, E.clear_d, njobs, clear_total, gw));
  }
  if (nadm > 0) {
    HIPCHK(ctx, hipMemcpyAsync(E.adm_d, E.adm_h, sizeof(plc::Admit) * nadm,
                               hipMemcpyHostToDevice, s));
    HIPCHK(ctx, plc::launch_batch_admit(s, a, E.adm_d, nadm, E.compact));
  }
  if (ngrow > 0) {
    HIPCHK(ctx, hipMemcpyAsync(E.grow_d, E.grow_h, sizeof(plc::Grow) * ngrow,
                               hipMemcpyHostToDevice, s));
    HIPCHK(ctx, plc::launch_table_grow(s, a, E.grow_d, ngrow, total_old, total_list, gw));
    // stream order: later users of these blocks run after the rehash
    for (void* b : old_blocks) ctx->arena.release(b);
  }
  // 2. one round for every running query
  bool any_run = false;
  for (int q = 0; q < E.B; q++) any_run |= E.state[q] == HS_RUN;
  const EventPair* scatter_ev = nullptr;
  if (any_run) {
    // while timing is on, the round is launched directly (graphs carry no
    // events) and the scatter carries events on its own dispatch timestamps
    Captured* rg = ctx->use_graphs && !ctx->timing ? batch_round_graph(ctx, g) : nullptr;
    if (rg) {
      // Dense slots with nothing waiting for admission (throughput mode) need
      // no host action between rounds (k_b_plan retires a slot whose
      // frontier emptied), so several rounds share one read-back.
      const int chain = defer_sweep && E.queue.empty() && !E.compact ? kBatchChain : 1;
      for (int i = 0; i < chain; i++) HIPCHK(ctx, hipGraphLaunch(rg->exec, s));
    } else {
      HIPCHK(ctx, plc::launch_batch_plan_self(s, a, shape(g->batch_self, ctx->grid_self),
                                              E.compact));
      hipEvent_t t0 = nullptr, t1 = nullptr;
      if (ctx->timing) {
        if (ctx->ev_scatter.empty()) ctx->ev_scatter.emplace_back();
        HIPCHK(ctx, ev_pair(ctx->ev_scatter[0]));
        scatter_ev = &ctx->ev_scatter[0];
        t0 = scatter_ev->a;
        t1 = scatter_ev->b;
      }
      HIPCHK(ctx, plc::launch_batch_scatter(s, a, shape(g->batch_scatter, ctx->grid_scatter),
                                            E.compact, t0, t1));
      HIPCHK(ctx, plc::launch_batch_round_end(s, a));
    }
  }
  // 3. sweep the queries whose frontier emptied in an earlier step
  int nseg = 0;
  long long total = 0, touch_total = 0, vol_bound = 0;
  E.sweeping.clear();
  // (a held query makes no progress, so it never delays the sweeps that free memory)
  bool any_active = false;
  for (int q = 0; q < E.B; q++) any_active |= E.state[q] == HS_RUN && !E.hold[q];
  const bool hold = defer_sweep && any_active && E.queue.empty();
  for (int q = 0; q < E.B && !hold; q++) {
    if (E.state[q] != HS_PUSHED) continue;
    const plc::Slot& S = E.slots_h[q];
    const long long N = S.support_cnt, T = S.touched_cnt;
    if (nseg > 0 && (total + N > a.s_cap || vol_bound + S.edges > a.e_cap)) continue;
    Result res;
    const bool keep_r = !(E.qflags[q] & PLC_QF_NO_RESIDUAL);
    const size_t Tr = keep_r ? (size_t)T : 0;
    size_t off_p = (4 * (size_t)N + 255) & ~(size_t)255;
    size_t off_rid = off_p + ((8 * (size_t)N + 255) & ~(size_t)255);
    size_t off_rval = off_rid + ((4 * Tr + 255) & ~(size_t)255);
    res.block = ctx->arena.alloc(off_rval + 8 * Tr);
    plc::SweepSeg& sg = E.segs_h[nseg];
    sg.slot = q;
    sg.n_elem = (int32_t)N;
    sg.elem_off = total;
    // finish entries: the touched list (dense) or every table record (compact)
    const long long F = E.compact ? (long long)E.qcap[q] : T;
    sg.touch_off = touch_total;
    sg.n_touch = (int32_t)F;
    sg.pad = 0;
    if (res.block) {
      char* b = static_cast<char*>(res.block);
      res.ids = reinterpret_cast<int32_t*>(b);
      res.p = reinterpret_cast<double*>(b + off_p);
      if (keep_r) {
        res.rid = reinterpret_cast<int32_t*>(b + off_rid);
        res.rval = reinterpret_cast<double*>(b + off_rval);
      }
    }
    sg.out_ids = res.ids;
    sg.out_p = res.p;
    sg.out_rid = res.rid;
    sg.out_rval = res.rval;
    E.sweeping.push_back(res);
    E.state[q] = HS_SWEEP;
    total += N;
    touch_total += F;
    vol_bound += S.edges;
    nseg++;
  }
  if (nseg > 0) {
    E.hdr_h->nseg = nseg;
    E.hdr_h->total = (int32_t)total;
    E.hdr_h->touch_total = touch_total;
    HIPCHK(ctx, hipMemcpyAsync(a.segs, E.segs_h, sizeof(plc::SweepSeg) * nseg,
                               hipMemcpyHostToDevice, s));
    HIPCHK(ctx, hipMemcpyAsync(reinterpret_cast<char*>(a.ctl) + offsetof(plc::BatchCtl, sw_nseg),
                               E.hdr_h, sizeof(SweepHdr), hipMemcpyHostToDevice, s));
    if (ctx->timing) {
      HIPCHK(ctx, ev_pair(ctx->ev_sweep));
      HIPCHK(ctx, hipEventRecord(ctx->ev_sweep.a, s));
    }
    HIPCHK(ctx, plc::launch_batch_sweep(s, a, nseg, total, shape(g->batch_sweep, ctx->grid_sweep),
                                        E.compact));
    if (ctx->timing) HIPCHK(ctx, hipEventRecord(ctx->ev_sweep.b, s));
  }
  // 4. read back and wait
  HIPCHK(ctx, hipMemcpyAsync(E.slots_h, a.slots, sizeof(plc::Slot) * E.B, hipMemcpyDeviceToHost, s));
  HIPCHK(ctx, hipMemcpyAsync(E.ctl_h, a.ctl, sizeof(plc::BatchCtl), hipMemcpyDeviceToHost, s));
  HIPCHK(ctx, hipStreamSynchronize(s));
  if (E.ctl_h->fault) {
    ctx->broken = true;
    return PLC_E_HIP;
  }
  if (ctx->timing) {
    float ms = 0;
    if (scatter_ev) {
      HIPCHK(ctx, hipEventElapsedTime(&ms, scatter_ev->a, scatter_ev->b));
      ctx->t_scatter.ms += ms;
      ctx->t_scatter.launches++;
      ctx->t_scatter.units += E.ctl_h->e_total;
      ctx->t_scatter.entries += E.ctl_h->nf_total;
    }
    if (nseg > 0) {
      HIPCHK(ctx, hipEventElapsedTime(&ms, ctx->ev_sweep.a, ctx->ev_sweep.b));
      ctx->t_sweep.ms += ms;
      ctx->t_sweep.launches++;
      ctx->t_sweep.units += E.ctl_h->sw_etotal;
      ctx->t_sweep.entries += total;
    }
  }
  // 5. retire swept queries; note the ones whose frontier emptied
  for (int i = 0; i < nseg; i++) {
    const int q = E.segs_h[i].slot;
    const plc::Slot& S = E.slots_h[q];
    Result& res = E.sweeping[i];
    plc_result_info& info = res.info;
    info.status = !res.block ? PLC_E_NOMEM : (S.limited ? PLC_E_LIMIT : PLC_OK);
    info.rounds = S.rounds;
    info.pushes = S.pushes;
    info.edges = S.edges;
    info.support = S.support_cnt;
    info.kstar = S.kstar;
    info.cut = S.best_cut;
    info.vol = S.best_vol;
    info.phi = S.phi;
    info.r_nnz = S.rnnz;
    info.device_ns =
        S.t_done > S.t_admit ? (int64_t)((double)(S.t_done - S.t_admit) * ctx->clock_ns) : 0;
    info.flags = E.qflags[q];
    info.table_grows = E.compact ? E.qgrows[q] : 0;
    info.table_cap = E.compact ? E.qcap[q] : 0;
    if (S.fault) {
      ctx->broken = true;
      return PLC_E_HIP;
    }
    const uint64_t id = E.qid[q];
    ctx->results[id] = res;
    ctx->inflight.erase(id);
    if (done_ids && nfail + i < done_cap) done_ids[nfail + i] = id;
    E.state[q] = HS_FREE;
    E.qid[q] = 0;
    if (E.qblock[q]) {
      ctx->arena.release(E.qblock[q]);
      E.qblock[q] = nullptr;
      E.qcap[q] = 0;
      auto ins = E.touched_hint.emplace(E.qbucket[q], (double)S.touched_cnt);
      if (!ins.second) ins.first->second = 0.75 * ins.first->second + 0.25 * S.touched_cnt;
    }
  }
  E.sweeping.clear();
  std::fill(E.fresh.begin(), E.fresh.end(), 0);
  int running = 0;
  for (int q = 0; q < E.B; q++) {
    if (E.state[q] == HS_RUN && E.slots_h[q].status == plc::SL_PUSHED) E.state[q] = HS_PUSHED;
    running += E.state[q] != HS_FREE;
  }
  if (in_flight) *in_flight = running + (int32_t)E.queue.size();
  if (n_done) *n_done = nfail + nseg;
  return PLC_OK;
}

extern "C" plc_status plc_progress(plc_ctx* ctx, plc_graph* g, int32_t* in_flight,
                                   uint64_t* done_ids, int32_t done_cap, int32_t* n_done) {
  if (!ctx || !g || !ctx->graphs.count(g) || done_cap < 0) return PLC_E_INVALID;
  if (ctx->broken) return PLC_E_HIP;
  if (!g->batch) return PLC_E_INVALID;
  (void)hipSetDevice(ctx->device);
  return batch_step(ctx, g, in_flight, done_ids, done_cap, n_done, false);
}

extern "C" plc_status plc_poll(plc_ctx* ctx, uint64_t id, int32_t* done) {
  if (!ctx || !done) return PLC_E_INVALID;
  if (ctx->results.count(id)) { *done = 1; return PLC_OK; }
  if (ctx->inflight.count(id)) { *done = 0; return PLC_OK; }
  return PLC_E_NOTFOUND;
}

extern "C" plc_status plc_wait(plc_ctx* ctx, uint64_t id, int64_t timeout_us) {
  if (!ctx) return PLC_E_INVALID;
  const double t0 = now_ms();
  for (;;) {
    if (ctx->results.count(id)) return PLC_OK;
    auto it = ctx->inflight.find(id);
    if (it == ctx->inflight.end()) return PLC_E_NOTFOUND;
    if (ctx->broken) return PLC_E_HIP;
    if (timeout_us >= 0 && (now_ms() - t0) * 1e3 >= (double)timeout_us) return PLC_E_NOTREADY;
    plc_graph* g = it->second;
    if (!ctx->graphs.count(g) || !g->batch) return PLC_E_NOTFOUND;
    (void)hipSetDevice(ctx->device);
    plc_status st = batch_step(ctx, g, nullptr, nullptr, 0, nullptr, false);
    if (st != PLC_OK) return st;
  }
}

extern "C" size_t plc_query_bytes_estimate(const plc_graph* g, const plc_query* q) {
  if (!g || !q || !query_ok(g, *q)) return 0;
  const double ap = q->rule == PLC_RULE_OPT ? 2.0 * q->alpha / (1.0 + q->alpha) : q->alpha;
  const double w = 1.0 / (ap * q->eps);  // bound on the pushed volume outside the seed
  const double nn = (double)g->n;
  const double sup = std::min(nn, 1.0 + std::floor(w));
  const double tch = (double)touched_bound(g, *q);
  // result block: support ids + p, nonzero ids + values of r, each part 256-B aligned
  const double res = 12.0 * sup + 12.0 * tch + 4 * 256.0;
  const size_t state = g->ctx && g->ctx->opt.batch_state == PLC_STATE_COMPACT
                           ? table_block_bytes(table_cap_for(g, (int64_t)tch, (int64_t)tch))
                           : batch_slot_bytes(g);
  return state + (size_t)res;
}

extern "C" plc_status plc_run_batched(plc_ctx* ctx, plc_graph* g, const plc_query* q,
                                      int32_t count, uint64_t* ids, plc_result_info* infos) {
  if (!ctx || !g || !ctx->graphs.count(g) || count < 0 || (count > 0 && !q)) return PLC_E_INVALID;
  if (ctx->broken) return PLC_E_HIP;
  if (!g->batch) return PLC_E_INVALID;
  std::vector<uint64_t> local(count > 0 ? count : 1);
  plc_status first = plc_submit(ctx, g, q, count, local.data());
  if (first == PLC_E_HIP) return first;
  (void)hipSetDevice(ctx->device);
  int32_t left = 1;
  while (left > 0) {
    plc_status st = batch_step(ctx, g, &left, nullptr, 0, nullptr, true);
    if (st != PLC_OK) return st;
  }
  for (int32_t i = 0; i < count; i++) {
    if (ids) ids[i] = local[i];
    if (infos) {
      auto it = local[i] ? ctx->results.find(local[i]) : ctx->results.end();
      if (it == ctx->results.end()) {
        std::memset(&infos[i], 0, sizeof(plc_result_info));
        infos[i].status = PLC_E_INVALID;
      } else {
        infos[i] = it->second.info;
        if (infos[i].status != PLC_OK && first == PLC_OK) first = infos[i].status;
      }
    }
  }
  return first;
}

// ---------------------------------------------------------------- autotuner


// Run the sample once under the graph's current shapes; wall time in ms.
static plc_status tune_run(plc_ctx* ctx, plc_graph* g, const plc_query* q, int32_t count,
                           bool batched, double* ms) {
  std::vector<uint64_t> ids(count);
  const double t0 = now_ms();
  plc_status st = batched ? plc_run_batched(ctx, g, q, count, ids.data(), nullptr)
                          : plc_run(ctx, g, q, count, ids.data(), nullptr);
  *ms = now_ms() - t0;
  for (uint64_t id : ids)
    if (id) (void)plc_release(ctx, id);
  return st == PLC_E_HIP ? st : PLC_OK;
}

extern "C" plc_status plc_autotune(plc_ctx* ctx, plc_graph* g, const plc_query* sample,
                                   int32_t count, int32_t which, plc_tune* out) {
  if (!ctx || !g || !ctx->graphs.count(g) || !sample || count <= 0) return PLC_E_INVALID;
  if (ctx->broken) return PLC_E_HIP;
  if ((which & PLC_TUNE_BATCH) && !g->batch) return PLC_E_INVALID;
  const int cu = ctx->num_cu;
  const bool timing = ctx->timing;
  ctx->timing = false;
  int tried = 0;
  double best_plain = 0, best_batch = 0;
  if (which & PLC_TUNE_PLAIN) {
    const int selfs[] = {cu / 8, cu / 4, cu / 2, cu, 2 * cu};
    const int scats[] = {cu / 2, cu, 2 * cu, 4 * cu};
    const int sweeps[] = {cu, 2 * cu};
    double ms = 0;
    g->plain_self = cu; g->plain_scatter = 4 * cu; g->plain_sweep = 2 * cu;
    plc_status st = tune_run(ctx, g, sample, count, false, &ms);  // warm-up
    if (st != PLC_OK) { ctx->timing = timing; return st; }
    int bs = cu, bc = 4 * cu, bw = 2 * cu;
    double best = 1e300;
    for (int gs : selfs)
      for (int gc : scats)
        for (int gw : sweeps) {
          g->plain_self = gs; g->plain_scatter = gc; g->plain_sweep = gw;
          st = tune_run(ctx, g, sample, count, false, &ms);
          if (st != PLC_OK) { ctx->timing = timing; return st; }
          tried++;
          if (ms < best) { best = ms; bs = gs; bc = gc; bw = gw; }
        }
    g->plain_self = bs; g->plain_scatter = bc; g->plain_sweep = bw;
    // the binning threshold, unless the context fixed it: the default, four
    // times it, or no binning (graphs whose large rounds already hit few
    // lines per destination, such as ring-local ones, gain nothing from it)
    if (g->args.nbins > 0 && ctx->opt.bin_min_edges == 0) {
      const long long emins[] = {plc::kBinEmin, 4ll * plc::kBinEmin, plc::kBinOff};
      long long be = g->args.bin_emin;
      for (long long e : emins) {
        g->args.bin_emin = e;
        st = tune_run(ctx, g, sample, count, false, &ms);
        if (st != PLC_OK) { ctx->timing = timing; return st; }
        tried++;
        if (ms < best) { best = ms; be = e; }
      }
      g->args.bin_emin = be;
    }
    best_plain = best;
  }
  if (which & PLC_TUNE_BATCH) {
    const int selfs[] = {cu, 2 * cu};
    const int scats[] = {2 * cu, 4 * cu, 8 * cu, 16 * cu};
    double ms = 0;
    g->batch_self = cu; g->batch_scatter = 4 * cu; g->batch_sweep = 2 * cu;
    plc_status st = tune_run(ctx, g, sample, count, true, &ms);  // warm-up
    if (st != PLC_OK) { ctx->timing = timing; return st; }
    int bs = cu, bc = 4 * cu;
    double best = 1e300;
    for (int gs : selfs)
      for (int gc : scats) {
        g->batch_self = gs; g->batch_scatter = gc;
        st = tune_run(ctx, g, sample, count, true, &ms);
        if (st != PLC_OK) { ctx->timing = timing; return st; }
        tried++;
        if (ms < best) { best = ms; bs = gs; bc = gc; }
      }
    g->batch_self = bs; g->batch_scatter = bc;
    best_batch = best;
  }
  ctx->timing = timing;
  if (out) {
    out->plain_self = shape(g->plain_self, ctx->grid_self);
    out->plain_scatter = shape(g->plain_scatter, ctx->grid_scatter);
    out->plain_sweep = shape(g->plain_sweep, ctx->grid_sweep);
    out->batch_self = shape(g->batch_self, ctx->grid_self);
    out->batch_scatter = shape(g->batch_scatter, ctx->grid_scatter);
    out->batch_sweep = shape(g->batch_sweep, ctx->grid_sweep);
    out->plain_ms = best_plain;
    out->batch_ms = best_batch;
    out->candidates = tried;
    out->plain_bin_min_edges =
        !plc::bins_possible(g->args) ? -1 : (int32_t)g->args.bin_emin;
  }
  return PLC_OK;
}
