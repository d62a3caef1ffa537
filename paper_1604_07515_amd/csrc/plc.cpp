// plc.cpp -- host side of libplc: the C ABI declared in include/plc.h.
//
// A context owns a view of the caller's device arena, the caller's stream and
// a pinned host mirror of the device control block.  plc_run drives the plain
// path: per query it queues the seed initialisation, a chunk of rounds whose
// kernels exit at once after the frontier empties, the whole sweep sequence
// (which only runs once the push has finished) and a read-back of the control
// block, then synchronises once; if the frontier was still non-empty it
// queues another, larger chunk.  Results are copied device-to-device into an
// exact-size arena block, and the dense per-vertex state is reset through the
// touched list.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <new>
#include <set>
#include <thread>
#include <vector>

#include "../../include/plc.h"
#include "arena.h"
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

struct KTime {
  int64_t launches = 0;
  double ms = 0;
  int64_t units = 0;
  int64_t entries = 0;
};

}  // namespace

struct plc_graph {
  plc_ctx* ctx = nullptr;
  int64_t n = 0, arcs = 0, maxdeg = 0;
  size_t bytes = 0;
  std::vector<void*> blocks;
  std::vector<int32_t> deg;  // host copy of degrees, for query validation
  PlainArgs args{};
};

struct plc_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  Arena arena;
  plc_options opt{};
  Ctl* ctl_host = nullptr;  // pinned
  std::map<uint64_t, Result> results;
  uint64_t next_id = 1;
  bool broken = false;
  std::set<plc_graph*> graphs;
  int num_cu = 256;
  int grid_self = 256, grid_scatter = 1024, grid_sweep = 512;
  int chunk_rounds = 16;
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
  if (c->opt.batch_slots <= 0) c->opt.batch_slots = 256;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
    c->num_cu = prop.multiProcessorCount;
  c->grid_self = c->num_cu;
  c->grid_scatter = 4 * c->num_cu;
  c->grid_sweep = 2 * c->num_cu;
  if (hipHostMalloc(reinterpret_cast<void**>(&c->ctl_host), sizeof(Ctl), hipHostMallocDefault) !=
      hipSuccess) {
    delete c;
    return PLC_E_HIP;
  }
  std::memset(c->ctl_host, 0, sizeof(Ctl));
  *out = c;
  return PLC_OK;
}

static void free_events(plc_ctx* c) {
  for (auto& e : c->ev_scatter) { (void)hipEventDestroy(e.a); (void)hipEventDestroy(e.b); }
  for (auto& e : c->ev_self) { (void)hipEventDestroy(e.a); (void)hipEventDestroy(e.b); }
  c->ev_scatter.clear();
  c->ev_self.clear();
  if (c->ev_sweep.a) { (void)hipEventDestroy(c->ev_sweep.a); (void)hipEventDestroy(c->ev_sweep.b); }
  c->ev_sweep = EventPair{};
}

extern "C" plc_status plc_destroy(plc_ctx* ctx) {
  if (!ctx) return PLC_E_INVALID;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  for (plc_graph* g : ctx->graphs) delete g;
  free_events(ctx);
  if (ctx->ctl_host) (void)hipHostFree(ctx->ctl_host);
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
  const size_t nsort = N / plc::kSortTile + 2;
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
  for (int s = 0; s < plc::NUM_SCANS; s++)
    a.desc[s] = static_cast<plc::ScanDesc*>(take(sizeof(plc::ScanDesc) * nscan));
  a.support = static_cast<int32_t*>(take(4 * N));
  a.touched = static_cast<int32_t*>(take(4 * N));
  a.keyA = static_cast<unsigned long long*>(take(8 * N));
  a.keyB = static_cast<unsigned long long*>(take(8 * N));
  a.idA = static_cast<int32_t*>(take(4 * N));
  a.idB = static_cast<int32_t*>(take(4 * N));
  a.hist = static_cast<uint32_t*>(take(4 * 256 * nsort));
  a.sdeg = static_cast<int32_t*>(take(4 * N));
  a.svol = static_cast<int64_t*>(take(8 * N));
  a.scnt = static_cast<int32_t*>(take(4 * N));
  a.sp = static_cast<double*>(take(8 * N));
  a.rid = static_cast<int32_t*>(take(4 * N));
  a.rval = static_cast<double*>(take(8 * N));
  a.bbest = static_cast<long long*>(take(24 * nscan));
  a.hist_tiles = (int32_t)nsort;
  a.tile_cap = (int64_t)ntile;
  int bits = 1;
  while (bits < 31 && ((int64_t)1 << bits) < n) bits++;
  a.id_bits = bits;
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
  if (hipMemsetAsync(a.ctl, 0, sizeof(Ctl), s) != hipSuccess) return fail();
  for (int k = 0; k < plc::NUM_SCANS; k++)
    if (hipMemsetAsync(a.desc[k], 0, sizeof(plc::ScanDesc) * nscan, s) != hipSuccess) return fail();
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
  return true;
}

static hipError_t ev_pair(EventPair& e) {
  if (e.a) return hipSuccess;
  hipError_t r = hipEventCreate(&e.a);
  if (r != hipSuccess) return r;
  return hipEventCreate(&e.b);
}

// Queue `rounds` rounds; with timing on, bracket each kernel with events.
static hipError_t queue_rounds(plc_ctx* ctx, const PlainArgs& a, int first, int rounds) {
  hipStream_t s = ctx->stream;
  for (int i = 0; i < rounds; i++) {
    hipError_t r;
    if (ctx->timing) {
      size_t k = (size_t)(first + i);
      while (ctx->ev_self.size() <= k) ctx->ev_self.emplace_back();
      while (ctx->ev_scatter.size() <= k) ctx->ev_scatter.emplace_back();
      if ((r = ev_pair(ctx->ev_self[k])) != hipSuccess) return r;
      if ((r = ev_pair(ctx->ev_scatter[k])) != hipSuccess) return r;
      (void)hipEventRecord(ctx->ev_self[k].a, s);
      if ((r = plc::launch_self(s, a, ctx->grid_self)) != hipSuccess) return r;
      (void)hipEventRecord(ctx->ev_self[k].b, s);
      (void)hipEventRecord(ctx->ev_scatter[k].a, s);
      if ((r = plc::launch_scatter(s, a, ctx->grid_scatter)) != hipSuccess) return r;
      (void)hipEventRecord(ctx->ev_scatter[k].b, s);
    } else {
      if ((r = plc::launch_self(s, a, ctx->grid_self)) != hipSuccess) return r;
      if ((r = plc::launch_scatter(s, a, ctx->grid_scatter)) != hipSuccess) return r;
    }
  }
  return hipSuccess;
}

static plc_status run_one(plc_ctx* ctx, plc_graph* g, const plc_query& q, uint64_t* id_out,
                          plc_result_info* info_out) {
  hipStream_t s = ctx->stream;
  const PlainArgs& a = g->args;
  HIPCHK(ctx, plc::launch_query_init(s, a, q.seed, (int32_t)q.rule, q.alpha, q.eps,
                                     ctx->opt.max_rounds));
  int queued = 0;
  int chunk = std::max(2, ctx->chunk_rounds);
  Ctl& h = *ctx->ctl_host;
  for (;;) {
    HIPCHK(ctx, queue_rounds(ctx, a, queued, chunk));
    queued += chunk;
    if (ctx->timing) {
      HIPCHK(ctx, ev_pair(ctx->ev_sweep));
      HIPCHK(ctx, hipEventRecord(ctx->ev_sweep.a, s));
    }
    HIPCHK(ctx, plc::launch_sweep(s, a, ctx->grid_sweep));
    if (ctx->timing) HIPCHK(ctx, hipEventRecord(ctx->ev_sweep.b, s));
    HIPCHK(ctx, hipMemcpyAsync(&h, a.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    if (h.status == plc::ST_SWEPT) break;
    if (h.status != plc::ST_PUSH) {  // unexpected state: device-side fault
      ctx->broken = true;
      return PLC_E_HIP;
    }
    chunk = std::min(chunk * 2, 256);
  }
  // Next query starts with a chunk that covers this one's rounds.
  ctx->chunk_rounds = std::min(256, std::max(4, h.round + 2));
  if (h.overflow) {
    ctx->broken = true;
    return PLC_E_HIP;
  }
  if (ctx->timing) {
    float ms = 0;
    for (int i = 0; i < h.round && i < queued; i++) {
      HIPCHK(ctx, hipEventElapsedTime(&ms, ctx->ev_scatter[i].a, ctx->ev_scatter[i].b));
      ctx->t_scatter.ms += ms;
      ctx->t_scatter.launches++;
      HIPCHK(ctx, hipEventElapsedTime(&ms, ctx->ev_self[i].a, ctx->ev_self[i].b));
      ctx->t_self.ms += ms;
      ctx->t_self.launches++;
    }
    ctx->t_scatter.units += h.edges;
    ctx->t_scatter.entries += h.pushes;
    ctx->t_self.units += h.pushes;
    ctx->t_self.entries += h.pushes;
    HIPCHK(ctx, hipEventElapsedTime(&ms, ctx->ev_sweep.a, ctx->ev_sweep.b));
    ctx->t_sweep.ms += ms;
    ctx->t_sweep.launches++;
    ctx->t_sweep.units += h.etotal;
    ctx->t_sweep.entries += h.N;
  }

  Result res;
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
  size_t N = (size_t)h.N, R = (size_t)h.rnnz;
  size_t off_p = (4 * N + 255) & ~(size_t)255;
  size_t off_rid = off_p + ((8 * N + 255) & ~(size_t)255);
  size_t off_rval = off_rid + ((4 * R + 255) & ~(size_t)255);
  size_t total = off_rval + 8 * R;
  plc_status st = PLC_OK;
  res.block = ctx->arena.alloc(total);
  if (!res.block) {
    info.status = PLC_E_NOMEM;
    st = PLC_E_NOMEM;
  } else {
    char* b = static_cast<char*>(res.block);
    res.ids = reinterpret_cast<int32_t*>(b);
    res.p = reinterpret_cast<double*>(b + off_p);
    res.rid = reinterpret_cast<int32_t*>(b + off_rid);
    res.rval = reinterpret_cast<double*>(b + off_rval);
    const int32_t* sorted = h.sort_flip ? a.idB : a.idA;
    if (N) {
      HIPCHK(ctx, hipMemcpyAsync(res.ids, sorted, 4 * N, hipMemcpyDeviceToDevice, s));
      HIPCHK(ctx, hipMemcpyAsync(res.p, a.sp, 8 * N, hipMemcpyDeviceToDevice, s));
    }
    if (R) {
      HIPCHK(ctx, hipMemcpyAsync(res.rid, a.rid, 4 * R, hipMemcpyDeviceToDevice, s));
      HIPCHK(ctx, hipMemcpyAsync(res.rval, a.rval, 8 * R, hipMemcpyDeviceToDevice, s));
    }
  }
  HIPCHK(ctx, plc::launch_cleanup(s, a, ctx->grid_sweep));
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
    plc_status st = run_one(ctx, g, q[i], ids ? &ids[i] : nullptr, infos ? &infos[i] : nullptr);
    if (st == PLC_E_HIP) return st;
    if (st != PLC_OK && first == PLC_OK) first = st;
  }
  if (hipStreamSynchronize(ctx->stream) != hipSuccess) {
    ctx->broken = true;
    return PLC_E_HIP;
  }
  return first;
}

extern "C" plc_status plc_result_info_get(plc_ctx* ctx, uint64_t id, plc_result_info* out) {
  if (!ctx || !out) return PLC_E_INVALID;
  auto it = ctx->results.find(id);
  if (it == ctx->results.end()) return PLC_E_NOTFOUND;
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
  size_t N = (size_t)r.info.support, R = (size_t)r.info.r_nnz;
  if (sweep_ids && N) HIPCHK(ctx, hipMemcpyAsync(sweep_ids, r.ids, 4 * N, hipMemcpyDeviceToHost, s));
  if (sweep_p && N) HIPCHK(ctx, hipMemcpyAsync(sweep_p, r.p, 8 * N, hipMemcpyDeviceToHost, s));
  if (r_ids && R) HIPCHK(ctx, hipMemcpyAsync(r_ids, r.rid, 4 * R, hipMemcpyDeviceToHost, s));
  if (r_vals && R) HIPCHK(ctx, hipMemcpyAsync(r_vals, r.rval, 8 * R, hipMemcpyDeviceToHost, s));
  HIPCHK(ctx, hipStreamSynchronize(s));
  return PLC_OK;
}

extern "C" plc_status plc_release(plc_ctx* ctx, uint64_t id) {
  if (!ctx) return PLC_E_INVALID;
  auto it = ctx->results.find(id);
  if (it == ctx->results.end()) return PLC_E_NOTFOUND;
  if (it->second.block) {
    // the block may still be the target of queued copies
    (void)hipSetDevice(ctx->device);
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) {
      ctx->broken = true;
      return PLC_E_HIP;
    }
    ctx->arena.release(it->second.block);
  }
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
