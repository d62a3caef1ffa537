// noalloc.cpp -- plc_run_noalloc: one plain PR-Nibble + sweep-cut query whose
// working state lives in a fixed device array of this library instead of a
// caller arena, for callers that cannot allocate device memory.
//
// The query runs the plain path's kernels (Sec. 3.3 push rounds, Sec. 3.1
// sweep) unchanged, launched directly (no recorded graphs): the per-vertex
// state records, frontier buffers, entry arrays, scan descriptors, sort and
// sweep buffers are carved from `scratch`, initialised by kernels on every
// call, and the result (support in sweep order, p on it) is copied into the
// caller's device buffers.  Nothing here calls hipMalloc, hipFree,
// hipHostMalloc, a stream or event constructor, or graph instantiation.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>

#include "../../include/plc.h"
#include "plc_device.h"

namespace {

constexpr size_t kScratchBytes = PLC_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

}  // namespace

// The working state of plc_run_noalloc.  Every GPU the library runs on holds
// its own copy until the process ends.  In host code this name is only a
// stand-in for the device symbol: its device address comes from
// hipGetSymbolAddress (scratch_base below) and only that address is used.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_mu;
void* g_base[kMaxDevices] = {};

// Device address of `scratch` on `device` (the current device), looked up
// once per device.
void* scratch_base(int device) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (device < 0 || device >= kMaxDevices) return nullptr;
  if (!g_base[device]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    g_base[device] = p;
  }
  return g_base[device];
}

// Bump carving of the scratch array (256-byte aligned blocks).
struct Carver {
  char* base;
  size_t used = 0;
  bool over = false;
  void* take(size_t bytes) {
    const size_t off = (used + 255) & ~(size_t)255;
    if (off + bytes > kScratchBytes) {
      over = true;
      return nullptr;
    }
    used = off + bytes;
    return base ? base + off : nullptr;
  }
};

// Lay the plain path's state for a graph of n vertices and `arcs` arcs out in
// the scratch array (base may be null to measure).  Returns false when it
// does not fit.
bool layout(char* base, int64_t n, int64_t arcs, plc::PlainArgs& a) {
  Carver cv{base};
  const size_t N = (size_t)n;
  const size_t nscan = N / plc::kScanBlock + 2;
  const size_t ntile = (size_t)arcs / plc::kEdgeTile + 2;
  a = plc::PlainArgs{};
  a.n = n;
  a.vol_total = arcs;
  a.vr = static_cast<plc::VRec*>(cv.take(sizeof(plc::VRec) * N));
  a.p = static_cast<double*>(cv.take(8 * N));
  a.ctl = static_cast<plc::Ctl*>(cv.take(sizeof(plc::Ctl)));
  a.fbuf0 = static_cast<int32_t*>(cv.take(4 * N));
  a.fbuf1 = static_cast<int32_t*>(cv.take(4 * N));
  a.coef = static_cast<double*>(cv.take(8 * N));
  a.estart = static_cast<int64_t*>(cv.take(8 * N));
  a.rowp = static_cast<int64_t*>(cv.take(8 * N));
  a.tile_start = static_cast<int32_t*>(cv.take(4 * ntile));
  a.tile_cap = (int64_t)ntile;
  a.desc_cap = (int32_t)nscan;
  for (int s = 0; s < plc::NUM_SCANS; s++)
    a.desc[s] = static_cast<unsigned long long*>(cv.take(2 * 8 * nscan));
  a.support = static_cast<int32_t*>(cv.take(4 * N));
  a.touched = static_cast<int32_t*>(cv.take(4 * N));
  a.sbuf[0] = static_cast<plc::SortElem*>(cv.take(sizeof(plc::SortElem) * N));
  a.sbuf[1] = static_cast<plc::SortElem*>(cv.take(sizeof(plc::SortElem) * N));
  a.sdeg = static_cast<int32_t*>(cv.take(4 * N));
  a.svol = static_cast<int64_t*>(cv.take(8 * N));
  a.scnt = static_cast<int32_t*>(cv.take(4 * N));
  a.sp = static_cast<double*>(cv.take(8 * N));
  a.sid = static_cast<int32_t*>(cv.take(4 * N));
  a.rid = static_cast<int32_t*>(cv.take(4 * N));
  a.rval = static_cast<double*>(cv.take(8 * N));
  a.bbest = static_cast<long long*>(cv.take(24 * nscan));
  a.hk_r1 = static_cast<double*>(cv.take(8 * N));  // cleared by the graph init kernel
  a.hk_tl[0] = a.touched;
  a.nbins = 0;  // the atomic scatter only: the binned form needs buffers sized by the graph
  return !cv.over;
}

// Clear `words` 8-byte words (kernels, not hipMemsetAsync, so that the
// sequence stays valid inside a captured graph).
__global__ void k_noalloc_clear(unsigned long long* p, size_t words) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < words;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

}  // namespace

extern "C" plc_status plc_run_noalloc(int32_t device, void* hip_stream, int64_t n,
                                      int64_t num_arcs, const int64_t* d_off,
                                      const int32_t* d_nbr, const plc_query* q,
                                      int32_t* d_sweep_ids, double* d_sweep_p,
                                      plc_result_info* info) {
  if (!d_off || !q || !d_sweep_ids || !d_sweep_p || !info) return PLC_E_INVALID;
  if (n <= 0 || num_arcs < 0 || (num_arcs > 0 && !d_nbr) || n >= (int64_t)INT32_MAX)
    return PLC_E_INVALID;
  if (!(q->alpha > 0.0 && q->alpha < 1.0) || !std::isfinite(q->eps) || !(q->eps >= 1e-250) ||
      (q->rule != PLC_RULE_OPT && q->rule != PLC_RULE_ORIG) || (q->flags & ~PLC_QF_ALL) != 0u ||
      q->seed < 0 || q->seed >= n)
    return PLC_E_INVALID;
  plc::PlainArgs a;
  if (!layout(nullptr, n, num_arcs, a)) return PLC_E_NOMEM;  // larger than the scratch array
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return PLC_E_INVALID;
  if (hipSetDevice(device) != hipSuccess) return PLC_E_HIP;
  char* base = static_cast<char*>(scratch_base(device));
  if (!base) return PLC_E_HIP;
  layout(base, n, num_arcs, a);
  a.off = d_off;
  a.nbr = d_nbr;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  int ncu = 256;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
      ncu <= 0)
    ncu = 256;
  int khz = 0;
  double clock_ns = 10.0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) == hipSuccess && khz > 0)
    clock_ns = 1e6 / (double)khz;
  // the seed must have a neighbour (two offsets read back into the stack)
  int64_t so[2] = {0, 0};
  if (hipMemcpyAsync(so, d_off + q->seed, sizeof(so), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return PLC_E_HIP;
  if (so[1] - so[0] < 1) return PLC_E_INVALID;
  const int gs = ncu, gc = 4 * ncu, gw = 2 * ncu, gb = 4 * ncu;
  const int max_rounds = 1 << 20;
#define NA_CHK(expr)                  \
  do {                                \
    if ((expr) != hipSuccess) {       \
      (void)hipGetLastError();        \
      return PLC_E_HIP;               \
    }                                 \
  } while (0)
  // state: records and p over all n (k_graph_init), control block and scan
  // descriptors zeroed, then the seed
  hipLaunchKernelGGL(k_noalloc_clear, dim3(1), dim3(256), 0, s,
                     reinterpret_cast<unsigned long long*>(a.ctl), sizeof(plc::Ctl) / 8);
  NA_CHK(hipGetLastError());
  for (int k = 0; k < plc::NUM_SCANS; k++) {
    hipLaunchKernelGGL(k_noalloc_clear, dim3(16), dim3(256), 0, s, a.desc[k],
                       2 * (size_t)a.desc_cap);
    NA_CHK(hipGetLastError());
  }
  NA_CHK(plc::launch_graph_init(s, a));
  NA_CHK(plc::launch_query_init(s, a, q->seed, (int32_t)q->rule, q->alpha, q->eps, max_rounds));
  plc::Ctl h;
  std::memset(&h, 0, sizeof(h));
  // rounds in chunks, each followed by a read-back of the control block
  for (int chunk = 8;; chunk = chunk < 64 ? 2 * chunk : 64) {
    for (int i = 0; i < chunk; i++) {
      NA_CHK(plc::launch_self(s, a, gs));
      NA_CHK(plc::launch_scatter(s, a, gc, nullptr, nullptr, -1, gb));
    }
    NA_CHK(hipMemcpyAsync(&h, a.ctl, sizeof(h), hipMemcpyDeviceToHost, s));
    NA_CHK(hipStreamSynchronize(s));
    if (h.fault || (h.status != plc::ST_PUSH && h.status != plc::ST_LIMIT)) return PLC_E_HIP;
    if (h.status == plc::ST_LIMIT || h.cnt[h.round & 1] == 0) break;
  }
  int64_t bound = 1024;
  while (bound < h.support_cnt) bound <<= 1;
  NA_CHK(plc::launch_sweep(s, a, gw, bound));
  NA_CHK(hipMemcpyAsync(&h, a.ctl, sizeof(h), hipMemcpyDeviceToHost, s));
  NA_CHK(hipStreamSynchronize(s));
  if (h.status != plc::ST_SWEPT || h.fault || h.N < 0 || h.N > n) return PLC_E_HIP;
  NA_CHK(plc::launch_copy_result(s, a, d_sweep_ids, d_sweep_p, nullptr, nullptr, h.N, 0, gw));
  NA_CHK(hipStreamSynchronize(s));
#undef NA_CHK
  std::memset(info, 0, sizeof(*info));
  info->status = h.limited ? PLC_E_LIMIT : PLC_OK;
  info->rounds = h.round;
  info->pushes = h.pushes;
  info->edges = h.edges;
  info->support = h.N;
  info->kstar = h.kstar;
  info->cut = h.best_cut;
  info->vol = h.best_vol;
  info->phi = h.phi;
  info->r_nnz = h.rnnz;
  info->launches = h.steps;
  info->loop_rounds = h.loop_rounds;
  info->loop_edges = h.loop_edges;
  info->device_ns = h.t_end > h.t_start ? (int64_t)((double)(h.t_end - h.t_start) * clock_ns) : 0;
  info->flags = q->flags;
  return PLC_OK;
}
