// zmc_api.hip -- host side of libzmc: descriptor validation, the work
// planner, and the C ABI entry points declared in include/zmc.h.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <thread>
#include <vector>

#include "zmc.h"
#include "zmc_device.hpp"
#include "zmc_internal.hpp"
#include "zmc_trace.hpp"

namespace {
thread_local char g_err[512] = "";
}  // namespace

namespace zmc {

zmc_status fail(zmc_status st, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return st;
}

zmc_status ok() {
  g_err[0] = '\0';
  return ZMC_OK;
}

int log_level() {
  static const int level = [] {
    const char* env = getenv("ZMC_LOG");
    return (env && *env) ? atoi(env) : 0;
  }();
  return level;
}

void log(int level, const char* fmt, ...) {
  if (log_level() < level) return;
  char line[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(line, sizeof(line), fmt, ap);
  va_end(ap);
  fprintf(stderr, "[zmc] %s\n", line);
}

// Every plan (make_plan for single scans, plan_tiles for batches and the
// server) passes here before any ScanParams is filled from it: the pieces
// [sp * gps, min((sp + 1) * gps, groups)) must cover the groups exactly once
// with none empty, since the device loops assume j0 <= the piece's last group.
zmc_status check_pieces(uint64_t groups, uint64_t gps, uint64_t splits) {
  if (groups < 1 || gps < 1 || splits < 1 || splits > 0x7FFFFFFFull ||
      (splits - 1) * gps >= groups || splits * gps < groups)
    return fail(ZMC_E_INVALID, "plan: %llu pieces of %llu groups do not cover %llu groups "
                "exactly once", (unsigned long long)splits, (unsigned long long)gps,
                (unsigned long long)groups);
  return ZMC_OK;
}

}  // namespace zmc

namespace {

using zmc::fail;
using zmc::ok;

#define ZMC_HIP(call)                                                              \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess)                                                          \
      return fail(e_ == hipErrorOutOfMemory ? ZMC_E_NOMEM : ZMC_E_DEVICE,          \
                  "%s failed: %s", #call, hipGetErrorString(e_));                  \
  } while (0)

constexpr uint64_t kMaxG = (uint64_t)1 << 62;

// Validation rules of the descriptor (include/zmc.h).
zmc_status validate(const zmc_scan_desc* d, uint64_t* G_out) {
  if (d == nullptr) return fail(ZMC_E_INVALID, "descriptor is NULL");
  if (d->M < 0 || d->M > zmc::kMaxParams)
    return fail(ZMC_E_INVALID, "M = %d outside 0..%d", d->M, zmc::kMaxParams);
  if (d->M > 0 && d->axis_len == nullptr) return fail(ZMC_E_INVALID, "axis_len is NULL with M > 0");
  uint64_t G = 1;
  for (int l = 0; l < d->M; ++l) {
    const int64_t L = d->axis_len[l];
    if (L < 1) return fail(ZMC_E_INVALID, "axis_len[%d] = %lld < 1", l, (long long)L);
    if (G > kMaxG / (uint64_t)L) return fail(ZMC_E_INVALID, "grid larger than 2^62 points");
    G *= (uint64_t)L;
  }
  if (d->N < 1 || d->N > zmc::kMaxDims)
    return fail(ZMC_E_INVALID, "N = %d outside 1..%d", d->N, zmc::kMaxDims);
  if (d->lo == nullptr || d->hi == nullptr) return fail(ZMC_E_INVALID, "lo or hi is NULL");
  for (int k = 0; k < d->N; ++k) {
    if (!isfinite(d->lo[k]) || !isfinite(d->hi[k]))
      return fail(ZMC_E_INVALID, "box edge %d is not finite", k);
    if (!(d->lo[k] < d->hi[k])) return fail(ZMC_E_INVALID, "box edge %d: lo >= hi", k);
  }
  if (d->samples < 2) return fail(ZMC_E_INVALID, "samples = %llu < 2", (unsigned long long)d->samples);
  if (d->samples > kMaxG / (uint64_t)d->N) return fail(ZMC_E_INVALID, "samples * N exceeds 2^62");
  switch (d->family) {
    case ZMC_SIN_SUM:
    case ZMC_CONST:
    case ZMC_LINEAR:
      break;
    case ZMC_GAUSS:
      if (d->M > d->N) return fail(ZMC_E_INVALID, "GAUSS needs M <= N (M = %d, N = %d)", d->M, d->N);
      break;
    case ZMC_COSEXP:
      if (d->M != 4 || d->N < 2)
        return fail(ZMC_E_INVALID, "COSEXP needs M = 4 and N >= 2 (M = %d, N = %d)", d->M, d->N);
      break;
    case ZMC_USER:
      if (d->integrand == nullptr) return fail(ZMC_E_INVALID, "ZMC_USER needs desc->integrand");
      break;
    default:
      return fail(ZMC_E_INVALID, "unknown family %d", d->family);
  }
  if (d->precision != ZMC_FP64 && d->precision != ZMC_FP32_MERGE64)
    return fail(ZMC_E_INVALID, "unknown precision %d", d->precision);
  if (d->family == ZMC_USER) {
    if (d->n_params < 0 || d->n_params > zmc::kMaxUserParams)
      return fail(ZMC_E_INVALID, "n_params = %d outside 0..%d", d->n_params, zmc::kMaxUserParams);
    if (d->n_params > 0 && d->params == nullptr) return fail(ZMC_E_INVALID, "params is NULL with n_params > 0");
    for (int i = 0; i < d->n_params; ++i)
      if (!isfinite(d->params[i])) return fail(ZMC_E_INVALID, "params[%d] is not finite", i);
  } else if (d->n_params != 0) {
    return fail(ZMC_E_INVALID, "n_params = %d; these families take none", d->n_params);
  }
  if (G_out) *G_out = G;
  return ok();
}

std::mutex g_cu_mu;
std::vector<int> g_cu_cache;

zmc_status device_cu_count(int* cu) {
  int dev = 0;
  ZMC_HIP(hipGetDevice(&dev));
  {
    std::lock_guard<std::mutex> lk(g_cu_mu);
    if ((int)g_cu_cache.size() > dev && g_cu_cache[dev] > 0) {
      *cu = g_cu_cache[dev];
      return ZMC_OK;
    }
  }
  int v = 0;
  ZMC_HIP(hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev));
  if (v <= 0) return fail(ZMC_E_DEVICE, "device reports %d compute units", v);
  std::lock_guard<std::mutex> lk(g_cu_mu);
  if ((int)g_cu_cache.size() <= dev) g_cu_cache.resize(dev + 1, 0);
  g_cu_cache[dev] = v;
  *cu = v;
  return ZMC_OK;
}

uint64_t cdiv(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

// Work planner.  Point-major when the grid alone gives every SIMD at least one
// wave; the sample range is then cut into enough pieces that the launch holds
// ~16 waves per wave slot (so the last round of blocks is a small fraction
// of the run), each piece keeping >= 64 groups (256 samples) per lane.
// Otherwise sample-major with enough blocks per point for ~4 waves per slot
// and >= 16 groups per lane.
constexpr uint64_t kMaxGridX = (uint64_t)1 << 30;
constexpr int kMaxSplits = 65535;
constexpr uint64_t kMaxWorkspace = (uint64_t)8 << 30;
constexpr uint64_t kDefaultChunk = (uint64_t)1 << 24;  // points per chunk of a chunked scan
// Largest device allocation the entry points will size (64 PiB, far above any
// device): products such as 16 x splits x G are checked against it before they
// are formed, so that no size can wrap around 2^64.
constexpr uint64_t kMaxBytes = (uint64_t)1 << 56;
size_t align256(size_t x) { return (x + 255) / 256 * 256; }

zmc_status make_plan(const zmc_scan_desc* d, uint64_t G, const zmc_launch_opts* o, zmc::Plan* pl) {
  int cu = (o && o->cu_count > 0) ? o->cu_count : 0;
  if (cu == 0) {
    zmc_status st = device_cu_count(&cu);
    if (st != ZMC_OK) return st;
  }
  const uint64_t slots = (uint64_t)cu * 4 * 8;  // wave slots: 4 SIMDs x 8 waves
  const uint64_t groups = cdiv(d->samples, 4);
  int mode = o ? o->mode : ZMC_MODE_AUTO;
  if (mode == ZMC_MODE_AUTO)
    mode = (G >= (uint64_t)cu * 4 * 64) ? ZMC_MODE_POINT_MAJOR : ZMC_MODE_SAMPLE_MAJOR;
  if (mode != ZMC_MODE_POINT_MAJOR && mode != ZMC_MODE_SAMPLE_MAJOR)
    return fail(ZMC_E_INVALID, "unknown mode %d", mode);
  int block = (o && o->block > 0) ? o->block : 256;
  if (block < 64 || block > 1024 || block % 64 != 0)
    return fail(ZMC_E_INVALID, "block = %d: needs a multiple of 64 in 64..1024", block);
  if (mode == ZMC_MODE_POINT_MAJOR && block > 256)
    return fail(ZMC_E_INVALID, "point-major blocks hold at most 256 threads");
  if (d->N > zmc::kAnyMaxDims && block > 256)
    return fail(ZMC_E_INVALID, "blocks of scans with N > %d hold at most 256 threads", zmc::kAnyMaxDims);
  uint64_t splits = (o && o->splits > 0) ? (uint64_t)o->splits : 0;
  if (splits == 0) {
    if (mode == ZMC_MODE_POINT_MAJOR) {
      const uint64_t waves = cdiv(G, 64);
      splits = cdiv(16 * slots, waves);
      uint64_t cap = groups / 64;
      if (cap < 1) cap = 1;
      if (splits > cap) splits = cap;
    } else {
      const uint64_t waves = G * (uint64_t)(block / 64);
      splits = cdiv(4 * slots, waves);
      uint64_t cap = groups / ((uint64_t)block * 16);
      if (cap < 1) cap = 1;
      if (splits > cap) splits = cap;
    }
    if (splits < 1) splits = 1;
    while (splits > 1 && 16.0 * (double)splits * (double)G > (double)kMaxWorkspace) splits /= 2;
  }
  if (splits > (uint64_t)kMaxSplits) splits = kMaxSplits;
  if (splits > groups) splits = groups;
  const uint64_t gps = cdiv(groups, splits);
  splits = cdiv(groups, gps);  // no empty piece
  zmc_status pst = zmc::check_pieces(groups, gps, splits);
  if (pst != ZMC_OK) return pst;
  if (splits > 1 && G > kMaxBytes / (16 * splits))
    return fail(ZMC_E_NOMEM, "split partials of %llu points x %llu pieces exceed %llu bytes",
                (unsigned long long)G, (unsigned long long)splits, (unsigned long long)kMaxBytes);
  pl->mode = mode;
  pl->block = block;
  pl->splits = (int)splits;
  pl->groups = groups;
  pl->gps = gps;
  pl->point_blocks = cdiv(G, (uint64_t)block);
  const uint64_t gx = (mode == ZMC_MODE_POINT_MAJOR) ? pl->point_blocks : G;
  pl->grid_x = gx < kMaxGridX ? gx : kMaxGridX;
  pl->workspace_bytes = splits > 1 ? 16 * splits * G : 0;
  zmc::log(2, "plan: G=%llu n=%llu N=%d %s block=%d splits=%llu groups/piece=%llu blocks=%llu "
           "workspace=%llu B", (unsigned long long)G, (unsigned long long)d->samples, d->N,
           mode == ZMC_MODE_POINT_MAJOR ? "point-major" : "sample-major", block,
           (unsigned long long)splits, (unsigned long long)gps,
           (unsigned long long)(pl->grid_x * splits), (unsigned long long)pl->workspace_bytes);
  return ZMC_OK;
}

void fill_params(const zmc_scan_desc* d, uint64_t G, const zmc::Plan& pl, const double* d_axis,
                 double* d_f, double* d_sigma, zmc::ScanParams* p, uint64_t g_base = 0) {
  memset(p, 0, sizeof(*p));
  p->G = G;
  p->g_base = g_base;
  p->n = d->samples;
  p->n_groups = pl.groups;
  p->gps = pl.gps;
  p->seed = d->seed;
  p->point_blocks = pl.point_blocks;
  p->M = d->M;
  p->N = d->N;
  p->splits = pl.splits;
  p->family = d->family;
  p->fast_counter =
      (g_base + G <= ((uint64_t)1 << 32) && pl.groups * (uint64_t)d->N <= ((uint64_t)1 << 32)) ? 1 : 0;
  int64_t off = 0;
  uint64_t stride = 1;
  for (int l = d->M - 1; l >= 0; --l) {
    p->axis_stride[l] = stride;
    stride *= (uint64_t)d->axis_len[l];
  }
  for (int l = 0; l < d->M; ++l) {
    p->axis_len[l] = d->axis_len[l];
    p->axis_off[l] = off;
    off += d->axis_len[l];
  }
  double vol = 1.0;
  for (int k = 0; k < d->N; ++k) {
    p->lo[k] = d->lo[k];
    p->hi[k] = d->hi[k];
    vol *= d->hi[k] - d->lo[k];
  }
  p->vol = vol;
  p->n_params = d->family == ZMC_USER ? d->n_params : 0;
  for (int i = 0; i < p->n_params; ++i) p->params[i] = d->params[i];
  p->axis = d_axis;
  p->f = d_f;
  p->sigma = d_sigma;
}

}  // namespace

namespace zmc {
zmc_status validate_desc(const zmc_scan_desc* d, uint64_t* G) { return validate(d, G); }
zmc_status cu_count(int* cu) { return device_cu_count(cu); }
void fill_scan_params(const zmc_scan_desc* d, uint64_t G, const Plan& pl, const double* d_axis,
                      double* d_f, double* d_sigma, ScanParams* p) {
  fill_params(d, G, pl, d_axis, d_f, d_sigma, p);
}
}  // namespace zmc

namespace {

// ---------------------------------------------------------------------------
// Split-partial workspaces of zmc_scan_device(_ex).  The stream-ordered
// allocator of HIP 7.2 makes the calling thread wait, at hipMallocAsync /
// hipFreeAsync, for the device work that last used the block it hands out
// (measured: each call's enqueue then lasts as long as the previous call's
// kernels), so back-to-back scans would be serialised on the host.  Outside
// stream capture, workspaces of up to kMaxCachedWorkspace bytes therefore come
// from a small per-device cache, without a host wait: buffers of power-of-two
// sizes from 1 MiB, each with an event recorded after the last kernel that
// uses it and that kernel's stream.
// A call takes, among the buffers large enough, one whose event has completed;
// else one last used on the same stream; else a new one while the device holds
// fewer than kMaxCachedBuffers; else any.  A buffer whose event is pending is
// ordered after that event on the device (hipStreamWaitEvent), never on the
// host.  Larger workspaces, whose scans take far longer than that host wait,
// and every call under capture (where the graph must own its memory as graph
// memory nodes) use the stream-ordered allocator.
// ---------------------------------------------------------------------------
struct Workspace {
  void* ptr = nullptr;
  size_t bytes = 0;
  hipEvent_t done = nullptr;   // recorded after the last kernel that used the buffer
  hipStream_t last = nullptr;  // the stream that kernel was launched on
  bool used = false;           // `done` has been recorded
};

struct DeviceWorkspaces {
  std::vector<Workspace> idle;  // buffers not held by a call
  int count = 0;                // idle + held
};

constexpr int kMaxWsDevices = 64;
constexpr size_t kMaxCachedWorkspace = (size_t)256 << 20;  // bytes of one cached buffer
constexpr int kMaxCachedBuffers = 4;                        // buffers per device, held ones included
std::mutex g_ws_mu;
DeviceWorkspaces g_ws[kMaxWsDevices];

// A workspace of at least `bytes` on device `dev` (the current device), usable
// by kernels launched on `s` once this returns.
hipError_t ws_acquire(int dev, size_t bytes, hipStream_t s, Workspace* out) {
  Workspace drop;  // a too-small idle buffer freed to keep the count bounded
  bool reuse = false;
  {
    std::lock_guard<std::mutex> lk(g_ws_mu);
    DeviceWorkspaces& D = g_ws[dev];
    std::vector<Workspace>& L = D.idle;
    auto pick = [&](auto&& ok) {
      int best = -1;
      for (int i = 0; i < (int)L.size(); ++i)
        if (L[i].bytes >= bytes && (best < 0 || L[i].bytes < L[best].bytes) && ok(L[i])) best = i;
      return best;
    };
    int i = pick([](const Workspace& w) { return !w.used || hipEventQuery(w.done) == hipSuccess; });
    if (i < 0) i = pick([&](const Workspace& w) { return w.last == s; });
    if (i < 0 && D.count >= kMaxCachedBuffers) i = pick([](const Workspace&) { return true; });
    if (i >= 0) {
      *out = L[i];
      L.erase(L.begin() + i);
      reuse = true;
    } else {
      if (D.count >= kMaxCachedBuffers && !L.empty()) {  // none fits: retire the smallest
        int j = 0;
        for (int k = 1; k < (int)L.size(); ++k)
          if (L[k].bytes < L[j].bytes) j = k;
        drop = L[j];
        L.erase(L.begin() + j);
        --D.count;
      }
      ++D.count;
    }
  }
  if (reuse) {
    if (out->used && hipEventQuery(out->done) != hipSuccess) return hipStreamWaitEvent(s, out->done, 0);
    return hipSuccess;
  }
  if (drop.ptr != nullptr) {  // the retired buffer's last kernel must finish first
    zmc::log(2, "workspace: retiring a %zu-byte buffer on device %d", drop.bytes, dev);
    if (drop.used) (void)hipEventSynchronize(drop.done);
    (void)hipEventDestroy(drop.done);
    (void)hipFree(drop.ptr);
  }
  // power-of-two sizes from 1 MiB: a buffer then also serves the smaller
  // workspaces of later calls, so a mix of sizes settles on a few buffers
  // instead of retiring (and freeing, which waits for the device) one per call
  size_t size = (size_t)1 << 20;
  while (size < bytes) size <<= 1;
  if (size > kMaxCachedWorkspace) size = bytes;
  zmc::log(2, "workspace: new %zu-byte buffer on device %d", size, dev);
  Workspace w;
  w.bytes = size;
  hipError_t e = hipMalloc(&w.ptr, size);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&w.done, hipEventDisableTiming);
  if (e != hipSuccess) {
    if (w.ptr) (void)hipFree(w.ptr);
    std::lock_guard<std::mutex> lk(g_ws_mu);
    --g_ws[dev].count;
    return e;
  }
  *out = w;
  return hipSuccess;
}

// Hands a workspace back once the last kernel that uses it is enqueued on `s`.
hipError_t ws_release(int dev, Workspace w, hipStream_t s) {
  hipError_t e = hipEventRecord(w.done, s);
  if (e != hipSuccess) {  // no event to order on: let the buffer's work finish first
    const hipError_t e2 = hipStreamSynchronize(s);
    (void)e2;
  }
  w.last = s;
  w.used = e == hipSuccess;
  std::lock_guard<std::mutex> lk(g_ws_mu);
  g_ws[dev].idle.push_back(w);
  return e;
}

void to_info(const zmc::Plan& pl, uint64_t G, zmc_plan_info* out) {
  memset(out, 0, sizeof(*out));
  out->mode = pl.mode;
  out->block = pl.block;
  out->splits = pl.splits;
  out->grid_points = G;
  out->groups = pl.groups;
  out->groups_per_split = pl.gps;
  out->blocks = pl.grid_x * (uint64_t)pl.splits;
  out->workspace_bytes = pl.workspace_bytes;
}

}  // namespace

extern "C" {

const char* zmc_last_error(void) { return g_err; }

const char* zmc_version(void) { return "zmc 0.9 gfx950"; }

zmc_status zmc_validate(const zmc_scan_desc* desc, uint64_t* grid_points) {
  return validate(desc, grid_points);
}

zmc_status zmc_plan(const zmc_scan_desc* desc, const zmc_launch_opts* opts, zmc_plan_info* out) {
  uint64_t G = 0;
  zmc_status st = validate(desc, &G);
  if (st != ZMC_OK) return st;
  if (out == nullptr) return fail(ZMC_E_INVALID, "out is NULL");
  zmc::Plan pl;
  st = make_plan(desc, G, opts, &pl);
  if (st != ZMC_OK) return st;
  to_info(pl, G, out);
  return ok();
}

zmc_status zmc_scan_device_ex(const zmc_scan_desc* desc, const double* d_axis_vals, double* d_f,
                              double* d_sigma, const zmc_launch_opts* opts, void* stream) {
  zmc::TraceRange trace_range("zmc_scan_device");
  uint64_t G = 0;
  zmc_status st = validate(desc, &G);
  if (st != ZMC_OK) return st;
  const bool stage = desc->M > 0 && d_axis_vals == nullptr;  // lists from desc->axis_vals
  if (stage && desc->axis_vals == nullptr)
    return fail(ZMC_E_INVALID, "d_axis_vals and desc->axis_vals are both NULL with M > 0");
  if (d_f == nullptr || d_sigma == nullptr) return fail(ZMC_E_INVALID, "d_f or d_sigma is NULL");
  hipStream_t s = (hipStream_t)stream;
  hipStreamCaptureStatus capture = hipStreamCaptureStatusNone;
  ZMC_HIP(hipStreamIsCapturing(s, &capture));
  if (stage && capture != hipStreamCaptureStatusNone)
    return fail(ZMC_E_INVALID, "under stream capture the lists must already be on the device "
                               "(d_axis_vals): a replay cannot re-read the caller's host memory");
  zmc::Plan pl;
  st = make_plan(desc, G, opts, &pl);
  if (st != ZMC_OK) return st;
  zmc::UserKernels uk;
  if (desc->family == ZMC_USER) {
    st = zmc::user_kernels(desc->integrand, desc->precision, desc->N, desc->M, &uk);
    if (st != ZMC_OK) return st;
  }
  int dev = 0, stream_dev = 0;
  ZMC_HIP(hipGetDevice(&dev));
  ZMC_HIP(hipStreamGetDevice(s, &stream_dev));
  const bool use_cache = pl.workspace_bytes > 0 && capture == hipStreamCaptureStatusNone &&
                         pl.workspace_bytes <= kMaxCachedWorkspace && dev == stream_dev &&
                         dev >= 0 && dev < kMaxWsDevices;

  // device memory of this call; every path below releases what it took
  double* staged = nullptr;  // the lists, when the caller passed none (freed on the stream)
  void* ws = nullptr;        // stream-ordered split partials
  Workspace cached;          // or split partials from the per-device cache
  hipError_t e = hipSuccess;
  if (stage) {
    uint64_t total = 0;
    for (int l = 0; l < desc->M; ++l) total += (uint64_t)desc->axis_len[l];
    e = hipMallocAsync((void**)&staged, 8 * total, s);
    // from pageable memory the copy has read the caller's lists when it returns
    if (e == hipSuccess)
      e = hipMemcpyAsync(staged, desc->axis_vals, 8 * total, hipMemcpyHostToDevice, s);
    d_axis_vals = staged;
  }
  zmc::ScanParams p;
  fill_params(desc, G, pl, d_axis_vals, d_f, d_sigma, &p);
  if (e == hipSuccess && pl.workspace_bytes > 0) {
    if (use_cache) {
      e = ws_acquire(dev, pl.workspace_bytes, s, &cached);
      p.part_mean = (double*)cached.ptr;
    } else {
      e = hipMallocAsync(&ws, pl.workspace_bytes, s);
      p.part_mean = (double*)ws;
    }
    p.part_m2 = p.part_mean + (uint64_t)pl.splits * G;
  }
  const char* what = "allocating or staging device memory";
  if (e == hipSuccess) {
    what = "scan launch";
    hipEvent_t ev_b = opts ? (hipEvent_t)opts->ev_begin : nullptr;
    hipEvent_t ev_e = opts ? (hipEvent_t)opts->ev_end : nullptr;
    e = desc->family == ZMC_USER ? zmc::launch_user_scan(uk, p, pl, s, ev_b, ev_e)
                                 : zmc::launch_scan(p, pl, desc->precision, s, ev_b, ev_e);
  }
  if (ws != nullptr) {
    hipError_t e2 = hipFreeAsync(ws, s);
    if (e == hipSuccess) e = e2;
  }
  if (cached.ptr != nullptr) {
    hipError_t e2 = ws_release(dev, cached, s);
    if (e == hipSuccess) e = e2;
  }
  if (staged != nullptr) {
    hipError_t e2 = hipFreeAsync(staged, s);
    if (e == hipSuccess) e = e2;
  }
  if (e != hipSuccess)
    return fail(e == hipErrorOutOfMemory ? ZMC_E_NOMEM : ZMC_E_DEVICE, "%s failed: %s", what,
                hipGetErrorString(e));
  return ok();
}

zmc_status zmc_scan_device(const zmc_scan_desc* desc, const double* d_axis_vals, double* d_f,
                           double* d_sigma, void* stream) {
  return zmc_scan_device_ex(desc, d_axis_vals, d_f, d_sigma, nullptr, stream);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Scratch of zmc_scan_device_noalloc: the split partials of its plans live in
// this fixed device array instead of stream-ordered allocations.  Each device
// holds its own copy (reserved when the library's code is loaded there, kept
// until the process ends), at its own address: host code uses the address
// that hipGetSymbolAddress returns on that device, never the array's name,
// which on the host is only a stand-in.
// ---------------------------------------------------------------------------
static __device__ __align__(256) double scratch[ZMC_NOALLOC_SCRATCH_BYTES / sizeof(double)];

namespace {

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};

// The current device's copy of `scratch`, looked up once per device.
zmc_status scratch_on_current_device(void** out) {
  int dev = 0;
  ZMC_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxScratchDevices)
    return fail(ZMC_E_UNSUPPORTED, "device %d: the allocation-free scan serves devices 0..%d", dev,
                kMaxScratchDevices - 1);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr)
      return fail(ZMC_E_DEVICE, "scratch of the allocation-free scan on device %d: %s", dev,
                  hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return ZMC_OK;
}

}  // namespace

extern "C" {

zmc_status zmc_scan_device_noalloc(const zmc_scan_desc* desc, const double* d_axis_vals,
                                   double* d_f, double* d_sigma, void* stream) {
  zmc::TraceRange trace_range("zmc_scan_device_noalloc");
  uint64_t G = 0;
  zmc_status st = validate(desc, &G);
  if (st != ZMC_OK) return st;
  if (desc->family == ZMC_USER)
    return fail(ZMC_E_UNSUPPORTED, "the allocation-free scan runs the compiled-in families only "
                                   "(a user integrand's kernels are built and loaded on first use)");
  if (desc->M > 0 && d_axis_vals == nullptr) return fail(ZMC_E_INVALID, "d_axis_vals is NULL with M > 0");
  if (d_f == nullptr || d_sigma == nullptr) return fail(ZMC_E_INVALID, "d_f or d_sigma is NULL");
  // set-up on the first call on a device: the address of its scratch
  void* base = nullptr;
  st = scratch_on_current_device(&base);
  if (st != ZMC_OK) return st;
  zmc::Plan pl;
  st = make_plan(desc, G, nullptr, &pl);
  if (st != ZMC_OK) return st;
  if (pl.workspace_bytes > ZMC_NOALLOC_SCRATCH_BYTES)
    return fail(ZMC_E_NOMEM,
                "split partials of %llu points x %d pieces need %llu bytes, more than the %llu "
                "bytes of the allocation-free scan's scratch (zmc_scan_device allocates them)",
                (unsigned long long)G, pl.splits, (unsigned long long)pl.workspace_bytes,
                (unsigned long long)ZMC_NOALLOC_SCRATCH_BYTES);
  zmc::ScanParams p;
  fill_params(desc, G, pl, d_axis_vals, d_f, d_sigma, &p);
  if (pl.workspace_bytes > 0) {
    // every (piece, point) slot is written by the main kernel before the
    // merge pass reads it, so nothing needs clearing
    p.part_mean = (double*)base;
    p.part_m2 = p.part_mean + (uint64_t)pl.splits * G;
  }
  const hipError_t e = zmc::launch_scan(p, pl, desc->precision, (hipStream_t)stream, nullptr, nullptr);
  if (e != hipSuccess) return fail(ZMC_E_DEVICE, "scan launch failed: %s", hipGetErrorString(e));
  return ok();
}

zmc_status zmc_scan(const zmc_scan_desc* desc, double* f, double* sigma) {
  zmc::TraceRange trace_range("zmc_scan");
  uint64_t G = 0;
  zmc_status st = validate(desc, &G);
  if (st != ZMC_OK) return st;
  if (desc->M > 0 && desc->axis_vals == nullptr) return fail(ZMC_E_INVALID, "axis_vals is NULL with M > 0");
  if (f == nullptr || sigma == nullptr) return fail(ZMC_E_INVALID, "f or sigma is NULL");
  if (G > kMaxBytes / 16)
    return fail(ZMC_E_NOMEM, "f and sigma of %llu points exceed %llu bytes of device staging",
                (unsigned long long)G, (unsigned long long)kMaxBytes);
  uint64_t total = 0;
  for (int l = 0; l < desc->M; ++l) total += (uint64_t)desc->axis_len[l];
  double *d_axis = nullptr, *d_out = nullptr;
  hipError_t e = hipSuccess;
  if (total > 0) e = hipMalloc(&d_axis, total * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&d_out, 2 * G * sizeof(double));
  if (e == hipSuccess && total > 0)
    e = hipMemcpy(d_axis, desc->axis_vals, total * sizeof(double), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(d_axis);
    (void)hipFree(d_out);
    return fail(e == hipErrorOutOfMemory ? ZMC_E_NOMEM : ZMC_E_DEVICE, "staging failed: %s",
                hipGetErrorString(e));
  }
  st = zmc_scan_device(desc, d_axis, d_out, d_out + G, nullptr);
  if (st == ZMC_OK) {
    e = hipMemcpy(f, d_out, G * sizeof(double), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(sigma, d_out + G, G * sizeof(double), hipMemcpyDeviceToHost);
    if (e != hipSuccess) st = fail(ZMC_E_DEVICE, "copy back failed: %s", hipGetErrorString(e));
  }
  (void)hipFree(d_axis);
  (void)hipFree(d_out);
  return st == ZMC_OK ? ok() : st;
}

zmc_status zmc_debug_words(uint64_t seed, uint64_t g, uint64_t w0, int64_t count, uint32_t* d_out,
                           void* stream) {
  if (count < 0 || (count > 0 && d_out == nullptr)) return fail(ZMC_E_INVALID, "bad output");
  if (count > ((int64_t)1 << 38)) return fail(ZMC_E_INVALID, "count too large");
  hipError_t e = zmc::launch_debug_words(seed, g, w0, count, d_out, (hipStream_t)stream);
  if (e != hipSuccess) return fail(ZMC_E_DEVICE, "launch failed: %s", hipGetErrorString(e));
  return ok();
}

zmc_status zmc_debug_valu_probe(int32_t blocks, int64_t iters, float* d_out, void* stream) {
  if (blocks < 1 || blocks > (1 << 20)) return fail(ZMC_E_INVALID, "blocks = %d outside 1..2^20", blocks);
  if (iters < 1) return fail(ZMC_E_INVALID, "iters = %lld < 1", (long long)iters);
  if (d_out == nullptr) return fail(ZMC_E_INVALID, "d_out is NULL");
  hipError_t e = zmc::launch_valu_probe(blocks, iters, d_out, (hipStream_t)stream);
  if (e != hipSuccess) return fail(ZMC_E_DEVICE, "launch failed: %s", hipGetErrorString(e));
  return ok();
}

zmc_status zmc_debug_rate_probe(int32_t op, int32_t blocks, int64_t iters, uint64_t* d_out,
                                void* stream) {
  if (op < ZMC_RATE_XOR_B32 || op > ZMC_RATE_FMA_F64) return fail(ZMC_E_INVALID, "unknown op %d", op);
  if (blocks < 1 || blocks > (1 << 20)) return fail(ZMC_E_INVALID, "blocks = %d outside 1..2^20", blocks);
  if (iters < 1) return fail(ZMC_E_INVALID, "iters = %lld < 1", (long long)iters);
  if (d_out == nullptr) return fail(ZMC_E_INVALID, "d_out is NULL");
  hipError_t e = zmc::launch_rate_probe(op, blocks, iters, d_out, (hipStream_t)stream);
  if (e != hipSuccess) return fail(ZMC_E_DEVICE, "launch failed: %s", hipGetErrorString(e));
  return ok();
}

zmc_status zmc_debug_values(const zmc_scan_desc* desc, const double* d_axis_vals, uint64_t g,
                            uint64_t s0, int64_t count, double* d_out, void* stream) {
  uint64_t G = 0;
  zmc_status st = validate(desc, &G);
  if (st != ZMC_OK) return st;
  if (g >= G) return fail(ZMC_E_INVALID, "g = %llu >= G", (unsigned long long)g);
  if (desc->M > 0 && d_axis_vals == nullptr) return fail(ZMC_E_INVALID, "d_axis_vals is NULL with M > 0");
  if (count < 0 || (count > 0 && d_out == nullptr)) return fail(ZMC_E_INVALID, "bad output");
  if (count > ((int64_t)1 << 38)) return fail(ZMC_E_INVALID, "count too large");
  zmc_launch_opts o{ZMC_MODE_POINT_MAJOR, 256, 1, 1, nullptr, nullptr};
  zmc::Plan pl;
  st = make_plan(desc, G, &o, &pl);
  if (st != ZMC_OK) return st;
  zmc::UserKernels uk;
  if (desc->family == ZMC_USER) {
    st = zmc::user_kernels(desc->integrand, desc->precision, desc->N, desc->M, &uk);
    if (st != ZMC_OK) return st;
  }
  zmc::ScanParams p;
  fill_params(desc, G, pl, d_axis_vals, nullptr, nullptr, &p);
  hipError_t e = desc->family == ZMC_USER
                     ? zmc::launch_user_values(uk, p, g, s0, count, d_out, (hipStream_t)stream)
                     : zmc::launch_debug_values(p, desc->precision, g, s0, count, d_out, (hipStream_t)stream);
  if (e != hipSuccess) return fail(ZMC_E_DEVICE, "launch failed: %s", hipGetErrorString(e));
  return ok();
}


}  // extern "C"

namespace {

// Host threads that store a chunk's results from pinned staging into pageable
// outputs: $ZMC_COPY_THREADS if set (1..64), else 8.
uint64_t copy_threads() {
  static const uint64_t n = [] {
    const char* env = getenv("ZMC_COPY_THREADS");
    const int v = (env && *env) ? atoi(env) : 0;
    return (uint64_t)(v >= 1 && v <= 64 ? v : 8);
  }();
  return n;
}

}  // namespace

extern "C" {

zmc_status zmc_scan_chunked(const zmc_scan_desc* desc, double* f, double* sigma,
                            uint64_t chunk_points) {
  uint64_t G = 0;
  zmc_status st = validate(desc, &G);
  if (st != ZMC_OK) return st;
  return zmc_scan_range(desc, 0, G, f, sigma, chunk_points);
}

zmc_status zmc_scan_range(const zmc_scan_desc* desc, uint64_t g_begin, uint64_t g_end, double* f,
                          double* sigma, uint64_t chunk_points) {
  zmc::TraceRange trace_range("zmc_scan_range");
  uint64_t G = 0;
  zmc_status st = validate(desc, &G);
  if (st != ZMC_OK) return st;
  if (desc->M > 0 && desc->axis_vals == nullptr) return fail(ZMC_E_INVALID, "axis_vals is NULL with M > 0");
  if (f == nullptr || sigma == nullptr) return fail(ZMC_E_INVALID, "f or sigma is NULL");
  if (g_begin >= g_end || g_end > G)
    return fail(ZMC_E_INVALID, "range [%llu, %llu) is empty or outside the grid of %llu points",
                (unsigned long long)g_begin, (unsigned long long)g_end, (unsigned long long)G);
  const uint64_t R = g_end - g_begin;  // points of the range; f[i] is point g_begin + i
  const uint64_t C = std::min<uint64_t>(R, chunk_points > 0 ? chunk_points : kDefaultChunk);
  if (C > kMaxBytes / 32)
    return fail(ZMC_E_NOMEM, "chunks of %llu points exceed %llu bytes of staging",
                (unsigned long long)C, (unsigned long long)kMaxBytes);
  zmc::UserKernels uk;
  if (desc->family == ZMC_USER) {
    st = zmc::user_kernels(desc->integrand, desc->precision, desc->N, desc->M, &uk);
    if (st != ZMC_OK) return st;
  }
  // every chunk runs the decomposition of the whole grid, so its points get
  // the same sample pieces (and results) as in a scan of the whole grid
  zmc::Plan full;
  st = make_plan(desc, G, nullptr, &full);
  if (st != ZMC_OK) return st;
  const zmc_launch_opts fixed{full.mode, full.block, full.splits, 0, nullptr, nullptr};
  zmc::Plan cp;
  st = make_plan(desc, C, &fixed, &cp);
  if (st != ZMC_OK) return st;
  if ((uint64_t)cp.splits != (uint64_t)full.splits || cp.gps != full.gps)
    return fail(ZMC_E_INVALID, "chunk plan differs from the grid's plan");

  uint64_t n_axis = 0;
  for (int l = 0; l < desc->M; ++l) n_axis += (uint64_t)desc->axis_len[l];
  const size_t off_out = align256(8 * n_axis);
  const size_t slot_bytes = align256(16 * C);   // f then sigma of one chunk
  const size_t off_ws = off_out + 2 * slot_bytes;
  const size_t total = off_ws + cp.workspace_bytes;
  // outputs already in pinned host memory take the copies directly
  bool pinned = true, on_device = false;
  for (double* ptr : {f, sigma}) {
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, ptr) != hipSuccess) {
      pinned = false;  // pageable host memory is unknown to HIP
      continue;
    }
    if (a.type == hipMemoryTypeDevice) on_device = true;
    if (a.type != hipMemoryTypeHost) pinned = false;
  }
  (void)hipGetLastError();  // pageable memory can leave an error behind
  if (on_device) return fail(ZMC_E_INVALID, "f and sigma must be host memory (device outputs: zmc_scan_device)");

  char* dmem = nullptr;
  double* stage = nullptr;
  hipStream_t streams[2] = {nullptr, nullptr};
  hipEvent_t computed[2] = {nullptr, nullptr}, copied[2] = {nullptr, nullptr};
  hipError_t e = hipMalloc((void**)&dmem, total);
  if (e == hipSuccess && !pinned) e = hipHostMalloc((void**)&stage, 2 * 16 * C, 0);
  for (int i = 0; e == hipSuccess && i < 2; ++i) e = hipStreamCreateWithFlags(&streams[i], hipStreamNonBlocking);
  for (int i = 0; e == hipSuccess && i < 2; ++i) {
    e = hipEventCreateWithFlags(&computed[i], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&copied[i], hipEventDisableTiming);
  }
  if (e == hipSuccess && n_axis > 0) e = hipMemcpy(dmem, desc->axis_vals, 8 * n_axis, hipMemcpyHostToDevice);
  const double* d_axis = (const double*)dmem;
  auto host_copy = [&](int slot, uint64_t g0, uint64_t n) {
    // pinned staging -> the caller's arrays, on a few host threads
    const double* src = stage + (size_t)slot * 2 * C;
    const uint64_t parts = n >= ((uint64_t)1 << 20) ? copy_threads() : 1;
    std::vector<std::thread> th;
    for (uint64_t t = 0; t < parts; ++t) {
      const uint64_t a = n * t / parts, b = n * (t + 1) / parts;
      th.emplace_back([=] {
        memcpy(f + g0 + a, src + a, 8 * (b - a));
        memcpy(sigma + g0 + a, src + C + a, 8 * (b - a));
      });
    }
    for (auto& x : th) x.join();
  };
  const uint64_t chunks = (R + C - 1) / C;
  uint64_t prev_g0 = 0, prev_n = 0;
  for (uint64_t i = 0; e == hipSuccess && i < chunks; ++i) {
    zmc::TraceRange chunk_range("zmc_scan_range chunk");
    const int slot = (int)(i & 1);
    const uint64_t g0 = i * C, n = std::min<uint64_t>(C, R - g0);  // g0: offset in the range
    double* d_f = (double*)(dmem + off_out + (size_t)slot * slot_bytes);
    double* d_s = d_f + C;
    zmc::Plan pl;
    st = make_plan(desc, n, &fixed, &pl);
    if (st != ZMC_OK) break;
    zmc::ScanParams p;
    fill_params(desc, n, pl, d_axis, d_f, d_s, &p, g_begin + g0);
    if (pl.workspace_bytes > 0) {
      p.part_mean = (double*)(dmem + off_ws);
      p.part_m2 = p.part_mean + (uint64_t)pl.splits * n;
    }
    // the device slot is free once chunk i-2 has been copied out of it
    if (i >= 2) e = hipStreamWaitEvent(streams[0], copied[slot], 0);
    if (e == hipSuccess)
      e = desc->family == ZMC_USER ? zmc::launch_user_scan(uk, p, pl, streams[0], nullptr, nullptr)
                                   : zmc::launch_scan(p, pl, desc->precision, streams[0], nullptr, nullptr);
    if (e == hipSuccess) e = hipEventRecord(computed[slot], streams[0]);
    if (e == hipSuccess) e = hipStreamWaitEvent(streams[1], computed[slot], 0);
    double* h_f = pinned ? f + g0 : stage + (size_t)slot * 2 * C;
    double* h_s = pinned ? sigma + g0 : stage + (size_t)slot * 2 * C + C;
    if (e == hipSuccess) e = hipMemcpyAsync(h_f, d_f, 8 * n, hipMemcpyDeviceToHost, streams[1]);
    if (e == hipSuccess) e = hipMemcpyAsync(h_s, d_s, 8 * n, hipMemcpyDeviceToHost, streams[1]);
    if (e == hipSuccess) e = hipEventRecord(copied[slot], streams[1]);
    // while the device works on chunk i, the host stores chunk i-1
    if (e == hipSuccess && i >= 1 && !pinned) {
      e = hipEventSynchronize(copied[slot ^ 1]);
      if (e == hipSuccess) host_copy(slot ^ 1, prev_g0, prev_n);
    }
    prev_g0 = g0;
    prev_n = n;
  }
  if (e == hipSuccess && st == ZMC_OK && chunks > 0) {
    e = hipEventSynchronize(copied[(chunks - 1) & 1]);
    if (e == hipSuccess && !pinned) host_copy((int)((chunks - 1) & 1), prev_g0, prev_n);
  }
  for (int i = 0; i < 2; ++i)
    if (streams[i]) (void)hipStreamSynchronize(streams[i]);
  for (int i = 0; i < 2; ++i) {
    if (computed[i]) (void)hipEventDestroy(computed[i]);
    if (copied[i]) (void)hipEventDestroy(copied[i]);
    if (streams[i]) (void)hipStreamDestroy(streams[i]);
  }
  if (stage) (void)hipHostFree(stage);
  if (dmem) (void)hipFree(dmem);
  if (st != ZMC_OK) return st;
  if (e != hipSuccess)
    return fail(e == hipErrorOutOfMemory ? ZMC_E_NOMEM : ZMC_E_DEVICE, "chunked scan failed: %s",
                hipGetErrorString(e));
  return ok();
}

}  // extern "C"
