// zmc_server.hip -- serving with continuous batching (include/zmc.h).
//
// A scheduler thread owns two HIP streams and alternates short slices
// between them so that the next slice's blocks start while the previous
// slice's last tiles finish.  Every slice takes tiles round-robin from all
// admitted requests (each request cut into the same tiles a batch would use)
// and runs them in one persistent kernel per precision (user integrands and
// scans of more than eight dimensions in kernels of their own, one per
// variant); requests whose last
// tile is in the slice get their split merge in the same slice and complete
// when its event does.  Admission takes the queue in arrival order, or
// shortest estimated work first (optionally with a bound on how long a
// request may be passed over), limited by the HBM budget for the requests'
// own device state (staged lists and split partials) and by the number of
// slots in the device table of scan descriptors.
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "zmc.h"
#include "zmc_device.hpp"
#include "zmc_internal.hpp"
#include "zmc_trace.hpp"

using zmc::fail;
using zmc::ok;

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
  uint64_t ticket = 0;
  zmc_scan_desc desc{};
  std::vector<int64_t> axis_len;
  std::vector<double> axis_vals, lo, hi, params;
  const double* d_axis_user = nullptr;
  double* d_f = nullptr;
  double* d_sigma = nullptr;
  uint64_t G = 0;
  zmc::Plan plan{};
  uint64_t total_tiles = 0, next_tile = 0;
  uint64_t tile_samples = 1;  // samples per tile, averaged over the request's tiles
  uint64_t staged_doubles = 0;
  uint64_t footprint = 0;
  double work = 0.0;          // estimated device work G * samples * N (admission order)
  zmc::UserKernels user;      // family ZMC_USER: kernels built for this shape
  unsigned own_blocks = 0;    // resident blocks of the request's own batch kernel
                              // (user integrands; compiled-in N > kAnyMaxDims)
  void* dmem = nullptr;
  int alloc_stream = 0;
  int slot = -1;
  Clock::time_point t_submit;
  double latency = 0.0;
  zmc_status status = ZMC_OK;
  bool done = false;
  // under zmc_server::mu: admission is decided (the scheduler sets `admitted`
  // before any device work of the request), or the request was cancelled
  bool admitted = false;
  bool cancelled = false;
};

using ReqPtr = std::shared_ptr<Request>;

struct Slice {
  hipEvent_t done_ev = nullptr;
  std::vector<ReqPtr> finishing;
  uint64_t samples = 0;        // samples of the slice's tiles
  Clock::time_point t_launch;  // when it was enqueued
};

// slice_us: slices of slice_samples samples until the device's throughput has
// been measured, then that throughput times slice_us, kept within these bounds
constexpr uint64_t kMinSliceSamples = (uint64_t)1 << 24;
constexpr uint64_t kMaxSliceSamples = (uint64_t)1 << 44;

constexpr int kStreams = 2;
// The latency percentiles cover the most recent completions only, so that a
// long-running server's memory and get_stats cost stay bounded.
constexpr size_t kLatencyWindow = 65536;

}  // namespace

struct zmc_server {
  zmc_server_opts opts{};
  int device = 0;
  hipStream_t streams[kStreams] = {nullptr, nullptr};
  unsigned blocks32 = 1, blocks64 = 1;
  int cu = 1;
  int counters_per_slot = 2;  // FP32 and FP64 any-family kernels, then one per own-kernel variant (at most one per admitted request)
  int ring = 3;
  // device memory: slot table | tile ring | counter ring | merge ring
  void* dmem = nullptr;
  zmc::ScanParams* d_slots = nullptr;
  zmc::Tile* d_tiles = nullptr;
  uint32_t* d_counters = nullptr;
  uint32_t* d_merge = nullptr;
  // pinned host mirrors
  zmc::ScanParams* h_slots = nullptr;
  zmc::Tile* h_tiles = nullptr;
  uint32_t* h_merge = nullptr;
  std::vector<hipEvent_t> done_events, admit_events;
  // shared with submitters
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<ReqPtr> incoming;
  std::unordered_map<uint64_t, ReqPtr> tickets;
  uint64_t next_ticket = 1;
  bool stop = false;
  zmc_server_stats stats{};
  std::vector<double> latencies;   // latest kLatencyWindow completions (a ring)
  uint64_t latency_count = 0;      // completions recorded in the ring so far
  Clock::time_point t_first_submit, t_last_done;
  bool any_submitted = false;
  // scheduler-thread state
  std::deque<ReqPtr> pending, active;
  std::deque<Slice> inflight;
  std::vector<int> free_slots;
  uint64_t bytes_in_use = 0;
  uint64_t slice_count = 0;
  uint64_t slice_budget = 0;        // samples of the next slice
  double rate = 0.0;                // slice_us only: measured samples/s of the device
  Clock::time_point t_last_retire;  // when the previous slice was seen done
  uint64_t acc_samples = 0, acc_slices = 0;  // retirements of the current window
  double acc_seconds = 0.0;
  std::thread thread;
};

namespace {

size_t align_up(size_t x) { return (x + 255) / 256 * 256; }

zmc::Tile tile_of(const Request& r, uint64_t t) {
  const bool pm = r.plan.mode == ZMC_MODE_POINT_MAJOR;
  const uint64_t per = pm ? r.plan.point_blocks : r.G;
  const uint64_t split = t / per, i = t % per;
  zmc::Tile tl;
  tl.scan = (uint32_t)r.slot;
  tl.split_mode = (uint32_t)split | (pm ? 0u : zmc::kTileSampleMajor);
  tl.first = pm ? i * zmc::kTileBlock : i;
  return tl;
}

void finish(zmc_server* s, const ReqPtr& r, zmc_status st) {
  r->latency = std::chrono::duration<double>(Clock::now() - r->t_submit).count();
  zmc::log(2, "server: request %llu done, status %d, %.6f s after submit",
           (unsigned long long)r->ticket, (int)st, r->latency);
  if (st == ZMC_OK) {
    // every copy and kernel of the request has completed, so the host copies
    // of its descriptor are not read again: a finished request keeps only its
    // status and latency until zmc_server_release (after a failure they stay
    // until then, since a copy from them may not have run)
    std::vector<int64_t>().swap(r->axis_len);
    std::vector<double>().swap(r->axis_vals);
    std::vector<double>().swap(r->lo);
    std::vector<double>().swap(r->hi);
    std::vector<double>().swap(r->params);
    r->desc.axis_len = nullptr;
    r->desc.axis_vals = r->desc.lo = r->desc.hi = r->desc.params = nullptr;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  r->status = st;
  r->done = true;
  if (st == ZMC_OK) {
    s->stats.completed++;
    s->stats.samples_completed += r->G * r->desc.samples;
    if (s->latencies.size() < kLatencyWindow)
      s->latencies.push_back(r->latency);
    else
      s->latencies[s->latency_count % kLatencyWindow] = r->latency;
    s->latency_count++;
    s->t_last_done = Clock::now();
  } else {
    s->stats.failed++;
    if (st == ZMC_E_CANCELLED) s->stats.cancelled++;
  }
  s->cv_done.notify_all();
}

// Admission: device state, staged lists, the slot's scan descriptor.
hipError_t admit(zmc_server* s, const ReqPtr& r, int si) {
  zmc::TraceRange trace_range("zmc_server admit");
  hipStream_t st = s->streams[si];
  hipError_t e = hipSuccess;
  if (r->footprint > 0) e = hipMallocAsync(&r->dmem, r->footprint, st);
  if (e != hipSuccess) return e;
  r->alloc_stream = si;
  char* base = (char*)r->dmem;
  const double* axis = r->d_axis_user;
  if (axis == nullptr && r->staged_doubles > 0) {
    e = hipMemcpyAsync(base, r->axis_vals.data(), 8 * r->staged_doubles, hipMemcpyHostToDevice, st);
    axis = (const double*)base;
  }
  r->slot = s->free_slots.back();
  s->free_slots.pop_back();
  zmc::ScanParams& p = s->h_slots[r->slot];
  zmc::fill_scan_params(&r->desc, r->G, r->plan, axis, r->d_f, r->d_sigma, &p);
  if (r->plan.splits > 1) {
    double* pm = (double*)(base + align_up(8 * r->staged_doubles));
    p.part_mean = pm;
    p.part_m2 = pm + (uint64_t)r->plan.splits * r->G;
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(s->d_slots + r->slot, &p, sizeof(p), hipMemcpyHostToDevice, st);
  return e;
}

// Requests whose tiles run in a batch kernel of their own rather than in the
// any-family kernel of their precision, and whether two of them share it.
bool own_kernel(const Request& r) {
  return r.desc.family == ZMC_USER || r.desc.N > zmc::kAnyMaxDims;
}

bool same_variant(const Request& a, const Request& b) {
  if (a.desc.family != b.desc.family || a.desc.precision != b.desc.precision || a.desc.N != b.desc.N)
    return false;
  return a.desc.family != ZMC_USER || (a.desc.integrand == b.desc.integrand && a.desc.M == b.desc.M);
}

// One slice on stream `si`: work round-robin over the admitted requests (an
// equal share of the slice's samples each, then what is left in admission
// order), FP32 tiles then FP64 tiles, one persistent kernel for each; then
// the split merges of the requests whose last tile is in the slice.  Slices
// are sized in samples, not tiles, because a request's tiles range from one
// point's sample piece to 256 points' pieces.
hipError_t launch_slice(zmc_server* s, int si, Slice* out) {
  zmc::TraceRange trace_range("zmc_server slice");
  const uint64_t cap = (uint64_t)s->opts.slice_tiles;
  const uint64_t budget = s->slice_budget;
  const int ring_slot = (int)(s->slice_count % (uint64_t)s->ring);
  zmc::Tile* ht = s->h_tiles + (size_t)ring_slot * cap;
  std::vector<std::pair<ReqPtr, uint64_t>> take;
  size_t with_work = 0;
  for (const ReqPtr& r : s->active)
    if (r->next_tile < r->total_tiles) ++with_work;
  if (with_work == 0) return hipSuccess;
  const uint64_t share = std::max<uint64_t>(1, budget / with_work);
  uint64_t used = 0, used_samples = 0;
  for (const ReqPtr& r : s->active) {
    const uint64_t left = r->total_tiles - r->next_tile;
    const uint64_t want = (share + r->tile_samples - 1) / r->tile_samples;
    const uint64_t k = std::min<uint64_t>({left, want, cap - used});
    if (k > 0) take.emplace_back(r, k), used += k, used_samples += k * r->tile_samples;
  }
  for (auto& tk : take) {
    if (used_samples >= budget || used >= cap) break;
    const Request& r = *tk.first;
    const uint64_t left = r.total_tiles - r.next_tile - tk.second;
    const uint64_t want = (budget - used_samples + r.tile_samples - 1) / r.tile_samples;
    const uint64_t more = std::min<uint64_t>({left, want, cap - used});
    tk.second += more;
    used += more;
    used_samples += more * r.tile_samples;
  }
  // tile table: FP32 tiles and FP64 tiles of the any-family kernels, then one
  // group per variant that runs in a kernel of its own: a user integrand
  // (integrand, precision, N, M) or a compiled-in family with
  // N > kAnyMaxDims (family, precision, N)
  uint32_t n32 = 0, n = 0;
  for (int pass = 0; pass < 2; ++pass) {
    const int prec = pass == 0 ? ZMC_FP32_MERGE64 : ZMC_FP64;
    for (auto& tk : take) {
      Request& r = *tk.first;
      if (r.desc.precision != prec || own_kernel(r)) continue;
      for (uint64_t t = 0; t < tk.second; ++t) ht[n++] = tile_of(r, r.next_tile + t);
    }
    if (pass == 0) n32 = n;
  }
  const uint32_t n_builtin = n;
  struct VariantGroup {
    const Request* first;
    uint32_t begin, end;
  };
  std::vector<VariantGroup> groups;
  std::vector<bool> placed(take.size(), false);
  for (size_t a = 0; a < take.size(); ++a) {
    const Request& ra = *take[a].first;
    if (!own_kernel(ra) || placed[a]) continue;
    VariantGroup grp{&ra, n, n};
    for (size_t b = a; b < take.size(); ++b) {
      Request& rb = *take[b].first;
      if (placed[b] || !own_kernel(rb) || !same_variant(ra, rb)) continue;
      placed[b] = true;
      for (uint64_t t = 0; t < take[b].second; ++t) ht[n++] = tile_of(rb, rb.next_tile + t);
    }
    grp.end = n;
    groups.push_back(grp);
  }
  std::vector<uint32_t> merges;
  uint64_t max_g = 0;
  out->finishing.clear();
  for (auto& tk : take) {
    Request& r = *tk.first;
    r.next_tile += tk.second;
    if (r.next_tile == r.total_tiles) {
      out->finishing.push_back(tk.first);
      if (r.plan.splits > 1) merges.push_back((uint32_t)r.slot), max_g = std::max(max_g, r.G);
    }
  }
  hipStream_t st = s->streams[si];
  zmc::Tile* dt = s->d_tiles + (size_t)ring_slot * cap;
  uint32_t* dc = s->d_counters + (size_t)s->counters_per_slot * ring_slot;
  // the other stream's admissions (slot table, staged lists) come first
  hipError_t e = hipStreamWaitEvent(st, s->admit_events[1 - si], 0);
  if (e == hipSuccess) e = hipMemcpyAsync(dt, ht, sizeof(zmc::Tile) * n, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = zmc::launch_reset_counters(dc, 2 + (int)groups.size(), st);
  if (e == hipSuccess && n32 > 0)
    e = zmc::launch_batch_any(ZMC_FP32_MERGE64, s->d_slots, dt, 0, n32, dc, s->blocks32, st);
  if (e == hipSuccess && n_builtin > n32)
    e = zmc::launch_batch_any(ZMC_FP64, s->d_slots, dt, n32, n_builtin, dc + 1, s->blocks64, st);
  for (size_t gi = 0; e == hipSuccess && gi < groups.size(); ++gi) {
    const VariantGroup& grp = groups[gi];
    const zmc_scan_desc& d = grp.first->desc;
    const unsigned blocks = std::max(1u, std::min(grp.first->own_blocks, grp.end - grp.begin));
    e = d.family == ZMC_USER
            ? zmc::launch_user_batch(grp.first->user, s->d_slots, dt, grp.begin, grp.end,
                                     dc + 2 + gi, blocks, st)
            : zmc::launch_batch_variant(d.precision, d.family, d.N, s->d_slots, dt, grp.begin,
                                        grp.end, dc + 2 + gi, blocks, st);
  }
  if (e == hipSuccess && !merges.empty()) {
    // a finishing request's earlier tiles may sit in the other stream's slice
    if (s->slice_count > 0) e = hipStreamWaitEvent(st, s->done_events[(ring_slot + s->ring - 1) % s->ring], 0);
    uint32_t* hm = s->h_merge + (size_t)ring_slot * (size_t)s->opts.max_slots;
    std::copy(merges.begin(), merges.end(), hm);
    uint32_t* dm = s->d_merge + (size_t)ring_slot * (size_t)s->opts.max_slots;
    if (e == hipSuccess)
      e = hipMemcpyAsync(dm, hm, sizeof(uint32_t) * merges.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = zmc::launch_merge_batch(s->d_slots, dm, (int)merges.size(), max_g, st);
  }
  if (e == hipSuccess) e = hipEventRecord(s->done_events[ring_slot], st);
  out->done_ev = s->done_events[ring_slot];
  out->samples = used_samples;
  out->t_launch = Clock::now();
  std::lock_guard<std::mutex> lk(s->mu);
  s->stats.slices++;
  s->stats.slice_samples_now = s->slice_budget;
  s->stats.tiles += n;
  return e;
}

// slice_us: the device's throughput is measured on slices of at least
// slice_samples samples (the default budget, enough tiles to keep the device
// busy with two slices in flight), as the samples such slices retire over the
// time they take, in windows of at least kRateWindow seconds and four slices
// (several slices are often seen done at once).  Each window updates an
// exponential average, and the budget becomes that rate times slice_us.
// Smaller slices are left out: a slice shorter than a tile's duration is
// bound by the tile, not by the device's throughput, and counting it would
// shrink the budget further.
constexpr double kRateWindow = 0.02;  // seconds

void update_slice_budget(zmc_server* s, const Slice& sl) {
  const Clock::time_point now = Clock::now();
  const Clock::time_point start = std::max(sl.t_launch, s->t_last_retire);
  s->t_last_retire = now;
  if (s->opts.slice_us <= 0) return;
  if (sl.samples < s->opts.slice_samples) {  // a small slice ends the window
    s->acc_samples = s->acc_slices = 0;
    s->acc_seconds = 0.0;
    return;
  }
  s->acc_samples += sl.samples;
  s->acc_slices += 1;
  s->acc_seconds += std::max(0.0, std::chrono::duration<double>(now - start).count());
  if (s->acc_seconds < kRateWindow || s->acc_slices < 4) return;
  const double r = (double)s->acc_samples / s->acc_seconds;
  s->acc_samples = s->acc_slices = 0;
  s->acc_seconds = 0.0;
  s->rate = s->rate > 0.0 ? 0.5 * s->rate + 0.5 * r : r;
  const double want = s->rate * 1e-6 * (double)s->opts.slice_us;
  s->slice_budget = (uint64_t)std::min<double>((double)kMaxSliceSamples,
                                               std::max<double>((double)kMinSliceSamples, want));
}

void retire(zmc_server* s, Slice& sl) {
  update_slice_budget(s, sl);
  for (const ReqPtr& r : sl.finishing) {
    if (r->dmem) (void)hipFreeAsync(r->dmem, s->streams[r->alloc_stream]);
    r->dmem = nullptr;
    s->bytes_in_use -= r->footprint;
    s->free_slots.push_back(r->slot);
    finish(s, r, ZMC_OK);
  }
  s->active.erase(std::remove_if(s->active.begin(), s->active.end(),
                                 [](const ReqPtr& r) { return r->done; }),
                  s->active.end());
}

// Queued requests in admission order: arrival order, or for shortest-first
// ascending estimated work, equal work in arrival order.
void enqueue_pending(zmc_server* s, const ReqPtr& r) {
  if (s->opts.admission != ZMC_ADMIT_SHORTEST) {
    s->pending.push_back(r);
    return;
  }
  const auto at = std::upper_bound(s->pending.begin(), s->pending.end(), r,
                                   [](const ReqPtr& a, const ReqPtr& b) { return a->work < b->work; });
  s->pending.insert(at, r);
}

// Index in `pending` of the request to admit next: the front, unless a
// shortest-first queue holds requests past max_wait_ms; then the oldest.
size_t next_pending(const zmc_server* s) {
  if (s->opts.admission != ZMC_ADMIT_SHORTEST || s->opts.max_wait_ms <= 0) return 0;
  size_t oldest = 0;
  for (size_t i = 1; i < s->pending.size(); ++i)
    if (s->pending[i]->ticket < s->pending[oldest]->ticket) oldest = i;
  const double waited =
      std::chrono::duration<double>(Clock::now() - s->pending[oldest]->t_submit).count();
  return waited * 1e3 > (double)s->opts.max_wait_ms ? oldest : 0;
}

// Finishes the queued requests that zmc_server_cancel has flagged.
void drop_cancelled(zmc_server* s) {
  std::vector<ReqPtr> gone;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    for (const ReqPtr& r : s->pending)
      if (r->cancelled) gone.push_back(r);
  }
  if (gone.empty()) return;
  s->pending.erase(std::remove_if(s->pending.begin(), s->pending.end(),
                                  [&](const ReqPtr& r) {
                                    return std::find(gone.begin(), gone.end(), r) != gone.end();
                                  }),
                   s->pending.end());
  for (const ReqPtr& r : gone) finish(s, r, ZMC_E_CANCELLED);
}

void fail_all(zmc_server* s, zmc_status st) {
  for (Slice& sl : s->inflight)
    for (const ReqPtr& r : sl.finishing)
      if (!r->done) finish(s, r, st);
  s->inflight.clear();
  for (const ReqPtr& r : s->active)
    if (!r->done) finish(s, r, st);
  s->active.clear();
  for (const ReqPtr& r : s->pending) finish(s, r, st);
  s->pending.clear();
}

void run(zmc_server* s) {
  (void)hipSetDevice(s->device);
  bool broken = false;
  for (;;) {
    bool stopping;
    {
      std::lock_guard<std::mutex> lk(s->mu);
      while (!s->incoming.empty()) {
        enqueue_pending(s, s->incoming.front());
        s->incoming.pop_front();
      }
      stopping = s->stop;
    }
    drop_cancelled(s);
    if (broken) {
      fail_all(s, ZMC_E_DEVICE);
      if (stopping) break;
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_work.wait_for(lk, std::chrono::milliseconds(50));
      continue;
    }
    bool progressed = false;
    while (!s->inflight.empty()) {
      const hipError_t q = hipEventQuery(s->inflight.front().done_ev);
      if (q == hipErrorNotReady) break;
      if (q != hipSuccess) {
        broken = true;
        break;
      }
      retire(s, s->inflight.front());
      s->inflight.pop_front();
      progressed = true;
    }
    if (broken) continue;
    const int si = (int)(s->slice_count % kStreams);
    bool admitted = false;
    while (!s->pending.empty() && !s->free_slots.empty()) {
      const size_t j = next_pending(s);
      ReqPtr r = s->pending[j];
      if (r->footprint > s->opts.hbm_budget_bytes) {
        s->pending.erase(s->pending.begin() + (std::ptrdiff_t)j);
        bool cancelled;
        {
          std::lock_guard<std::mutex> lk(s->mu);
          cancelled = r->cancelled;
        }
        finish(s, r, cancelled ? ZMC_E_CANCELLED : ZMC_E_NOMEM);
        continue;
      }
      if (s->bytes_in_use + r->footprint > s->opts.hbm_budget_bytes) break;
      s->pending.erase(s->pending.begin() + (std::ptrdiff_t)j);
      {
        // from here the request is admitted: zmc_server_cancel answers BUSY
        std::lock_guard<std::mutex> lk(s->mu);
        if (!r->cancelled) r->admitted = true;
      }
      if (!r->admitted) {
        finish(s, r, ZMC_E_CANCELLED);
        continue;
      }
      if (r->desc.family == ZMC_USER) {
        // built (first use of this shape) and loaded on the server's device
        const zmc_status us = zmc::user_kernels(r->desc.integrand, r->desc.precision, r->desc.N,
                                                r->desc.M, &r->user);
        int per_cu = 0;
        if (us != ZMC_OK || zmc::user_batch_occupancy(r->user, &per_cu) != hipSuccess) {
          finish(s, r, us != ZMC_OK ? us : ZMC_E_DEVICE);
          continue;
        }
        r->own_blocks = (unsigned)std::max(1, s->cu * std::max(1, per_cu));
      } else if (r->desc.N > zmc::kAnyMaxDims) {
        int per_cu = 0;
        if (zmc::batch_occupancy(r->desc.precision, r->desc.family, r->desc.N, &per_cu) != hipSuccess) {
          finish(s, r, ZMC_E_DEVICE);
          continue;
        }
        r->own_blocks = (unsigned)std::max(1, s->cu * std::max(1, per_cu));
      }
      if (admit(s, r, si) != hipSuccess) {
        finish(s, r, ZMC_E_DEVICE);
        broken = true;
        break;
      }
      s->bytes_in_use += r->footprint;
      zmc::log(2, "server: request %llu admitted (slot %d, %llu B, %llu tiles)",
               (unsigned long long)r->ticket, r->slot, (unsigned long long)r->footprint,
               (unsigned long long)r->total_tiles);
      s->active.push_back(r);
      admitted = progressed = true;
      std::lock_guard<std::mutex> lk(s->mu);
      s->stats.admitted++;
      s->stats.bytes_in_use = s->bytes_in_use;
      s->stats.bytes_peak = std::max(s->stats.bytes_peak, s->bytes_in_use);
    }
    if (broken) continue;
    if (admitted && hipEventRecord(s->admit_events[si], s->streams[si]) != hipSuccess) {
      broken = true;
      continue;
    }
    if ((int)s->inflight.size() < s->opts.max_inflight) {
      Slice sl;
      if (launch_slice(s, si, &sl) != hipSuccess) {
        broken = true;
        continue;
      }
      if (sl.done_ev != nullptr) {
        s->inflight.push_back(std::move(sl));
        s->slice_count++;
        progressed = true;
      }
    }
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->stats.pending = s->pending.size() + s->incoming.size();
      s->stats.active = s->active.size();
      s->stats.bytes_in_use = s->bytes_in_use;
    }
    if (stopping && s->pending.empty() && s->active.empty() && s->inflight.empty()) break;
    if (!progressed) {
      if (!s->inflight.empty()) {
        if (hipEventSynchronize(s->inflight.front().done_ev) != hipSuccess) broken = true;
      } else {
        std::unique_lock<std::mutex> lk(s->mu);
        s->cv_work.wait_for(lk, std::chrono::milliseconds(20),
                            [&] { return !s->incoming.empty() || s->stop; });
      }
    }
  }
  for (int i = 0; i < kStreams; ++i) (void)hipStreamSynchronize(s->streams[i]);
}

void release(zmc_server* s) {
  for (hipEvent_t ev : s->done_events)
    if (ev) (void)hipEventDestroy(ev);
  for (hipEvent_t ev : s->admit_events)
    if (ev) (void)hipEventDestroy(ev);
  for (int i = 0; i < kStreams; ++i)
    if (s->streams[i]) (void)hipStreamDestroy(s->streams[i]);
  if (s->dmem) (void)hipFree(s->dmem);
  if (s->h_slots) (void)hipHostFree(s->h_slots);
  if (s->h_tiles) (void)hipHostFree(s->h_tiles);
  if (s->h_merge) (void)hipHostFree(s->h_merge);
  delete s;
}

}  // namespace

extern "C" {

zmc_status zmc_server_create(const zmc_server_opts* opts, zmc_server** out) {
  if (out == nullptr) return fail(ZMC_E_INVALID, "out is NULL");
  *out = nullptr;
  zmc_server* s = new (std::nothrow) zmc_server();
  if (s == nullptr) return fail(ZMC_E_NOMEM, "host allocation failed");
  if (opts) s->opts = *opts;
  zmc_server_opts& o = s->opts;
  if (o.hbm_budget_bytes == 0) o.hbm_budget_bytes = (uint64_t)64 << 30;
  if (o.max_slots <= 0) o.max_slots = 256;
  if (o.max_inflight <= 0) o.max_inflight = 2;
  if (o.max_slots > 65536 || o.max_inflight > 16) {
    delete s;
    return fail(ZMC_E_INVALID, "max_slots <= 65536 and max_inflight <= 16 required");
  }
  if ((o.admission != ZMC_ADMIT_FIFO && o.admission != ZMC_ADMIT_SHORTEST) || o.max_wait_ms < 0) {
    delete s;
    return fail(ZMC_E_INVALID, "admission must be ZMC_ADMIT_FIFO or ZMC_ADMIT_SHORTEST and "
                "max_wait_ms >= 0");
  }
  if (o.slice_us < 0) {
    delete s;
    return fail(ZMC_E_INVALID, "slice_us = %d < 0", o.slice_us);
  }
  s->ring = o.max_inflight + 1;
  hipError_t e = hipGetDevice(&s->device);
  int cu = o.cu_count;
  if (e == hipSuccess && cu <= 0) {
    zmc_status st = zmc::cu_count(&cu);
    if (st != ZMC_OK) {
      delete s;
      return st;
    }
  }
  int per32 = 1, per64 = 1;
  if (e == hipSuccess) e = zmc::batch_any_occupancy(ZMC_FP32_MERGE64, &per32);
  if (e == hipSuccess) e = zmc::batch_any_occupancy(ZMC_FP64, &per64);
  s->cu = std::max(1, cu);
  s->blocks32 = (unsigned)std::max(1, cu * std::max(1, per32));
  s->blocks64 = (unsigned)std::max(1, cu * std::max(1, per64));
  if (o.slice_tiles <= 0) o.slice_tiles = (int32_t)std::min<uint64_t>(64ull * s->blocks32, 1u << 20);
  if (o.slice_samples == 0) o.slice_samples = 4000000000ull;
  s->slice_budget = o.slice_samples;
  const size_t cap = (size_t)o.slice_tiles, ring = (size_t)s->ring, slots = (size_t)o.max_slots;
  const size_t off_tiles = align_up(sizeof(zmc::ScanParams) * slots);
  const size_t off_counters = off_tiles + align_up(sizeof(zmc::Tile) * cap * ring);
  s->counters_per_slot = 2 + o.max_slots;
  const size_t off_merge =
      off_counters + align_up(sizeof(uint32_t) * (size_t)s->counters_per_slot * ring);
  const size_t total = off_merge + align_up(sizeof(uint32_t) * slots * ring);
  if (e == hipSuccess) e = hipMalloc(&s->dmem, total);
  if (e == hipSuccess) e = hipHostMalloc((void**)&s->h_slots, sizeof(zmc::ScanParams) * slots, 0);
  if (e == hipSuccess) e = hipHostMalloc((void**)&s->h_tiles, sizeof(zmc::Tile) * cap * ring, 0);
  if (e == hipSuccess) e = hipHostMalloc((void**)&s->h_merge, sizeof(uint32_t) * slots * ring, 0);
  for (int i = 0; e == hipSuccess && i < kStreams; ++i)
    e = hipStreamCreateWithFlags(&s->streams[i], hipStreamNonBlocking);
  s->done_events.assign(ring, nullptr);
  s->admit_events.assign(kStreams, nullptr);
  for (size_t i = 0; e == hipSuccess && i < ring; ++i)
    e = hipEventCreateWithFlags(&s->done_events[i], hipEventDisableTiming | hipEventBlockingSync);
  for (int i = 0; e == hipSuccess && i < kStreams; ++i) {
    e = hipEventCreateWithFlags(&s->admit_events[i], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(s->admit_events[i], s->streams[i]);
  }
  if (e != hipSuccess) {
    release(s);
    return fail(ZMC_E_DEVICE, "server setup failed: %s", hipGetErrorString(e));
  }
  char* base = (char*)s->dmem;
  s->d_slots = (zmc::ScanParams*)base;
  s->d_tiles = (zmc::Tile*)(base + off_tiles);
  s->d_counters = (uint32_t*)(base + off_counters);
  s->d_merge = (uint32_t*)(base + off_merge);
  for (int i = o.max_slots - 1; i >= 0; --i) s->free_slots.push_back(i);
  try {
    s->thread = std::thread(run, s);
  } catch (...) {
    release(s);
    return fail(ZMC_E_NOMEM, "could not start the scheduler thread");
  }
  zmc::log(1, "server: budget %llu B, %d slots, %d tiles and %llu samples per slice, device %d",
           (unsigned long long)o.hbm_budget_bytes, o.max_slots, o.slice_tiles,
           (unsigned long long)o.slice_samples, s->device);
  *out = s;
  return ok();
}

zmc_status zmc_server_submit(zmc_server* s, const zmc_scan_desc* desc, const double* d_axis_vals,
                             double* d_f, double* d_sigma, uint64_t* ticket) {
  zmc::TraceRange trace_range("zmc_server_submit");
  if (s == nullptr || ticket == nullptr) return fail(ZMC_E_INVALID, "NULL server or ticket");
  uint64_t G = 0;
  zmc_status st = zmc::validate_desc(desc, &G);
  if (st != ZMC_OK) return st;
  if (d_f == nullptr || d_sigma == nullptr) return fail(ZMC_E_INVALID, "d_f or d_sigma is NULL");
  if (desc->M > 0 && d_axis_vals == nullptr && desc->axis_vals == nullptr)
    return fail(ZMC_E_INVALID, "no parameter lists (host or device)");
  auto r = std::make_shared<Request>();
  r->desc = *desc;
  r->axis_len.assign(desc->axis_len, desc->axis_len + desc->M);
  uint64_t total = 0;
  for (int l = 0; l < desc->M; ++l) total += (uint64_t)desc->axis_len[l];
  if (d_axis_vals == nullptr) {
    r->axis_vals.assign(desc->axis_vals, desc->axis_vals + total);
    r->staged_doubles = total;
  }
  r->lo.assign(desc->lo, desc->lo + desc->N);
  r->hi.assign(desc->hi, desc->hi + desc->N);
  r->desc.axis_len = r->axis_len.data();
  r->desc.axis_vals = r->axis_vals.empty() ? nullptr : r->axis_vals.data();
  r->desc.lo = r->lo.data();
  r->desc.hi = r->hi.data();
  r->params.assign(desc->params, desc->params + std::max(0, desc->n_params));
  r->desc.params = r->params.empty() ? nullptr : r->params.data();
  r->d_axis_user = d_axis_vals;
  r->d_f = d_f;
  r->d_sigma = d_sigma;
  r->G = G;
  st = zmc::plan_tiles(&r->desc, G, 0, 0, 0, &r->plan, &r->total_tiles);
  if (st != ZMC_OK) return st;
  r->tile_samples = (uint64_t)std::max(
      1.0, (double)G * (double)desc->samples / (double)std::max<uint64_t>(1, r->total_tiles));
  r->footprint = align_up(8 * r->staged_doubles) + r->plan.workspace_bytes;
  r->work = (double)G * (double)r->desc.samples * (double)r->desc.N;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return fail(ZMC_E_BUSY, "server is shutting down");
    r->t_submit = Clock::now();  // in ticket order: the oldest request has the lowest ticket
    r->ticket = s->next_ticket++;
    s->tickets[r->ticket] = r;
    if (!s->any_submitted) {
      s->any_submitted = true;
      s->t_first_submit = r->t_submit;
    }
    s->incoming.push_back(r);
    s->stats.submitted++;
  }
  s->cv_work.notify_one();
  *ticket = r->ticket;
  return ok();
}

zmc_status zmc_server_poll(zmc_server* s, uint64_t ticket, int32_t* done, zmc_status* result,
                           double* latency_s) {
  if (s == nullptr || done == nullptr) return fail(ZMC_E_INVALID, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return fail(ZMC_E_INVALID, "unknown ticket %llu", (unsigned long long)ticket);
  *done = it->second->done ? 1 : 0;
  if (result) *result = it->second->done ? it->second->status : ZMC_OK;
  if (latency_s) *latency_s = it->second->done ? it->second->latency : 0.0;
  return ok();
}

zmc_status zmc_server_wait(zmc_server* s, uint64_t ticket, zmc_status* result, double* latency_s) {
  if (s == nullptr) return fail(ZMC_E_INVALID, "NULL server");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return fail(ZMC_E_INVALID, "unknown ticket %llu", (unsigned long long)ticket);
  ReqPtr r = it->second;
  s->cv_done.wait(lk, [&] { return r->done; });
  if (result) *result = r->status;
  if (latency_s) *latency_s = r->latency;
  return ok();
}

zmc_status zmc_server_release(zmc_server* s, uint64_t ticket) {
  if (s == nullptr) return fail(ZMC_E_INVALID, "NULL server");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return fail(ZMC_E_INVALID, "unknown ticket %llu", (unsigned long long)ticket);
  if (!it->second->done)
    return fail(ZMC_E_BUSY, "request %llu has not finished", (unsigned long long)ticket);
  s->tickets.erase(it);  // a thread still in zmc_server_wait holds its own reference
  return ok();
}

zmc_status zmc_server_cancel(zmc_server* s, uint64_t ticket) {
  if (s == nullptr) return fail(ZMC_E_INVALID, "NULL server");
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return fail(ZMC_E_INVALID, "unknown ticket %llu", (unsigned long long)ticket);
    Request& r = *it->second;
    if (r.done || r.admitted)
      return fail(ZMC_E_BUSY, "request %llu has %s", (unsigned long long)ticket,
                  r.done ? "finished" : "been admitted");
    r.cancelled = true;
  }
  s->cv_work.notify_one();
  return ok();
}

zmc_status zmc_server_get_stats(zmc_server* s, zmc_server_stats* stats) {
  if (s == nullptr || stats == nullptr) return fail(ZMC_E_INVALID, "NULL argument");
  std::vector<double> v;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    *stats = s->stats;
    stats->tickets = (uint64_t)s->tickets.size();
    v = s->latencies;
    const double span =
        std::chrono::duration<double>(s->t_last_done - s->t_first_submit).count();
    stats->samples_per_s =
        (!v.empty() && span > 0.0) ? (double)s->stats.samples_completed / span : 0.0;
  }
  stats->latency_p50_s = stats->latency_p99_s = stats->latency_max_s = 0.0;
  if (!v.empty()) {
    std::sort(v.begin(), v.end());
    // linear interpolation between order statistics at q (n - 1)
    const auto pct = [&v](double q) {
      const double pos = q * (double)(v.size() - 1);
      const size_t i = (size_t)pos;
      const double frac = pos - (double)i;
      return i + 1 < v.size() ? v[i] + frac * (v[i + 1] - v[i]) : v[i];
    };
    stats->latency_p50_s = pct(0.50);
    stats->latency_p99_s = pct(0.99);
    stats->latency_max_s = v.back();
  }
  return ok();
}

zmc_status zmc_server_destroy(zmc_server* s) {
  if (s == nullptr) return ok();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->thread.joinable()) s->thread.join();
  release(s);
  return ok();
}

}  // extern "C"
