// zmc_batch.hip -- host side of batched scans: tile planning from the tuned
// table, device tables, and the captured hipGraph (include/zmc.h).
//
// The paper cuts one grid into batches and gives each batch to a GPU (Sec. 2,
// Fig. 1).  Here many scans share one GPU: every scan is cut into tiles whose
// shape depends only on that scan and the tuned table, the tiles of each
// kernel variant are sorted longest first, and one persistent kernel per
// variant drains them; split partials are merged afterwards in split order.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <functional>
#include <new>
#include <vector>

#include "zmc.h"
#include "zmc_device.hpp"
#include "zmc_internal.hpp"
#include "zmc_trace.hpp"

using zmc::fail;
using zmc::ok;

namespace zmc {

// The tiled decomposition of one scan (batches and the server): a function of
// the scan and the tuned table only, so a scan's results do not depend on
// what else runs with it.  Point-major tiles hold 256 consecutive points and
// `pm_groups` groups of four samples per lane; grids below `pm_min_points`
// get sample-major tiles of `sm_groups` groups (all lanes together).  The
// partials of one scan are kept below 2 GiB by lengthening its pieces.
zmc_status plan_tiles(const zmc_scan_desc* d, uint64_t G, int64_t pm_groups_override,
                      int64_t sm_groups_override, int64_t pm_min_override, Plan* pl,
                      uint64_t* tiles) {
  const TuneEntry t = tune_lookup(d->family, d->precision, d->N);
  const int64_t pm_groups = pm_groups_override > 0 ? pm_groups_override : t.pm_groups;
  const int64_t sm_groups = sm_groups_override > 0 ? sm_groups_override : t.sm_groups;
  const int64_t pm_min = pm_min_override > 0 ? pm_min_override : t.pm_min_points;
  const uint64_t groups = (d->samples + 3) / 4;
  pl->mode = (G >= (uint64_t)pm_min) ? ZMC_MODE_POINT_MAJOR : ZMC_MODE_SAMPLE_MAJOR;
  pl->block = kTileBlock;
  const uint64_t gpt = (uint64_t)(pl->mode == ZMC_MODE_POINT_MAJOR ? pm_groups : sm_groups);
  uint64_t splits = (groups + gpt - 1) / gpt;
  while (splits > 1 && 16.0 * (double)splits * (double)G > (double)kMaxPartialBytesPerScan)
    splits = (splits + 1) / 2;
  if (splits > 0x7FFFFFFFull) return fail(ZMC_E_UNSUPPORTED, "too many sample pieces");
  const uint64_t gps = (groups + splits - 1) / splits;
  splits = (groups + gps - 1) / gps;
  const zmc_status pst = check_pieces(groups, gps, splits);
  if (pst != ZMC_OK) return pst;
  pl->splits = (int)splits;
  pl->groups = groups;
  pl->gps = gps;
  pl->point_blocks = (G + kTileBlock - 1) / kTileBlock;
  pl->grid_x = 0;
  pl->workspace_bytes = splits > 1 ? 16 * splits * G : 0;
  *tiles = (pl->mode == ZMC_MODE_POINT_MAJOR ? pl->point_blocks : G) * splits;
  return ZMC_OK;
}

}  // namespace zmc

namespace {

constexpr int kBlock = zmc::kTileBlock;
constexpr uint64_t kMaxTiles = (uint64_t)1 << 31;
constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// One persistent kernel per key: (precision, family, N) for the compiled-in
// families (family -1: the any-family kernel), plus the handle and M for a
// user integrand, whose kernel is built at run time for that shape.
struct VariantKey {
  int precision, family, N;
  const zmc_integrand* integrand = nullptr;
  int M = 0;
  bool operator<(const VariantKey& o) const {
    if (precision != o.precision) return precision < o.precision;
    if (family != o.family) return family < o.family;
    if (N != o.N) return N < o.N;
    if (integrand != o.integrand) return std::less<const zmc_integrand*>()(integrand, o.integrand);
    return M < o.M;
  }
  bool operator==(const VariantKey& o) const {
    return precision == o.precision && family == o.family && N == o.N &&
           integrand == o.integrand && M == o.M;
  }
};

struct ScanPlanB {
  uint64_t G = 0;
  zmc::Plan plan{};
  int variant = -1;
  uint64_t tiles = 0;
  uint64_t partial_bytes = 0;
  uint64_t axis_len_total = 0;
};

struct Variant {
  VariantKey key;
  uint32_t begin = 0, end = 0;
  unsigned blocks = 0;
  zmc::UserKernels user;  // family ZMC_USER: the run-time-built kernels
};

struct TileCost {
  zmc::Tile tile;
  uint64_t cost;
};

struct BatchPlan {
  std::vector<ScanPlanB> scans;
  std::vector<Variant> variants;
  std::vector<zmc::Tile> tiles;
  std::vector<uint32_t> merge;
  uint64_t partial_bytes = 0, staged_doubles = 0, max_merge_G = 0, samples = 0, points = 0;
};

zmc_status plan_scan(const zmc_scan_desc* d, uint64_t G, const zmc_batch_opts* o, ScanPlanB* sp) {
  zmc_status st = zmc::plan_tiles(d, G, o ? o->pm_groups : 0, o ? o->sm_groups : 0,
                                  o ? o->pm_min_points : 0, &sp->plan, &sp->tiles);
  if (st != ZMC_OK) return st;
  sp->G = G;
  sp->partial_bytes = sp->plan.workspace_bytes;
  return ZMC_OK;
}

zmc_status plan_batch(const zmc_scan_desc* scans, int32_t n, const zmc_batch_opts* o,
                      bool build_tiles, BatchPlan* bp) {
  if (n < 1) return fail(ZMC_E_INVALID, "n_scans = %d < 1", n);
  if (scans == nullptr) return fail(ZMC_E_INVALID, "scans is NULL");
  bp->scans.assign((size_t)n, ScanPlanB{});
  std::vector<VariantKey> keys;
  uint64_t total_tiles = 0;
  for (int i = 0; i < n; ++i) {
    uint64_t G = 0;
    zmc_status st = zmc::validate_desc(&scans[i], &G);
    if (st != ZMC_OK) {
      char why[400];
      snprintf(why, sizeof(why), "%s", zmc_last_error());
      return fail(st, "scan %d: %s", i, why);
    }
    ScanPlanB& sp = bp->scans[(size_t)i];
    st = plan_scan(&scans[i], G, o, &sp);
    if (st != ZMC_OK) return st;
    for (int l = 0; l < scans[i].M; ++l) sp.axis_len_total += (uint64_t)scans[i].axis_len[l];
    total_tiles += sp.tiles;
    if (total_tiles > kMaxTiles) return fail(ZMC_E_UNSUPPORTED, "batch has more than 2^31 tiles");
    if (scans[i].family == ZMC_USER)
      keys.push_back(VariantKey{scans[i].precision, ZMC_USER, scans[i].N, scans[i].integrand,
                                scans[i].M});
    else if (o && o->one_kernel && scans[i].N <= zmc::kAnyMaxDims)
      keys.push_back(VariantKey{scans[i].precision, -1, 0});
    else
      keys.push_back(VariantKey{scans[i].precision, scans[i].family, scans[i].N});
    bp->samples += G * scans[i].samples;
    bp->points += G;
    bp->staged_doubles += sp.axis_len_total;
    if (sp.plan.splits > 1) {
      bp->partial_bytes += sp.partial_bytes;
      bp->merge.push_back((uint32_t)i);
      bp->max_merge_G = std::max(bp->max_merge_G, G);
    }
  }
  std::vector<VariantKey> uniq = keys;
  std::sort(uniq.begin(), uniq.end());
  uniq.erase(std::unique(uniq.begin(), uniq.end()), uniq.end());
  bp->variants.assign(uniq.size(), Variant{});
  for (size_t v = 0; v < uniq.size(); ++v) bp->variants[v].key = uniq[v];
  for (int i = 0; i < n; ++i)
    bp->scans[(size_t)i].variant =
        (int)(std::lower_bound(uniq.begin(), uniq.end(), keys[(size_t)i]) - uniq.begin());
  if (!build_tiles) return ZMC_OK;

  // Tiles per variant, longest first (cost = lane-samples x per-sample work),
  // ties broken by (scan, first point, piece) so the order is reproducible.
  std::vector<std::vector<TileCost>> per(uniq.size());
  for (int i = 0; i < n; ++i) {
    const ScanPlanB& sp = bp->scans[(size_t)i];
    const zmc::Plan& pl = sp.plan;
    const uint64_t work = (uint64_t)(10 * scans[i].N + 8);
    auto& vec = per[(size_t)sp.variant];
    for (uint64_t s = 0; s < (uint64_t)pl.splits; ++s) {
      const uint64_t samples = zmc::split_samples(scans[i].samples, pl.groups, pl.gps, s);
      if (pl.mode == ZMC_MODE_POINT_MAJOR) {
        for (uint64_t pb = 0; pb < pl.point_blocks; ++pb) {
          const uint64_t first = pb * kBlock;
          const uint64_t lanes = std::min<uint64_t>(kBlock, sp.G - first);
          vec.push_back(TileCost{zmc::Tile{(uint32_t)i, (uint32_t)s, first}, lanes * samples * work});
        }
      } else {
        for (uint64_t g = 0; g < sp.G; ++g)
          vec.push_back(TileCost{zmc::Tile{(uint32_t)i, (uint32_t)s | zmc::kTileSampleMajor, g},
                                 samples * work});
      }
    }
  }
  bp->tiles.clear();
  bp->tiles.reserve((size_t)total_tiles);
  for (size_t v = 0; v < per.size(); ++v) {
    auto& vec = per[v];
    std::stable_sort(vec.begin(), vec.end(), [](const TileCost& a, const TileCost& b) {
      if (a.cost != b.cost) return a.cost > b.cost;
      if (a.tile.scan != b.tile.scan) return a.tile.scan < b.tile.scan;
      if (a.tile.first != b.tile.first) return a.tile.first < b.tile.first;
      return a.tile.split_mode < b.tile.split_mode;
    });
    bp->variants[v].begin = (uint32_t)bp->tiles.size();
    for (const TileCost& tc : vec) bp->tiles.push_back(tc.tile);
    bp->variants[v].end = (uint32_t)bp->tiles.size();
    std::vector<TileCost>().swap(vec);
  }
  return ZMC_OK;
}

void fill_info(const BatchPlan& bp, int n, bool graph, zmc_batch_info* info) {
  memset(info, 0, sizeof(*info));
  info->scans = n;
  info->variants = (int32_t)bp.variants.size();
  uint64_t tiles = 0;
  for (const ScanPlanB& sp : bp.scans) tiles += sp.tiles;
  info->tiles = (int64_t)tiles;
  info->samples = bp.samples;
  info->points = bp.points;
  const size_t tables = align_up(sizeof(zmc::ScanParams) * bp.scans.size()) +
                        align_up(sizeof(zmc::Tile) * tiles) +
                        align_up(sizeof(uint32_t) * bp.variants.size()) +
                        align_up(sizeof(uint32_t) * bp.merge.size());
  info->workspace_bytes = tables + align_up(8 * bp.staged_doubles) + bp.partial_bytes;
  info->merge_scans = (int32_t)bp.merge.size();
  info->graph = graph ? 1 : 0;
}

}  // namespace

struct zmc_batch {
  int device = 0;
  void* dmem = nullptr;
  zmc::ScanParams* d_scans = nullptr;
  zmc::Tile* d_tiles = nullptr;
  uint32_t* d_counters = nullptr;
  uint32_t* d_merge = nullptr;
  std::vector<Variant> variants;
  int n_merge = 0;
  uint64_t max_merge_G = 0;
  bool use_graph = true, parallel = true;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  zmc_batch_info info{};
};

namespace {

// Enqueues reset -> variant kernels -> merge.  With `branches` the variant
// kernels are forked onto their own streams and joined again, so that a
// capture records them as parallel graph branches.
hipError_t enqueue(zmc_batch* b, hipStream_t s, const std::vector<hipStream_t>& branches,
                   const std::vector<hipEvent_t>& events) {
  hipError_t e = zmc::launch_reset_counters(b->d_counters, (int)b->variants.size(), s);
  const bool fork = !branches.empty();
  if (e == hipSuccess && fork) e = hipEventRecord(events[0], s);
  for (size_t v = 0; e == hipSuccess && v < b->variants.size(); ++v) {
    const Variant& var = b->variants[v];
    hipStream_t sv = fork ? branches[v] : s;
    if (fork) e = hipStreamWaitEvent(sv, events[0], 0);
    if (e == hipSuccess && var.key.family < 0)
      e = zmc::launch_batch_any(var.key.precision, b->d_scans, b->d_tiles, var.begin, var.end,
                                b->d_counters + v, var.blocks, sv);
    else if (e == hipSuccess && var.key.family == ZMC_USER)
      e = zmc::launch_user_batch(var.user, b->d_scans, b->d_tiles, var.begin, var.end,
                                 b->d_counters + v, var.blocks, sv);
    else if (e == hipSuccess)
      e = zmc::launch_batch_variant(var.key.precision, var.key.family, var.key.N, b->d_scans,
                                    b->d_tiles, var.begin, var.end, b->d_counters + v, var.blocks,
                                    sv);
    if (e == hipSuccess && fork) e = hipEventRecord(events[1 + v], sv);
  }
  for (size_t v = 0; e == hipSuccess && fork && v < b->variants.size(); ++v)
    e = hipStreamWaitEvent(s, events[1 + v], 0);
  if (e == hipSuccess) e = zmc::launch_merge_batch(b->d_scans, b->d_merge, b->n_merge, b->max_merge_G, s);
  return e;
}

void release(zmc_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->dmem) (void)hipFree(b->dmem);
  delete b;
}

}  // namespace

extern "C" {

void zmc_batch_default_opts(zmc_batch_opts* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->use_graph = 1;
  o->parallel_variants = 1;
}

zmc_status zmc_batch_plan(const zmc_scan_desc* scans, int32_t n_scans, const zmc_batch_opts* opts,
                          zmc_batch_info* info) {
  if (info == nullptr) return fail(ZMC_E_INVALID, "info is NULL");
  BatchPlan bp;
  zmc_status st = plan_batch(scans, n_scans, opts, false, &bp);
  if (st != ZMC_OK) return st;
  fill_info(bp, n_scans, opts ? opts->use_graph != 0 : true, info);
  return ok();
}

zmc_status zmc_batch_create(const zmc_scan_desc* scans, int32_t n_scans,
                            const double* const* d_axis_vals, double* const* d_f,
                            double* const* d_sigma, const zmc_batch_opts* opts, zmc_batch** out) {
  zmc::TraceRange trace_range("zmc_batch_create");
  if (out == nullptr) return fail(ZMC_E_INVALID, "out is NULL");
  *out = nullptr;
  if (d_f == nullptr || d_sigma == nullptr) return fail(ZMC_E_INVALID, "d_f or d_sigma is NULL");
  zmc_batch_opts o;
  zmc_batch_default_opts(&o);
  if (opts) o = *opts;
  BatchPlan bp;
  zmc_status st = plan_batch(scans, n_scans, &o, true, &bp);
  if (st != ZMC_OK) return st;
  for (Variant& var : bp.variants) {
    if (var.key.family != ZMC_USER) continue;
    st = zmc::user_kernels(var.key.integrand, var.key.precision, var.key.N, var.key.M, &var.user);
    if (st != ZMC_OK) return st;
  }
  for (int i = 0; i < n_scans; ++i) {
    if (d_f[i] == nullptr || d_sigma[i] == nullptr)
      return fail(ZMC_E_INVALID, "scan %d: output pointer is NULL", i);
    if (scans[i].M > 0 && d_axis_vals == nullptr && scans[i].axis_vals == nullptr)
      return fail(ZMC_E_INVALID, "scan %d: no parameter lists (host or device)", i);
    if (scans[i].M > 0 && d_axis_vals != nullptr && d_axis_vals[i] == nullptr)
      return fail(ZMC_E_INVALID, "scan %d: d_axis_vals entry is NULL with M > 0", i);
  }
  int cu = o.cu_count;
  if (cu <= 0) {
    st = zmc::cu_count(&cu);
    if (st != ZMC_OK) return st;
  }

  zmc_batch* b = new (std::nothrow) zmc_batch();
  if (b == nullptr) return fail(ZMC_E_NOMEM, "host allocation failed");
  (void)hipGetDevice(&b->device);
  b->use_graph = o.use_graph != 0;
  b->parallel = o.parallel_variants != 0;
  b->variants = bp.variants;
  b->n_merge = (int)bp.merge.size();
  b->max_merge_G = bp.max_merge_G;
  fill_info(bp, n_scans, b->use_graph, &b->info);

  // one device allocation: scans | tiles | counters | merge list | lists | partials
  const size_t off_scans = 0;
  const size_t off_tiles = off_scans + align_up(sizeof(zmc::ScanParams) * (size_t)n_scans);
  const size_t off_counters = off_tiles + align_up(sizeof(zmc::Tile) * bp.tiles.size());
  const size_t off_merge = off_counters + align_up(sizeof(uint32_t) * bp.variants.size());
  const size_t off_axis = off_merge + align_up(sizeof(uint32_t) * std::max<size_t>(1, bp.merge.size()));
  const size_t off_part = off_axis + align_up(8 * (d_axis_vals ? 0 : bp.staged_doubles));
  const size_t total = off_part + align_up((size_t)bp.partial_bytes);
  hipError_t e = hipMalloc(&b->dmem, total);
  if (e != hipSuccess) {
    release(b);
    return fail(ZMC_E_NOMEM, "batch workspace of %zu bytes: %s", total, hipGetErrorString(e));
  }
  char* base = (char*)b->dmem;
  b->d_scans = (zmc::ScanParams*)(base + off_scans);
  b->d_tiles = (zmc::Tile*)(base + off_tiles);
  b->d_counters = (uint32_t*)(base + off_counters);
  b->d_merge = (uint32_t*)(base + off_merge);

  std::vector<zmc::ScanParams> params((size_t)n_scans);
  size_t axis_off = 0, part_off = 0;
  for (int i = 0; i < n_scans && e == hipSuccess; ++i) {
    const ScanPlanB& sp = bp.scans[(size_t)i];
    const double* axis = nullptr;
    if (d_axis_vals) {
      axis = d_axis_vals[i];
    } else if (sp.axis_len_total > 0) {
      double* dst = (double*)(base + off_axis) + axis_off;
      e = hipMemcpy(dst, scans[i].axis_vals, 8 * sp.axis_len_total, hipMemcpyHostToDevice);
      axis = dst;
      axis_off += sp.axis_len_total;
    }
    zmc::fill_scan_params(&scans[i], sp.G, sp.plan, axis, d_f[i], d_sigma[i], &params[(size_t)i]);
    if (sp.plan.splits > 1) {
      double* pm = (double*)(base + off_part + part_off);
      params[(size_t)i].part_mean = pm;
      params[(size_t)i].part_m2 = pm + (uint64_t)sp.plan.splits * sp.G;
      part_off += sp.partial_bytes;
    }
  }
  if (e == hipSuccess)
    e = hipMemcpy(b->d_scans, params.data(), sizeof(zmc::ScanParams) * params.size(),
                  hipMemcpyHostToDevice);
  if (e == hipSuccess && !bp.tiles.empty())
    e = hipMemcpy(b->d_tiles, bp.tiles.data(), sizeof(zmc::Tile) * bp.tiles.size(),
                  hipMemcpyHostToDevice);
  if (e == hipSuccess && !bp.merge.empty())
    e = hipMemcpy(b->d_merge, bp.merge.data(), sizeof(uint32_t) * bp.merge.size(),
                  hipMemcpyHostToDevice);
  // persistent grid per variant: what the device holds at once, no more
  // blocks than tiles
  for (size_t v = 0; e == hipSuccess && v < b->variants.size(); ++v) {
    Variant& var = b->variants[v];
    int per_cu = 0;
    e = var.key.family < 0          ? zmc::batch_any_occupancy(var.key.precision, &per_cu)
        : var.key.family == ZMC_USER ? zmc::user_batch_occupancy(var.user, &per_cu)
                                     : zmc::batch_occupancy(var.key.precision, var.key.family,
                                                            var.key.N, &per_cu);
    if (per_cu < 1) per_cu = 1;
    const uint64_t want = (uint64_t)cu * (uint64_t)per_cu;
    const uint64_t tiles = var.end - var.begin;
    var.blocks = (unsigned)std::max<uint64_t>(1, std::min(want, tiles));
  }
  if (e != hipSuccess) {
    release(b);
    return fail(ZMC_E_DEVICE, "batch setup failed: %s", hipGetErrorString(e));
  }

  if (b->use_graph) {
    hipStream_t cs = nullptr;
    std::vector<hipStream_t> branches;
    std::vector<hipEvent_t> events;
    e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e == hipSuccess && b->parallel && b->variants.size() > 1) {
      branches.assign(b->variants.size(), nullptr);
      events.assign(b->variants.size() + 1, nullptr);
      for (size_t i = 0; e == hipSuccess && i < branches.size(); ++i)
        e = hipStreamCreateWithFlags(&branches[i], hipStreamNonBlocking);
      for (size_t i = 0; e == hipSuccess && i < events.size(); ++i)
        e = hipEventCreateWithFlags(&events[i], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      hipError_t e_enq = enqueue(b, cs, branches, events);
      hipError_t e_end = hipStreamEndCapture(cs, &b->graph);
      e = e_enq != hipSuccess ? e_enq : e_end;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    for (hipEvent_t ev : events)
      if (ev) (void)hipEventDestroy(ev);
    for (hipStream_t s : branches)
      if (s) (void)hipStreamDestroy(s);
    if (cs) (void)hipStreamDestroy(cs);
    if (e != hipSuccess) {
      release(b);
      return fail(ZMC_E_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
    }
  }
  zmc::log(1, "batch: %d scans, %d variants, %lld tiles, %llu samples, %zu B of device memory, %s",
           n_scans, (int)b->variants.size(), (long long)b->info.tiles,
           (unsigned long long)b->info.samples, total, b->use_graph ? "one graph" : "direct launches");
  *out = b;
  return ok();
}

zmc_status zmc_batch_launch(zmc_batch* b, void* stream) {
  zmc::TraceRange trace_range("zmc_batch_launch");
  if (b == nullptr) return fail(ZMC_E_INVALID, "batch is NULL");
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  if (b->use_graph) {
    e = hipGraphLaunch(b->exec, s);
  } else {
    e = enqueue(b, s, {}, {});
  }
  if (e != hipSuccess) return fail(ZMC_E_DEVICE, "batch launch failed: %s", hipGetErrorString(e));
  return ok();
}

zmc_status zmc_batch_get_info(const zmc_batch* b, zmc_batch_info* info) {
  if (b == nullptr || info == nullptr) return fail(ZMC_E_INVALID, "NULL argument");
  *info = b->info;
  return ok();
}

zmc_status zmc_batch_destroy(zmc_batch* b) {
  if (b == nullptr) return ok();
  hipError_t e = hipDeviceSynchronize();
  release(b);
  if (e != hipSuccess) return fail(ZMC_E_DEVICE, "synchronize failed: %s", hipGetErrorString(e));
  return ok();
}

zmc_status zmc_scan_batch(const zmc_scan_desc* scans, int32_t n_scans,
                          const double* const* d_axis_vals, double* const* d_f,
                          double* const* d_sigma, void* stream) {
  zmc_batch* b = nullptr;
  zmc_status st = zmc_batch_create(scans, n_scans, d_axis_vals, d_f, d_sigma, nullptr, &b);
  if (st != ZMC_OK) return st;
  st = zmc_batch_launch(b, stream);
  hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  zmc_status st2 = zmc_batch_destroy(b);
  if (st != ZMC_OK) return st;
  if (e != hipSuccess) return fail(ZMC_E_DEVICE, "stream synchronize failed: %s", hipGetErrorString(e));
  return st2;
}

const char* zmc_tune_source(void) { return zmc::tune_source(); }

}  // extern "C"
