// zmc_internal.hpp -- declarations shared by the host API and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "zmc.h"

namespace zmc {

struct ScanParams;

// A work decomposition (see zmc_plan_info in zmc.h).
struct Plan {
  int mode;             // ZMC_MODE_POINT_MAJOR or ZMC_MODE_SAMPLE_MAJOR
  int block;            // threads per block
  int splits;           // sample-range pieces per point
  uint64_t groups;      // ceil(n / 4)
  uint64_t gps;         // groups per piece
  uint64_t grid_x;      // blocks along x (point blocks or points, capped)
  uint64_t point_blocks;
  uint64_t workspace_bytes;
};

hipError_t launch_scan(const ScanParams& p, const Plan& plan, int precision, hipStream_t stream,
                       hipEvent_t ev_begin, hipEvent_t ev_end);
struct Tile;

// Diagnostics on stderr, prefixed "[zmc] ", when the environment variable
// ZMC_LOG is at least `level` (1: set-up events such as tune-table loads,
// batch and server creation, run-time compiles; 2: also every plan and every
// server admission and completion).  The level is read once per process.
int log_level();
void log(int level, const char* fmt, ...) __attribute__((format(printf, 2, 3)));

// Host helpers shared by the single-scan and the batched entry points.
zmc_status fail(zmc_status st, const char* fmt, ...);
zmc_status ok();
zmc_status validate_desc(const zmc_scan_desc* d, uint64_t* G);
zmc_status check_pieces(uint64_t groups, uint64_t gps, uint64_t splits);
zmc_status cu_count(int* cu);
void fill_scan_params(const zmc_scan_desc* d, uint64_t G, const Plan& pl, const double* d_axis,
                      double* d_f, double* d_sigma, ScanParams* p);

// Tuned tile shapes of one kernel variant (family, precision, N).
struct TuneEntry {
  int64_t pm_groups;      // groups of four samples per lane in a point-major tile
  int64_t sm_groups;      // groups per sample-major tile (all lanes of the block)
  int64_t pm_min_points;  // grids smaller than this use sample-major tiles
};
TuneEntry tune_lookup(int family, int precision, int N);

constexpr int kTileBlock = 256;
constexpr uint64_t kMaxPartialBytesPerScan = (uint64_t)2 << 30;
zmc_status plan_tiles(const zmc_scan_desc* d, uint64_t G, int64_t pm_groups_override,
                      int64_t sm_groups_override, int64_t pm_min_override, Plan* pl,
                      uint64_t* tiles);
const char* tune_source();
hipError_t batch_occupancy(int precision, int family, int N, int* blocks_per_cu);
hipError_t launch_batch_variant(int precision, int family, int N, const ScanParams* scans,
                                const Tile* tiles, uint32_t begin, uint32_t end,
                                uint32_t* counter, unsigned blocks, hipStream_t stream);
hipError_t batch_any_occupancy(int precision, int* blocks_per_cu);
hipError_t launch_batch_any(int precision, const ScanParams* scans, const Tile* tiles,
                            uint32_t begin, uint32_t end, uint32_t* counter, unsigned blocks,
                            hipStream_t stream);
hipError_t launch_reset_counters(uint32_t* counters, int n, hipStream_t stream);
hipError_t launch_merge_batch(const ScanParams* scans, const uint32_t* merge_scans, int n_merge,
                              uint64_t max_points, hipStream_t stream);
hipError_t launch_debug_words(uint64_t seed, uint64_t g, uint64_t w0, int64_t count,
                              uint32_t* out, hipStream_t stream);
hipError_t launch_merge_splits(const ScanParams& p, hipStream_t stream);
hipError_t launch_valu_probe(int32_t blocks, int64_t iters, float* out, hipStream_t stream);
hipError_t launch_rate_probe(int32_t op, int32_t blocks, int64_t iters, uint64_t* out,
                             hipStream_t stream);

// Kernels of a user integrand for one (precision, N, M), built on first use.
struct UserKernels {
  hipFunction_t pm = nullptr, sm = nullptr, values = nullptr, batch = nullptr;
};
zmc_status user_kernels(const zmc_integrand* h, int precision, int N, int M, UserKernels* out);
hipError_t launch_user_scan(const UserKernels& k, const ScanParams& p, const Plan& plan,
                            hipStream_t stream, hipEvent_t ev_begin, hipEvent_t ev_end);
hipError_t launch_user_values(const UserKernels& k, const ScanParams& p, uint64_t g, uint64_t s0,
                              int64_t count, double* out, hipStream_t stream);
hipError_t user_batch_occupancy(const UserKernels& k, int* blocks_per_cu);
hipError_t launch_user_batch(const UserKernels& k, const ScanParams* scans, const Tile* tiles,
                             uint32_t begin, uint32_t end, uint32_t* counter, unsigned blocks,
                             hipStream_t stream);
hipError_t launch_debug_values(const ScanParams& p, int precision, uint64_t g, uint64_t s0,
                               int64_t count, double* out, hipStream_t stream);

}  // namespace zmc
