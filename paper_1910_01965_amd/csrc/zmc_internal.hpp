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
hipError_t launch_debug_words(uint64_t seed, uint64_t g, uint64_t w0, int64_t count,
                              uint32_t* out, hipStream_t stream);
hipError_t launch_debug_values(const ScanParams& p, int precision, uint64_t g, uint64_t s0,
                               int64_t count, double* out, hipStream_t stream);

}  // namespace zmc
