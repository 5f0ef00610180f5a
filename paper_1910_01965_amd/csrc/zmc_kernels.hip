// zmc_kernels.hip -- the kernels that do not depend on the integrand (split
// merges, counter reset, debug words) and the (family, precision, N) dispatch
// onto the per-family translation units.
#include "zmc_tiles.hpp"

namespace zmc {

// Second pass: merge the split partials of each point in split order.
__global__ __launch_bounds__(256) void k_merge_splits(ScanParams p) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < p.G; g += stride)
    merge_point(p, g);
}

// Zeroes the batch's tile counters (a kernel rather than a memset, so that
// the captured graph holds kernel nodes only).
__global__ void k_reset_counters(uint32_t* counters, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) counters[i] = 0u;
}

// Split merge for every scan of a batch that has more than one sample piece:
// blockIdx.y selects the scan.
__global__ __launch_bounds__(256) void k_merge_batch(const ScanParams* __restrict__ scans,
                                                     const uint32_t* __restrict__ merge_scans) {
  const ScanParams& p = scans[merge_scans[blockIdx.y]];
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < p.G; g += stride)
    merge_point(p, g);
}

__global__ void k_debug_words(uint64_t seed, uint64_t g, uint64_t w0, int64_t count,
                              uint32_t* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const uint64_t w = w0 + (uint64_t)i;
  const Words4 r = philox_block(w >> 2, g, seed);
  const unsigned lane = (unsigned)(w & 3u);
  out[i] = lane == 0 ? r.r[0] : lane == 1 ? r.r[1] : lane == 2 ? r.r[2] : r.r[3];
}

// Calibration load for the VALU counters: eight independent FP32 multiply-add
// chains per lane, 64 multiply-adds per loop trip (the loop control is
// wave-uniform, on the scalar unit), so a full launch keeps every SIMD's VALU
// issue busy.
__global__ __launch_bounds__(256) void k_valu_probe(int64_t iters, float* out) {
  const float b = 0.999f + 1e-9f * (float)(threadIdx.x & 7);
  const float c = 1e-3f;
  float a0 = 1e-3f * (float)threadIdx.x, a1 = a0 + 1.0f, a2 = a0 + 2.0f, a3 = a0 + 3.0f;
  float a4 = a0 + 4.0f, a5 = a0 + 5.0f, a6 = a0 + 6.0f, a7 = a0 + 7.0f;
  for (int64_t i = 0; i != iters; ++i) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      a0 = __builtin_fmaf(a0, b, c);
    a1 = __builtin_fmaf(a1, b, c);
    a2 = __builtin_fmaf(a2, b, c);
    a3 = __builtin_fmaf(a3, b, c);
    a4 = __builtin_fmaf(a4, b, c);
    a5 = __builtin_fmaf(a5, b, c);
    a6 = __builtin_fmaf(a6, b, c);
      a7 = __builtin_fmaf(a7, b, c);
    }
  }
  out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = ((a0 + a1) + (a2 + a3)) + ((a4 + a5) + (a6 + a7));
}

namespace {

template <typename T, class Fn>
hipError_t by_family(int family, const Fn& fn) {
  switch (family) {
    case ZMC_SIN_SUM: return fn(FamilyOps<SinSum, T>{});
    case ZMC_GAUSS: return fn(FamilyOps<Gauss, T>{});
    case ZMC_COSEXP: return fn(FamilyOps<CosExp, T>{});
    case ZMC_CONST: return fn(FamilyOps<Const, T>{});
    case ZMC_LINEAR: return fn(FamilyOps<Linear, T>{});
    default: return hipErrorInvalidValue;
  }
}

template <class Fn>
hipError_t by_precision(int precision, int family, const Fn& fn) {
  if (precision == ZMC_FP64) return by_family<double>(family, fn);
  return by_family<float>(family, fn);
}

}  // namespace

hipError_t launch_scan(const ScanParams& p, const Plan& plan, int precision, hipStream_t stream,
                       hipEvent_t ev_begin, hipEvent_t ev_end) {
  hipError_t e = hipSuccess;
  if (ev_begin != nullptr) e = hipEventRecord(ev_begin, stream);
  if (e == hipSuccess)
    e = by_precision(precision, p.family, [&](auto ops) { return ops.main(p.N, p, plan, stream); });
  if (e == hipSuccess && ev_end != nullptr) e = hipEventRecord(ev_end, stream);
  if (e != hipSuccess || p.splits == 1) return e;
  return launch_merge_splits(p, stream);
}

hipError_t launch_merge_splits(const ScanParams& p, hipStream_t stream) {
  uint64_t blocks = (p.G + 255) / 256;
  if (blocks > (1u << 20)) blocks = 1u << 20;
  hipLaunchKernelGGL(k_merge_splits, dim3((unsigned)blocks), dim3(256), 0, stream, p);
  return hipGetLastError();
}

hipError_t batch_occupancy(int precision, int family, int N, int* blocks_per_cu) {
  return by_precision(precision, family, [&](auto ops) { return ops.occupancy(N, blocks_per_cu); });
}

hipError_t launch_batch_variant(int precision, int family, int N, const ScanParams* scans,
                                const Tile* tiles, uint32_t begin, uint32_t end,
                                uint32_t* counter, unsigned blocks, hipStream_t stream) {
  return by_precision(precision, family, [&](auto ops) {
    return ops.batch(N, scans, tiles, begin, end, counter, blocks, stream);
  });
}

hipError_t batch_any_occupancy(int precision, int* blocks_per_cu) {
  if (precision == ZMC_FP64) return AnyOps<double>::occupancy(blocks_per_cu);
  return AnyOps<float>::occupancy(blocks_per_cu);
}

hipError_t launch_batch_any(int precision, const ScanParams* scans, const Tile* tiles,
                            uint32_t begin, uint32_t end, uint32_t* counter, unsigned blocks,
                            hipStream_t stream) {
  if (precision == ZMC_FP64) return AnyOps<double>::batch(scans, tiles, begin, end, counter, blocks, stream);
  return AnyOps<float>::batch(scans, tiles, begin, end, counter, blocks, stream);
}

hipError_t launch_reset_counters(uint32_t* counters, int n, hipStream_t stream) {
  hipLaunchKernelGGL(k_reset_counters, dim3(1), dim3(256), 0, stream, counters, n);
  return hipGetLastError();
}

hipError_t launch_merge_batch(const ScanParams* scans, const uint32_t* merge_scans, int n_merge,
                              uint64_t max_points, hipStream_t stream) {
  if (n_merge <= 0) return hipSuccess;
  uint64_t bx = (max_points + 255) / 256;
  if (bx > 4096) bx = 4096;
  hipLaunchKernelGGL(k_merge_batch, dim3((unsigned)bx, (unsigned)n_merge), dim3(256), 0, stream,
                     scans, merge_scans);
  return hipGetLastError();
}

hipError_t launch_debug_words(uint64_t seed, uint64_t g, uint64_t w0, int64_t count,
                              uint32_t* out, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_debug_words, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, stream,
                     seed, g, w0, count, out);
  return hipGetLastError();
}

hipError_t launch_valu_probe(int32_t blocks, int64_t iters, float* out, hipStream_t stream) {
  hipLaunchKernelGGL(k_valu_probe, dim3((unsigned)blocks), dim3(256), 0, stream, iters, out);
  return hipGetLastError();
}

hipError_t launch_debug_values(const ScanParams& p, int precision, uint64_t g, uint64_t s0,
                               int64_t count, double* out, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  return by_precision(precision, p.family,
                      [&](auto ops) { return ops.values(p.N, p, g, s0, count, out, stream); });
}

}  // namespace zmc
