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

// Instruction-rate loads for the roofline's op mix: each lane runs eight
// dependent chains of one instruction form, 64 instructions per loop trip
// (loop control on the scalar unit), every step reading two or three chains
// so that nothing folds.  The forms are those the scan kernels issue: two-operand
// xor and add, three-operand FP32 fma, the 32x32->64 multiply-add and the
// three-input xor of Philox, the FP32 exp2 and sine units, and FP64 fma.
template <int Op> struct RateOp;
// xor steps alternate with integer adds (both two-operand forms), since a
// chain of xors alone is linear and the compiler folds it
template <> struct RateOp<ZMC_RATE_XOR_B32> {
  using V = uint32_t;
  static __device__ V init(unsigned t, int i) { return 0x9E3779B9u * (t + 1u) + (V)i; }
  static __device__ __forceinline__ V step(V a, V b, V, int u) { return (u & 1) ? a + b : a ^ b; }
};
template <> struct RateOp<ZMC_RATE_ADD_F32> {
  using V = float;
  static __device__ V init(unsigned t, int i) { return 1e-3f * (float)t + (float)i; }
  static __device__ __forceinline__ V step(V a, V b, V, int) { return a + b; }
};
template <> struct RateOp<ZMC_RATE_FMA_F32> {
  using V = float;
  static __device__ V init(unsigned t, int i) { return 1.0f + 1e-6f * (float)t + 1e-3f * (float)i; }
  static __device__ __forceinline__ V step(V a, V b, V c, int) { return __builtin_fmaf(a, b, c); }
};
template <> struct RateOp<ZMC_RATE_MAD_U64_U32> {
  using V = uint64_t;
  static __device__ V init(unsigned t, int i) { return 0xD2511F53ull * (t + 1u) + (V)i; }
  static __device__ __forceinline__ V step(V a, V b, V c, int) {
    return (uint64_t)(uint32_t)a * (uint32_t)b + c;
  }
};
template <> struct RateOp<ZMC_RATE_BITOP3_B32> {
  using V = uint32_t;
  static __device__ V init(unsigned t, int i) { return 0xCD9E8D57u * (t + 1u) + (V)i; }
  static __device__ __forceinline__ V step(V a, V b, V c, int) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
  }
};
template <> struct RateOp<ZMC_RATE_EXP_F32> {
  using V = float;
  static __device__ V init(unsigned t, int i) { return 1e-4f * (float)t + 0.1f * (float)i; }
  static __device__ __forceinline__ V step(V a, V, V, int) { return __builtin_amdgcn_exp2f(-a); }
};
template <> struct RateOp<ZMC_RATE_SIN_F32> {
  using V = float;
  static __device__ V init(unsigned t, int i) { return 1e-4f * (float)t + 0.1f * (float)i; }
  static __device__ __forceinline__ V step(V a, V, V, int) { return __builtin_amdgcn_sinf(a); }
};
template <> struct RateOp<ZMC_RATE_FMA_F64> {
  using V = double;
  static __device__ V init(unsigned t, int i) { return 1.0 + 1e-9 * (double)t + 1e-3 * (double)i; }
  static __device__ __forceinline__ V step(V a, V b, V c, int) { return __builtin_fma(a, b, c); }
};

template <int Op>
__global__ __launch_bounds__(256) void k_rate_probe(int64_t iters, uint64_t* out) {
  using R = RateOp<Op>;
  typename R::V x[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) x[i] = R::init(threadIdx.x, i);
  for (int64_t it = 0; it != iters; ++it) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
#pragma unroll
      for (int i = 0; i < 8; ++i) x[i] = R::step(x[i], x[(i + 1) & 7], x[(i + 2) & 7], u);
    }
  }
  uint64_t h = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    uint64_t bits = 0;
    __builtin_memcpy(&bits, &x[i], sizeof(x[i]));
    h ^= bits + (uint64_t)i;
  }
  out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = h;
}

namespace {

template <typename T, int Lo, class Fn>
hipError_t by_family(int family, const Fn& fn) {
  switch (family) {
    case ZMC_SIN_SUM: return fn(FamilyOps<SinSum, T, Lo>{});
    case ZMC_GAUSS: return fn(FamilyOps<Gauss, T, Lo>{});
    case ZMC_COSEXP: return fn(FamilyOps<CosExp, T, Lo>{});
    case ZMC_CONST: return fn(FamilyOps<Const, T, Lo>{});
    case ZMC_LINEAR: return fn(FamilyOps<Linear, T, Lo>{});
    default: return hipErrorInvalidValue;
  }
}

// N = 1..8 and 9..16 are built in separate translation units.
template <class Fn>
hipError_t by_precision(int precision, int family, int N, const Fn& fn) {
  constexpr int Wide = 1 + kDimsPerUnit;
  if (precision == ZMC_FP64)
    return N < Wide ? by_family<double, 1>(family, fn) : by_family<double, Wide>(family, fn);
  return N < Wide ? by_family<float, 1>(family, fn) : by_family<float, Wide>(family, fn);
}

}  // namespace

hipError_t launch_scan(const ScanParams& p, const Plan& plan, int precision, hipStream_t stream,
                       hipEvent_t ev_begin, hipEvent_t ev_end) {
  hipError_t e = hipSuccess;
  if (ev_begin != nullptr) e = hipEventRecord(ev_begin, stream);
  if (e == hipSuccess)
    e = by_precision(precision, p.family, p.N, [&](auto ops) { return ops.main(p.N, p, plan, stream); });
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
  return by_precision(precision, family, N, [&](auto ops) { return ops.occupancy(N, blocks_per_cu); });
}

hipError_t launch_batch_variant(int precision, int family, int N, const ScanParams* scans,
                                const Tile* tiles, uint32_t begin, uint32_t end,
                                uint32_t* counter, unsigned blocks, hipStream_t stream) {
  return by_precision(precision, family, N, [&](auto ops) {
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
  return by_precision(precision, p.family, p.N,
                      [&](auto ops) { return ops.values(p.N, p, g, s0, count, out, stream); });
}

hipError_t launch_rate_probe(int32_t op, int32_t blocks, int64_t iters, uint64_t* out,
                             hipStream_t stream) {
  const dim3 grid((unsigned)blocks), block(256);
  switch (op) {
    case ZMC_RATE_XOR_B32: hipLaunchKernelGGL(k_rate_probe<ZMC_RATE_XOR_B32>, grid, block, 0, stream, iters, out); break;
    case ZMC_RATE_ADD_F32: hipLaunchKernelGGL(k_rate_probe<ZMC_RATE_ADD_F32>, grid, block, 0, stream, iters, out); break;
    case ZMC_RATE_FMA_F32: hipLaunchKernelGGL(k_rate_probe<ZMC_RATE_FMA_F32>, grid, block, 0, stream, iters, out); break;
    case ZMC_RATE_MAD_U64_U32: hipLaunchKernelGGL(k_rate_probe<ZMC_RATE_MAD_U64_U32>, grid, block, 0, stream, iters, out); break;
    case ZMC_RATE_BITOP3_B32: hipLaunchKernelGGL(k_rate_probe<ZMC_RATE_BITOP3_B32>, grid, block, 0, stream, iters, out); break;
    case ZMC_RATE_EXP_F32: hipLaunchKernelGGL(k_rate_probe<ZMC_RATE_EXP_F32>, grid, block, 0, stream, iters, out); break;
    case ZMC_RATE_SIN_F32: hipLaunchKernelGGL(k_rate_probe<ZMC_RATE_SIN_F32>, grid, block, 0, stream, iters, out); break;
    case ZMC_RATE_FMA_F64: hipLaunchKernelGGL(k_rate_probe<ZMC_RATE_FMA_F64>, grid, block, 0, stream, iters, out); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace zmc
