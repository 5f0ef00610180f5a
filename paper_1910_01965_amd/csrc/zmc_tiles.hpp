// zmc_tiles.hpp -- the compiled-in scan kernels for gfx950 (templates over
// the integrand family, working precision and dimension) and the per-family
// launchers that each family translation unit instantiates.  The loops they
// run are in zmc_scan.hpp.
#pragma once

#include "zmc_internal.hpp"
#include "zmc_scan.hpp"

namespace zmc {

// Waves per SIMD asked of the point-major and batch kernels.  FP32 with
// 4 <= N <= 8 runs faster at 8 (the compiler then keeps 64 VGPRs and spills a
// few set-up values); at N <= 3, in FP64, and for N > 8 (where 64 VGPRs
// would spill the per-point constants of every sample) its own choice is
// taken.
template <typename T, int N>
constexpr int kMinWaves = (sizeof(T) == 4 && N >= 4 && N <= kAnyMaxDims) ? 8 : 1;

template <class Fam, typename T, int N>
__global__ __launch_bounds__(256, (kMinWaves<T, N>)) void k_point_major(ScanParams p) {
  point_major_body<Fam, T, N>(p);
}

// Threads per sample-major block: up to 1024, or 256 for N > kAnyMaxDims,
// whose per-point constants and variates need more than the 128 VGPRs that a
// 1024-thread block leaves each lane.
template <int N> constexpr int kSmMaxThreads = N > kAnyMaxDims ? 256 : 1024;

template <class Fam, typename T, int N>
__global__ __launch_bounds__(kSmMaxThreads<N>) void k_sample_major(ScanParams p) {
  __shared__ double lds[48];
  sample_major_body<Fam, T, N>(p, lds);
}

// Batched scans: a persistent kernel per (family, precision, N) variant.  Its
// blocks pop tiles [begin, end) of the batch's tile table through one atomic
// counter (tiles are sorted longest first) and exit once the table is
// exhausted; every block reaches that exit.
template <class Fam, typename T, int N>
__global__ __launch_bounds__(256, (kMinWaves<T, N>)) void k_batch(const ScanParams* __restrict__ scans,
                                               const Tile* __restrict__ tiles, uint32_t begin,
                                               uint32_t end, uint32_t* counter) {
  __shared__ uint32_t next;
  __shared__ double lds[48];
  batch_body<Fam, T, N>(scans, tiles, begin, end, counter, &next, lds);
}

// One tile of any family with N <= kAnyMaxDims in working precision T: the
// switch picks the template instance from the scan's own (family, N).  Scans
// of more dimensions run in their own per-variant kernels (k_batch), so that
// this kernel's register use stays that of its N <= 8 branches.
template <typename T>
__device__ __forceinline__ void run_tile_any(const ScanParams& p, const Tile& tl, double* lds) {
  const uint64_t sp = tl.split_mode & ~kTileSampleMajor;
  const bool sm = (tl.split_mode & kTileSampleMajor) != 0;
#define ZMC_TILE_CASE(FAM, NN)                                  \
  case FAM##_ID * 32 + NN:                                      \
    if (sm)                                                     \
      sm_tile<FAM<T, NN>, T, NN>(p, tl.first, sp, lds);         \
    else                                                        \
      pm_tile<FAM<T, NN>, T, NN>(p, tl.first, sp);              \
    break;
#define ZMC_TILE_CASES(FAM)                                                                  \
  ZMC_TILE_CASE(FAM, 1) ZMC_TILE_CASE(FAM, 2) ZMC_TILE_CASE(FAM, 3) ZMC_TILE_CASE(FAM, 4) \
  ZMC_TILE_CASE(FAM, 5) ZMC_TILE_CASE(FAM, 6) ZMC_TILE_CASE(FAM, 7) ZMC_TILE_CASE(FAM, 8)
  constexpr int SinSum_ID = ZMC_SIN_SUM, Gauss_ID = ZMC_GAUSS, Const_ID = ZMC_CONST,
                Linear_ID = ZMC_LINEAR, CosExp_ID = ZMC_COSEXP;
  static_assert(kAnyMaxDims == 8 && kMaxDims < 32, "the cases list N = 1..8");
  switch (p.family * 32 + p.N) {
    ZMC_TILE_CASES(SinSum)
    ZMC_TILE_CASES(Gauss)
    ZMC_TILE_CASES(Const)
    ZMC_TILE_CASES(Linear)
    ZMC_TILE_CASE(CosExp, 2) ZMC_TILE_CASE(CosExp, 3) ZMC_TILE_CASE(CosExp, 4)
    ZMC_TILE_CASE(CosExp, 5) ZMC_TILE_CASE(CosExp, 6) ZMC_TILE_CASE(CosExp, 7)
    ZMC_TILE_CASE(CosExp, 8)
    default:
      break;
  }
#undef ZMC_TILE_CASES
#undef ZMC_TILE_CASE
}

// Batched scans, one kernel for every family (N <= kAnyMaxDims) of one
// working precision: the blocks pop tiles of all scans from one queue.
template <typename T>
__global__ __launch_bounds__(256) void k_batch_any(const ScanParams* __restrict__ scans,
                                                   const Tile* __restrict__ tiles, uint32_t begin,
                                                   uint32_t end, uint32_t* counter) {
  __shared__ uint32_t next;
  __shared__ double lds[48];
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) next = begin + atomicAdd(counter, 1u);
    __syncthreads();
    const uint32_t t = next;
    if (t >= end) break;
    const Tile tl = tiles[t];
    run_tile_any<T>(scans[tl.scan], tl, lds);
  }
}

template <class Fam, typename T, int N>
__global__ void k_debug_values(ScanParams p, uint64_t g, uint64_t s0, int64_t count,
                               double* out) {
  debug_values_body<Fam, T, N>(p, g, s0, count, out);
}

// ---------------------------------------------------------------------------
// Launchers of one family F in working precision T for N = Lo .. Lo + 7
// (Lo = 1 or 9); each (family, precision, N range) triple is instantiated in
// its own translation unit.
// ---------------------------------------------------------------------------
constexpr int kDimsPerUnit = 8;

template <template <typename, int> class F, typename T, int Lo>
struct FamilyOps {
  template <int N>
  static hipError_t main_n(const ScanParams& p, const Plan& plan, hipStream_t stream) {
    const dim3 block((unsigned)plan.block);
    const dim3 grid((unsigned)plan.grid_x, (unsigned)plan.splits);
    if (plan.mode == ZMC_MODE_POINT_MAJOR) {
      hipLaunchKernelGGL((k_point_major<F<T, N>, T, N>), grid, block, 0, stream, p);
    } else {
      hipLaunchKernelGGL((k_sample_major<F<T, N>, T, N>), grid, block, 0, stream, p);
    }
    return hipGetLastError();
  }
  template <int N>
  static hipError_t values_n(const ScanParams& p, uint64_t g, uint64_t s0, int64_t count,
                             double* out, hipStream_t stream) {
    const unsigned blocks = (unsigned)((count + 255) / 256);
    hipLaunchKernelGGL((k_debug_values<F<T, N>, T, N>), dim3(blocks), dim3(256), 0, stream, p, g,
                       s0, count, out);
    return hipGetLastError();
  }
  template <int N>
  static hipError_t occupancy_n(int* blocks_per_cu) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_batch<F<T, N>, T, N>, 256, 0);
  }
  template <int N>
  static hipError_t batch_n(const ScanParams* scans, const Tile* tiles, uint32_t begin,
                            uint32_t end, uint32_t* counter, unsigned blocks, hipStream_t stream) {
    hipLaunchKernelGGL((k_batch<F<T, N>, T, N>), dim3(blocks), dim3(256), 0, stream, scans, tiles,
                       begin, end, counter);
    return hipGetLastError();
  }

  // Dispatch on N.  Defined out of line (not inline), so that the explicit
  // instantiation declarations below keep every other translation unit from
  // instantiating the kernels again.
  static hipError_t main(int N, const ScanParams& p, const Plan& plan, hipStream_t stream);
  static hipError_t values(int N, const ScanParams& p, uint64_t g, uint64_t s0, int64_t count,
                           double* out, hipStream_t stream);
  static hipError_t occupancy(int N, int* blocks_per_cu);
  static hipError_t batch(int N, const ScanParams* scans, const Tile* tiles, uint32_t begin,
                          uint32_t end, uint32_t* counter, unsigned blocks, hipStream_t stream);
};

// Instances below a family's smallest N (COSEXP needs two dimensions) are
// never built; validation rejects those descriptors before dispatch.
#define ZMC_BY_DIMS(CALL)                                                                 \
  switch (N - Lo) {                                                                       \
    case 0: if constexpr (Lo >= F<T, Lo>::kMinDims) return CALL(Lo); else break;          \
    case 1: return CALL(Lo + 1);                                                          \
    case 2: return CALL(Lo + 2);                                                          \
    case 3: return CALL(Lo + 3);                                                          \
    case 4: return CALL(Lo + 4);                                                          \
    case 5: return CALL(Lo + 5);                                                          \
    case 6: return CALL(Lo + 6);                                                          \
    case 7: return CALL(Lo + 7);                                                          \
    default: break;                                                                       \
  }                                                                                       \
  return hipErrorInvalidValue;
static_assert(kDimsPerUnit == 8, "ZMC_BY_DIMS lists eight dimensions");

template <template <typename, int> class F, typename T, int Lo>
hipError_t FamilyOps<F, T, Lo>::main(int N, const ScanParams& p, const Plan& plan, hipStream_t stream) {
#define ZMC_CALL(NN) main_n<NN>(p, plan, stream)
  ZMC_BY_DIMS(ZMC_CALL)
#undef ZMC_CALL
}

template <template <typename, int> class F, typename T, int Lo>
hipError_t FamilyOps<F, T, Lo>::values(int N, const ScanParams& p, uint64_t g, uint64_t s0,
                                       int64_t count, double* out, hipStream_t stream) {
#define ZMC_CALL(NN) values_n<NN>(p, g, s0, count, out, stream)
  ZMC_BY_DIMS(ZMC_CALL)
#undef ZMC_CALL
}

template <template <typename, int> class F, typename T, int Lo>
hipError_t FamilyOps<F, T, Lo>::occupancy(int N, int* blocks_per_cu) {
#define ZMC_CALL(NN) occupancy_n<NN>(blocks_per_cu)
  ZMC_BY_DIMS(ZMC_CALL)
#undef ZMC_CALL
}

template <template <typename, int> class F, typename T, int Lo>
hipError_t FamilyOps<F, T, Lo>::batch(int N, const ScanParams* scans, const Tile* tiles,
                                      uint32_t begin, uint32_t end, uint32_t* counter,
                                      unsigned blocks, hipStream_t stream) {
#define ZMC_CALL(NN) batch_n<NN>(scans, tiles, begin, end, counter, blocks, stream)
  ZMC_BY_DIMS(ZMC_CALL)
#undef ZMC_CALL
}
#undef ZMC_BY_DIMS

// Launchers of the any-family batch kernel in working precision T.
template <typename T>
struct AnyOps {
  static hipError_t occupancy(int* blocks_per_cu);
  static hipError_t batch(const ScanParams* scans, const Tile* tiles, uint32_t begin, uint32_t end,
                          uint32_t* counter, unsigned blocks, hipStream_t stream);
};

template <typename T>
hipError_t AnyOps<T>::occupancy(int* blocks_per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_batch_any<T>, 256, 0);
}

template <typename T>
hipError_t AnyOps<T>::batch(const ScanParams* scans, const Tile* tiles, uint32_t begin,
                            uint32_t end, uint32_t* counter, unsigned blocks, hipStream_t stream) {
  hipLaunchKernelGGL(k_batch_any<T>, dim3(blocks), dim3(256), 0, stream, scans, tiles, begin, end,
                     counter);
  return hipGetLastError();
}

#define ZMC_DECLARE_FAMILY_OPS(F)                                \
  extern template struct FamilyOps<F, float, 1>;                 \
  extern template struct FamilyOps<F, double, 1>;                \
  extern template struct FamilyOps<F, float, 1 + kDimsPerUnit>;  \
  extern template struct FamilyOps<F, double, 1 + kDimsPerUnit>;
ZMC_DECLARE_FAMILY_OPS(SinSum)
ZMC_DECLARE_FAMILY_OPS(Gauss)
ZMC_DECLARE_FAMILY_OPS(CosExp)
ZMC_DECLARE_FAMILY_OPS(Const)
ZMC_DECLARE_FAMILY_OPS(Linear)
#undef ZMC_DECLARE_FAMILY_OPS
extern template struct AnyOps<float>;
extern template struct AnyOps<double>;

}  // namespace zmc
