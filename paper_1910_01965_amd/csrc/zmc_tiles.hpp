// zmc_tiles.hpp -- the scan kernels for gfx950 (templates) and the per-family
// launchers that each family translation unit instantiates.
//
// Point-major kernel: a lane owns one grid point and all lanes of a wave walk
// the same groups of four samples in step, so the Philox counter words that
// depend only on the sample index (the word block b) are wave-uniform and
// live in scalar registers; only the grid-index half of the counter differs
// between lanes.  A point's sample range may be cut into `splits` pieces run
// by different blocks; their FP64 partials are merged by a second pass.
//
// Sample-major kernel: a block owns one grid point and its lanes share the
// samples (lane t takes groups t, t+T, ...); lane sums are merged over the
// wave by a shuffle butterfly, then over the block's waves through LDS, then
// (for several blocks per point) by the same second pass.
//
// Method: direct Monte Carlo per grid point, ZMCintegral-v5 Sec. 2, Eq. (1);
// the paper gives each point to one GPU thread (Sec. 2, Fig. 1), which is the
// point-major kernel without splits.
#pragma once

#include "zmc_device.hpp"
#include "zmc_internal.hpp"

namespace zmc {


// Groups j0 .. jfull-1 in full, then (when `ragged`) the scan's short last
// group; every lane of the wave walks the same j.
// The lane's sums are shifted by its first sample, so that the final
// M2 = S2 - S1^2 / n does not cancel even when the samples are close to each
// other and far from the integrand's typical value.
template <class Fam, typename T, int N, class Gen>
__device__ __forceinline__ void lane_groups(const Fam& fam, const Gen& gen, uint64_t j0,
                                            uint64_t jfull, bool ragged, int tail,
                                            LaneAcc<T>& acc) {
  uint64_t j = j0;
  if (j < jfull) {
    T v[4];
    eval_group<Fam, T, N>(fam, j, gen, v);
    acc.init(v[0]);
    acc.add4(v);
    ++j;
  }
  for (; j < jfull; ++j) {
    T v[4];
    eval_group<Fam, T, N>(fam, j, gen, v);
    acc.add4(v);
  }
  if (ragged) {
    T v[4];
    eval_group<Fam, T, N>(fam, jfull, gen, v);
    if (jfull == j0) acc.init(v[0]);
    acc.add_partial(v, tail);
  }
}

// One point-major tile: the block's lanes take grid points first,
// first + 1, ... (one each) over sample piece sp.
template <class Fam, typename T, int N>
__device__ __forceinline__ void pm_tile(const ScanParams& p, uint64_t first, uint64_t sp) {
  const uint64_t j0 = sp * p.gps;
  const uint64_t j1 = (j0 + p.gps < p.n_groups) ? j0 + p.gps : p.n_groups;
  const bool ragged = (j1 == p.n_groups) && ((p.n & 3u) != 0);
  const uint64_t jfull = ragged ? j1 - 1 : j1;
  const int tail = (int)(p.n - 4 * (p.n_groups - 1));
  const uint64_t g = first + threadIdx.x;
  if (g >= p.G) return;
  Fam fam;
  fam.setup(p, g);
  LaneAcc<T> acc;
  acc.init((T)0);
  with_form(fam, [&](const auto& f) {
    using F = std::decay_t<decltype(f)>;
    if (p.fast_counter) {
      const GenPointMajor gen{philox_lane((uint32_t)g, p.seed)};
      lane_groups<F, T, N>(f, gen, j0, jfull, ragged, tail, acc);
    } else {
      const GenAny gen{g, p.seed};
      lane_groups<F, T, N>(f, gen, j0, jfull, ragged, tail, acc);
    }
  });
  const Moments m = to_moments(acc, (double)split_samples(p.n, p.n_groups, p.gps, sp));
  if (p.splits == 1) {
    finalize(p, g, m);
  } else {
    p.part_mean[sp * p.G + g] = m.mean;
    p.part_m2[sp * p.G + g] = m.m2;
  }
}

// One sample-major tile: the whole block works on grid point g over sample
// piece sp (lane t takes groups j0 + t, j0 + t + T, ...), then merges its
// lanes.  Every thread of the block must call it (it synchronises); `lds`
// holds 3 x 16 doubles.
template <class Fam, typename T, int N>
__device__ __forceinline__ void sm_tile(const ScanParams& p, uint64_t g, uint64_t sp, double* lds) {
  const uint64_t j0 = sp * p.gps;
  const uint64_t j1 = (j0 + p.gps < p.n_groups) ? j0 + p.gps : p.n_groups;
  const uint64_t last = p.n_groups - 1;
  const int tail = (int)(p.n - 4 * last);  // samples in the scan's last group
  const unsigned waves = blockDim.x >> 6;
  Fam fam;
  fam.setup(p, g);
  LaneAcc<T> acc;
  acc.init((T)0);
  double count = 0.0;
  const GenAny gen{g, p.seed};
  with_form(fam, [&](const auto& f) {
    using F = std::decay_t<decltype(f)>;
    for (uint64_t j = j0 + threadIdx.x; j < j1; j += blockDim.x) {
      T v[4];
      eval_group<F, T, N>(f, j, gen, v);
      if (count == 0.0) acc.init(v[0]);  // shift by the lane's first sample
      if (j == last && tail != 4) {
        acc.add_partial(v, tail);
        count += (double)tail;
      } else {
        acc.add4(v);
        count += 4.0;
      }
    }
  });
  Moments m = wave_merge(to_moments(acc, count));
  const unsigned w = threadIdx.x >> 6;
  if ((threadIdx.x & 63u) == 0) {
    lds[w] = m.n;
    lds[16 + w] = m.mean;
    lds[32 + w] = m.m2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    Moments t{lds[0], lds[16], lds[32]};
    for (unsigned i = 1; i < waves; ++i) t = merge(t, Moments{lds[i], lds[16 + i], lds[32 + i]});
    if (p.splits == 1) {
      finalize(p, g, t);
    } else {
      p.part_mean[sp * p.G + g] = t.mean;
      p.part_m2[sp * p.G + g] = t.m2;
    }
  }
  __syncthreads();
}

// Merge of point g's split partials in split order, then f and sigma.
__device__ __forceinline__ void merge_point(const ScanParams& p, uint64_t g) {
  Moments t{(double)split_samples(p.n, p.n_groups, p.gps, 0), p.part_mean[g], p.part_m2[g]};
  for (int sp = 1; sp < p.splits; ++sp) {
    const Moments b{(double)split_samples(p.n, p.n_groups, p.gps, (uint64_t)sp),
                    p.part_mean[(uint64_t)sp * p.G + g], p.part_m2[(uint64_t)sp * p.G + g]};
    t = merge(t, b);
  }
  finalize(p, g, t);
}

template <class Fam, typename T, int N>
__global__ __launch_bounds__(256) void k_point_major(ScanParams p) {
  for (uint64_t pb = blockIdx.x; pb < p.point_blocks; pb += gridDim.x)
    pm_tile<Fam, T, N>(p, pb * blockDim.x, blockIdx.y);
}

template <class Fam, typename T, int N>
__global__ __launch_bounds__(1024) void k_sample_major(ScanParams p) {
  __shared__ double lds[48];
  for (uint64_t g = blockIdx.x; g < p.G; g += gridDim.x) sm_tile<Fam, T, N>(p, g, blockIdx.y, lds);
}

// Batched scans: a persistent kernel per (family, precision, N) variant.  Its
// blocks pop tiles [begin, end) of the batch's tile table through one atomic
// counter (tiles are sorted longest first) and exit once the table is
// exhausted; every block reaches that exit.
template <class Fam, typename T, int N>
__global__ __launch_bounds__(256) void k_batch(const ScanParams* __restrict__ scans,
                                               const Tile* __restrict__ tiles, uint32_t begin,
                                               uint32_t end, uint32_t* counter) {
  __shared__ uint32_t next;
  __shared__ double lds[48];
  for (;;) {
    __syncthreads();  // the previous tile is done with `next` and `lds`
    if (threadIdx.x == 0) next = begin + atomicAdd(counter, 1u);
    __syncthreads();
    const uint32_t t = next;
    if (t >= end) break;
    const Tile tl = tiles[t];
    const ScanParams& p = scans[tl.scan];
    const uint64_t sp = tl.split_mode & ~kTileSampleMajor;
    if (tl.split_mode & kTileSampleMajor) {
      sm_tile<Fam, T, N>(p, tl.first, sp, lds);
    } else {
      pm_tile<Fam, T, N>(p, tl.first, sp);
    }
  }
}

// One tile of any family and dimension in working precision T: the switch
// picks the template instance from the scan's own (family, N).
template <typename T>
__device__ __forceinline__ void run_tile_any(const ScanParams& p, const Tile& tl, double* lds) {
  const uint64_t sp = tl.split_mode & ~kTileSampleMajor;
  const bool sm = (tl.split_mode & kTileSampleMajor) != 0;
#define ZMC_TILE_CASE(FAM, NN)                                  \
  case FAM##_ID * 16 + NN:                                      \
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
  switch (p.family * 16 + p.N) {
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

// Batched scans, one kernel for every family and dimension of one working
// precision: the blocks pop tiles of all scans from one queue.
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
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const uint64_t s = s0 + (uint64_t)i;
  Fam fam;
  fam.setup(p, g);
  T v[4];
  eval_group<Fam, T, N>(fam, s >> 2, GenAny{g, p.seed}, v);
  const unsigned k = (unsigned)(s & 3u);
  out[i] = (double)(k == 0 ? v[0] : k == 1 ? v[1] : k == 2 ? v[2] : v[3]);
}

// ---------------------------------------------------------------------------
// Launchers of one family F in working precision T, for every N; each
// (family, precision) pair is instantiated in its own translation unit.
// ---------------------------------------------------------------------------
template <template <typename, int> class F, typename T>
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
#define ZMC_BY_DIMS(CALL)                                                           \
  switch (N) {                                                                      \
    case 1: if constexpr (1 >= F<T, 1>::kMinDims) return CALL(1); else break;       \
    case 2: return CALL(2);                                                         \
    case 3: return CALL(3);                                                         \
    case 4: return CALL(4);                                                         \
    case 5: return CALL(5);                                                         \
    case 6: return CALL(6);                                                         \
    case 7: return CALL(7);                                                         \
    case 8: return CALL(8);                                                         \
    default: break;                                                                 \
  }                                                                                 \
  return hipErrorInvalidValue;

template <template <typename, int> class F, typename T>
hipError_t FamilyOps<F, T>::main(int N, const ScanParams& p, const Plan& plan, hipStream_t stream) {
#define ZMC_CALL(NN) main_n<NN>(p, plan, stream)
  ZMC_BY_DIMS(ZMC_CALL)
#undef ZMC_CALL
}

template <template <typename, int> class F, typename T>
hipError_t FamilyOps<F, T>::values(int N, const ScanParams& p, uint64_t g, uint64_t s0,
                                   int64_t count, double* out, hipStream_t stream) {
#define ZMC_CALL(NN) values_n<NN>(p, g, s0, count, out, stream)
  ZMC_BY_DIMS(ZMC_CALL)
#undef ZMC_CALL
}

template <template <typename, int> class F, typename T>
hipError_t FamilyOps<F, T>::occupancy(int N, int* blocks_per_cu) {
#define ZMC_CALL(NN) occupancy_n<NN>(blocks_per_cu)
  ZMC_BY_DIMS(ZMC_CALL)
#undef ZMC_CALL
}

template <template <typename, int> class F, typename T>
hipError_t FamilyOps<F, T>::batch(int N, const ScanParams* scans, const Tile* tiles,
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

#define ZMC_DECLARE_FAMILY_OPS(F)                 \
  extern template struct FamilyOps<F, float>;     \
  extern template struct FamilyOps<F, double>;
ZMC_DECLARE_FAMILY_OPS(SinSum)
ZMC_DECLARE_FAMILY_OPS(Gauss)
ZMC_DECLARE_FAMILY_OPS(CosExp)
ZMC_DECLARE_FAMILY_OPS(Const)
ZMC_DECLARE_FAMILY_OPS(Linear)
#undef ZMC_DECLARE_FAMILY_OPS
extern template struct AnyOps<float>;
extern template struct AnyOps<double>;

}  // namespace zmc
