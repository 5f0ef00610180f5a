// zmc_kernels.hip -- the scan kernels for gfx950 and their launch dispatch.
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
#include "zmc_device.hpp"
#include "zmc_internal.hpp"

namespace zmc {

template <class Fam, typename T, int N>
__device__ __forceinline__ T centre_value(const Fam& fam) {
  T tc[N];
#pragma unroll
  for (int k = 0; k < N; ++k) tc[k] = Unif<T>::center;
  return fam.value(tc);
}

// Groups j0 .. jfull-1 in full, then (when `ragged`) the scan's short last
// group; every lane of the wave walks the same j.
template <class Fam, typename T, int N, class Gen>
__device__ __forceinline__ void lane_groups(const Fam& fam, const Gen& gen, uint64_t j0,
                                            uint64_t jfull, bool ragged, int tail,
                                            LaneAcc<T>& acc) {
  for (uint64_t j = j0; j < jfull; ++j) {
    T v[4];
    eval_group<Fam, T, N>(fam, j, gen, v);
    acc.add4(v);
  }
  if (ragged) {
    T v[4];
    eval_group<Fam, T, N>(fam, jfull, gen, v);
    acc.add_partial(v, tail);
  }
}

template <class Fam, typename T, int N>
__global__ __launch_bounds__(256) void k_point_major(ScanParams p) {
  const uint64_t sp = blockIdx.y;
  const uint64_t j0 = sp * p.gps;
  const uint64_t j1 = (j0 + p.gps < p.n_groups) ? j0 + p.gps : p.n_groups;
  const bool ragged = (j1 == p.n_groups) && ((p.n & 3u) != 0);
  const uint64_t jfull = ragged ? j1 - 1 : j1;
  const int tail = (int)(p.n - 4 * (p.n_groups - 1));
  const double count = (double)split_samples(p.n, p.n_groups, p.gps, sp);
  for (uint64_t pb = blockIdx.x; pb < p.point_blocks; pb += gridDim.x) {
    const uint64_t g = pb * blockDim.x + threadIdx.x;
    if (g >= p.G) continue;
    Fam fam;
    fam.setup(p, g);
    LaneAcc<T> acc;
    acc.init(centre_value<Fam, T, N>(fam));
    if (p.fast_counter) {
      const GenPointMajor gen{philox_lane((uint32_t)g, p.seed)};
      lane_groups<Fam, T, N>(fam, gen, j0, jfull, ragged, tail, acc);
    } else {
      const GenAny gen{g, p.seed};
      lane_groups<Fam, T, N>(fam, gen, j0, jfull, ragged, tail, acc);
    }
    const Moments m = to_moments(acc, count);
    if (p.splits == 1) {
      finalize(p, g, m);
    } else {
      p.part_mean[sp * p.G + g] = m.mean;
      p.part_m2[sp * p.G + g] = m.m2;
    }
  }
}

template <class Fam, typename T, int N>
__global__ __launch_bounds__(1024) void k_sample_major(ScanParams p) {
  __shared__ double lds_n[16], lds_mean[16], lds_m2[16];
  const uint64_t sp = blockIdx.y;
  const uint64_t j0 = sp * p.gps;
  const uint64_t j1 = (j0 + p.gps < p.n_groups) ? j0 + p.gps : p.n_groups;
  const uint64_t last = p.n_groups - 1;
  const int tail = (int)(p.n - 4 * last);  // samples in the scan's last group
  const unsigned waves = blockDim.x >> 6;
  for (uint64_t g = blockIdx.x; g < p.G; g += gridDim.x) {
    Fam fam;
    fam.setup(p, g);
    LaneAcc<T> acc;
    acc.init(centre_value<Fam, T, N>(fam));
    double count = 0.0;
    const GenAny gen{g, p.seed};
    for (uint64_t j = j0 + threadIdx.x; j < j1; j += blockDim.x) {
      T v[4];
      eval_group<Fam, T, N>(fam, j, gen, v);
      if (j == last && tail != 4) {
        acc.add_partial(v, tail);
        count += (double)tail;
      } else {
        acc.add4(v);
        count += 4.0;
      }
    }
    Moments m = wave_merge(to_moments(acc, count));
    const unsigned w = threadIdx.x >> 6;
    if ((threadIdx.x & 63u) == 0) {
      lds_n[w] = m.n;
      lds_mean[w] = m.mean;
      lds_m2[w] = m.m2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      Moments t{lds_n[0], lds_mean[0], lds_m2[0]};
      for (unsigned i = 1; i < waves; ++i) t = merge(t, Moments{lds_n[i], lds_mean[i], lds_m2[i]});
      if (p.splits == 1) {
        finalize(p, g, t);
      } else {
        p.part_mean[sp * p.G + g] = t.mean;
        p.part_m2[sp * p.G + g] = t.m2;
      }
    }
    __syncthreads();
  }
}

// Second pass: merge the split partials of each point in split order.
__global__ __launch_bounds__(256) void k_merge_splits(ScanParams p) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < p.G; g += stride) {
    Moments t{(double)split_samples(p.n, p.n_groups, p.gps, 0), p.part_mean[g], p.part_m2[g]};
    for (int sp = 1; sp < p.splits; ++sp) {
      const Moments b{(double)split_samples(p.n, p.n_groups, p.gps, (uint64_t)sp),
                      p.part_mean[(uint64_t)sp * p.G + g], p.part_m2[(uint64_t)sp * p.G + g]};
      t = merge(t, b);
    }
    finalize(p, g, t);
  }
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
// Dispatch: (family, precision, N) -> template instance.
// ---------------------------------------------------------------------------
namespace {

struct MainLaunch {
  const ScanParams* p;
  const Plan* plan;
  hipStream_t stream;
  template <class Fam, typename T, int N>
  hipError_t run() const {
    const dim3 block((unsigned)plan->block);
    const unsigned gx = (unsigned)plan->grid_x;
    const dim3 grid(gx, (unsigned)plan->splits);
    if (plan->mode == ZMC_MODE_POINT_MAJOR) {
      hipLaunchKernelGGL((k_point_major<Fam, T, N>), grid, block, 0, stream, *p);
    } else {
      hipLaunchKernelGGL((k_sample_major<Fam, T, N>), grid, block, 0, stream, *p);
    }
    return hipGetLastError();
  }
};

struct ValuesLaunch {
  const ScanParams* p;
  uint64_t g, s0;
  int64_t count;
  double* out;
  hipStream_t stream;
  template <class Fam, typename T, int N>
  hipError_t run() const {
    const unsigned blocks = (unsigned)((count + 255) / 256);
    hipLaunchKernelGGL((k_debug_values<Fam, T, N>), dim3(blocks), dim3(256), 0, stream, *p, g, s0,
                       count, out);
    return hipGetLastError();
  }
};

// Instances below a family's smallest N (COSEXP needs two dimensions) are
// never built; validation rejects those descriptors before dispatch.
template <template <typename, int> class F, typename T, int N, class Op>
hipError_t run_if_valid(const Op& op) {
  if constexpr (N >= F<T, N>::kMinDims) {
    return op.template run<F<T, N>, T, N>();
  } else {
    return hipErrorInvalidValue;
  }
}

template <template <typename, int> class F, typename T, class Op>
hipError_t by_dims(int N, const Op& op) {
  switch (N) {
    case 1: return run_if_valid<F, T, 1>(op);
    case 2: return run_if_valid<F, T, 2>(op);
    case 3: return run_if_valid<F, T, 3>(op);
    case 4: return run_if_valid<F, T, 4>(op);
    case 5: return run_if_valid<F, T, 5>(op);
    case 6: return run_if_valid<F, T, 6>(op);
    case 7: return run_if_valid<F, T, 7>(op);
    case 8: return run_if_valid<F, T, 8>(op);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, class Op>
hipError_t by_family(int family, int N, const Op& op) {
  switch (family) {
    case ZMC_SIN_SUM: return by_dims<SinSum, T>(N, op);
    case ZMC_GAUSS: return by_dims<Gauss, T>(N, op);
    case ZMC_COSEXP: return by_dims<CosExp, T>(N, op);
    case ZMC_CONST: return by_dims<Const, T>(N, op);
    case ZMC_LINEAR: return by_dims<Linear, T>(N, op);
    default: return hipErrorInvalidValue;
  }
}

template <class Op>
hipError_t by_precision(int precision, int family, int N, const Op& op) {
  if (precision == ZMC_FP64) return by_family<double>(family, N, op);
  return by_family<float>(family, N, op);
}

}  // namespace

hipError_t launch_scan(const ScanParams& p, const Plan& plan, int precision, hipStream_t stream,
                       hipEvent_t ev_begin, hipEvent_t ev_end) {
  MainLaunch op{&p, &plan, stream};
  hipError_t e = hipSuccess;
  if (ev_begin != nullptr) e = hipEventRecord(ev_begin, stream);
  if (e == hipSuccess) e = by_precision(precision, p.family, p.N, op);
  if (e == hipSuccess && ev_end != nullptr) e = hipEventRecord(ev_end, stream);
  if (e != hipSuccess || p.splits == 1) return e;
  uint64_t blocks = (p.G + 255) / 256;
  if (blocks > (1u << 20)) blocks = 1u << 20;
  hipLaunchKernelGGL(k_merge_splits, dim3((unsigned)blocks), dim3(256), 0, stream, p);
  return hipGetLastError();
}

hipError_t launch_debug_words(uint64_t seed, uint64_t g, uint64_t w0, int64_t count,
                              uint32_t* out, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_debug_words, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, stream,
                     seed, g, w0, count, out);
  return hipGetLastError();
}

hipError_t launch_debug_values(const ScanParams& p, int precision, uint64_t g, uint64_t s0,
                               int64_t count, double* out, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  ValuesLaunch op{&p, g, s0, count, out, stream};
  return by_precision(precision, p.family, p.N, op);
}

}  // namespace zmc
