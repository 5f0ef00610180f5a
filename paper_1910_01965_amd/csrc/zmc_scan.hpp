// zmc_scan.hpp -- the scan loops on gfx950, device code only (no host
// dependencies), so that both the compiled-in kernels and the kernels built at
// run time for user integrands use them.
//
// Point-major: a lane owns one grid point and all lanes of a wave walk the
// same groups of four samples in step, so the Philox counter words that
// depend only on the sample index (the word block b) are wave-uniform and
// live in scalar registers; only the grid-index half of the counter differs
// between lanes.  A point's sample range may be cut into `splits` pieces run
// by different blocks; their FP64 partials are merged by a second pass.
//
// Sample-major: a block owns one grid point and its lanes share the samples
// (lane t takes groups t, t+T, ...); lane sums are merged over the wave by a
// shuffle butterfly, then over the block's waves through LDS, then (for
// several blocks per point) by the same second pass.
//
// Method: direct Monte Carlo per grid point, ZMCintegral-v5 Sec. 2, Eq. (1);
// the paper gives each point to one GPU thread (Sec. 2, Fig. 1), which is the
// point-major layout without splits.
#pragma once

#include "zmc_device.hpp"

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
  // j <= jfull here; the inequality test keeps the (wave-uniform) loop
  // control on the scalar unit, which has no unsigned 64-bit "less than"
  for (; j != jfull; ++j) {
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
  const uint64_t g = first + threadIdx.x;  // local index: outputs
  if (g >= p.G) return;
  const uint64_t gg = p.g_base + g;        // global index: parameters and stream
  Fam fam;
  fam.setup(p, gg);
  LaneAcc<T> acc;
  acc.init((T)0);
  with_form(fam, [&](const auto& f) {
    using F = std::decay_t<decltype(f)>;
    if (p.fast_counter) {
      const GenPointMajor gen{philox_lane((uint32_t)gg, p.seed)};
      lane_groups<F, T, N>(f, gen, j0, jfull, ragged, tail, acc);
    } else {
      const GenAny gen{gg, p.seed};
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

// One sample-major tile: the whole block works on grid point g (local index;
// its global index is p.g_base + g) over sample piece sp (lane t takes
// groups j0 + t, j0 + t + T, ...), then merges its lanes.  Every thread of
// the block must call it (it synchronises); `lds` holds 3 x 16 doubles.
template <class Fam, typename T, int N>
__device__ __forceinline__ void sm_tile(const ScanParams& p, uint64_t g, uint64_t sp, double* lds) {
  const uint64_t j0 = sp * p.gps;
  const uint64_t j1 = (j0 + p.gps < p.n_groups) ? j0 + p.gps : p.n_groups;
  const uint64_t last = p.n_groups - 1;
  const int tail = (int)(p.n - 4 * last);  // samples in the scan's last group
  const unsigned waves = blockDim.x >> 6;
  Fam fam;
  fam.setup(p, p.g_base + g);
  LaneAcc<T> acc;
  acc.init((T)0);
  double count = 0.0;
  const GenAny gen{p.g_base + g, p.seed};
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

// Kernel bodies: the point-major scan (grid.x = point blocks, grid.y = sample
// pieces), the sample-major scan (grid.x = points, grid.y = pieces; `lds`
// holds 3 x 16 doubles) and per-sample integrand values of global point g
// (debugging, parity).
template <class Fam, typename T, int N>
__device__ __forceinline__ void point_major_body(const ScanParams& p) {
  for (uint64_t pb = blockIdx.x; pb < p.point_blocks; pb += gridDim.x)
    pm_tile<Fam, T, N>(p, pb * blockDim.x, blockIdx.y);
}

template <class Fam, typename T, int N>
__device__ __forceinline__ void sample_major_body(const ScanParams& p, double* lds) {
  for (uint64_t g = blockIdx.x; g < p.G; g += gridDim.x) sm_tile<Fam, T, N>(p, g, blockIdx.y, lds);
}

// Persistent batch body: the block pops tiles [begin, end) of the tile table
// through one atomic counter and runs them until the table is exhausted;
// every block reaches that exit.  `next` and `lds` are the kernel's shared
// memory (one word, 3 x 16 doubles).
template <class Fam, typename T, int N>
__device__ __forceinline__ void batch_body(const ScanParams* __restrict__ scans,
                                           const Tile* __restrict__ tiles, uint32_t begin,
                                           uint32_t end, uint32_t* counter, uint32_t* next,
                                           double* lds) {
  for (;;) {
    __syncthreads();  // the previous tile is done with `next` and `lds`
    if (threadIdx.x == 0) *next = begin + atomicAdd(counter, 1u);
    __syncthreads();
    const uint32_t t = *next;
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

template <class Fam, typename T, int N>
__device__ __forceinline__ void debug_values_body(const ScanParams& p, uint64_t g, uint64_t s0,
                                                  int64_t count, double* out) {
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

}  // namespace zmc
