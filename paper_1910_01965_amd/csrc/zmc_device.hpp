// zmc_device.hpp -- device building blocks of the parameter-scan kernels
// (gfx950, wave64): the counter-based generator, the uniform maps, the
// integrand families, per-lane accumulators and the FP64 merges.
//
// Method: direct Monte Carlo at every grid point (ZMCintegral-v5, Sec. 2,
// Eq. (1)); the paper leaves the generator, the sample layout and the error
// estimate open, and the library fixes them as stated in include/zmc.h.
#pragma once

#if defined(__HIPCC_RTC__)
// hipRTC (user integrands): its runtime header keeps the fixed-width types
// in its own namespace
using __hip_internal::int32_t;
using __hip_internal::int64_t;
using __hip_internal::uint32_t;
using __hip_internal::uint64_t;
#else
#include <hip/hip_runtime.h>
#include <stdint.h>
#endif

#include <type_traits>

namespace zmc {

constexpr int kMaxParams = 16;
constexpr int kMaxDims = 16;
constexpr int kAnyMaxDims = 8;  // integration dimensions of the any-family batch kernel
constexpr int kMaxUserParams = 16;  // constants passed to a user integrand

// Everything a scan kernel needs, passed by value as the kernel argument.
struct ScanParams {
  uint64_t G;            // grid points of this launch (local indices 0..G-1)
  uint64_t g_base;       // global flat index of local point 0 (chunked scans)
  uint64_t n;            // samples per point
  uint64_t n_groups;     // ceil(n / 4)
  uint64_t gps;          // groups per split
  uint64_t seed;
  uint64_t point_blocks; // ceil(G / block) (point-major)
  int32_t M, N, splits, family;
  int32_t fast_counter;  // 1 when every word block b and global index g is < 2^32
  int32_t n_params;      // user integrands: entries of params in use
  int64_t axis_len[kMaxParams];
  int64_t axis_off[kMaxParams];
  uint64_t axis_stride[kMaxParams];  // prod of the lengths of later axes
  double lo[kMaxDims], hi[kMaxDims];
  double vol;
  double params[kMaxUserParams];
  const double* axis;    // device: concatenated value lists
  double* f;             // device outputs [G]
  double* sigma;
  double* part_mean;     // device split partials [splits][G] (or null)
  double* part_m2;
};

// One unit of batched work: a point-major tile (256 consecutive grid points
// of one scan over one sample piece) or a sample-major tile (one grid point,
// one sample piece, the whole block).
struct Tile {
  uint32_t scan;        // index into the batch's scan table
  uint32_t split_mode;  // bits 0..30: sample piece; bit 31: 1 = sample-major
  uint64_t first;       // point-major: first grid point; sample-major: the point
};

constexpr uint32_t kTileSampleMajor = 0x80000000u;

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  A round takes the high
// and low halves of the products of words 0 and 2 with the two multipliers
// and mixes the highs with words 1, 3 and the round key; the key advances by
// the two Weyl increments.  On gfx950 a 32x32->64 product is one full-rate
// v_mad_u64_u32 and the three-way xor is one v_bitop3_b32 (truth table 0x96).
// ---------------------------------------------------------------------------
constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u;
constexpr uint32_t kPhiloxW1 = 0xBB67AE85u;

__host__ __device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
#else
  return a ^ b ^ c;
#endif
}

struct Words4 {
  uint32_t r[4];
};

// One Philox round on (c0, c1, c2, c3) with round key (k0, k1).
__host__ __device__ __forceinline__ void philox_round(uint32_t& c0, uint32_t& c1, uint32_t& c2,
                                                      uint32_t& c3, uint32_t k0, uint32_t k1) {
  const uint64_t p0 = (uint64_t)kPhiloxM0 * c0;
  const uint64_t p1 = (uint64_t)kPhiloxM1 * c2;
  const uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, k0);
  const uint32_t n2 = xor3((uint32_t)(p0 >> 32), c3, k1);
  c1 = (uint32_t)p1;
  c3 = (uint32_t)p0;
  c0 = n0;
  c2 = n2;
}

__host__ __device__ __forceinline__ Words4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                                         uint32_t c3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    philox_round(c0, c1, c2, c3, k0, k1);
    k0 += kPhiloxW0;
    k1 += kPhiloxW1;
  }
  Words4 w;
  w.r[0] = c0; w.r[1] = c1; w.r[2] = c2; w.r[3] = c3;
  return w;
}

// Block b of grid point g: counter (b lo, b hi, g lo, g hi), key = seed.
__host__ __device__ __forceinline__ Words4 philox_block(uint64_t b, uint64_t g, uint64_t seed) {
  return philox4x32_10((uint32_t)b, (uint32_t)(b >> 32), (uint32_t)g, (uint32_t)(g >> 32),
                       (uint32_t)seed, (uint32_t)(seed >> 32));
}

// ---------------------------------------------------------------------------
// The same blocks for the point-major layout when b < 2^32 and g < 2^32 (the
// host checks both for the whole scan).  All lanes of a wave then share b and
// differ in g only, so the first two rounds split into a per-lane part that
// does not change from block to block (computed once per point) and a
// wave-uniform part that the compiler keeps in scalar registers:
//   round 1: (hi, lo)(M1 g) is per lane and fixed; (hi, lo)(M0 b) is uniform;
//   round 2: M0 times the round-1 word 0 = hi(M1 g) ^ k0 is per lane and
//            fixed; M1 times the round-1 word 2 = hi(M0 b) ^ k1 is uniform.
// Only rounds 3..10 multiply per-lane, per-block values.
// ---------------------------------------------------------------------------
struct PhiloxLane {
  uint32_t r1;   // round-1 output word 1: lo(M1 g)
  uint32_t h2;   // hi(M0 * round-1 word 0)
  uint32_t l2;   // lo(M0 * round-1 word 0)
  uint32_t k0, k1;
};

__host__ __device__ __forceinline__ PhiloxLane philox_lane(uint32_t g, uint64_t seed) {
  PhiloxLane L;
  L.k0 = (uint32_t)seed;
  L.k1 = (uint32_t)(seed >> 32);
  const uint64_t p1 = (uint64_t)kPhiloxM1 * g;
  const uint32_t w0 = (uint32_t)(p1 >> 32) ^ L.k0;  // counter word 1 (b hi) is 0
  L.r1 = (uint32_t)p1;
  const uint64_t p2 = (uint64_t)kPhiloxM0 * w0;
  L.h2 = (uint32_t)(p2 >> 32);
  L.l2 = (uint32_t)p2;
  return L;
}

__host__ __device__ __forceinline__ Words4 philox_block_pm(uint32_t b, const PhiloxLane& L) {
  // round 1 (key k): words 0, 1 per lane and fixed; words 2, 3 uniform
  const uint64_t q0 = (uint64_t)kPhiloxM0 * b;
  const uint32_t u2 = (uint32_t)(q0 >> 32) ^ L.k1;  // counter word 3 (g hi) is 0
  const uint32_t u3 = (uint32_t)q0;
  // round 2 (key k + W): the product with word 2 is uniform
  const uint32_t k0b = L.k0 + kPhiloxW0, k1b = L.k1 + kPhiloxW1;
  const uint64_t q1 = (uint64_t)kPhiloxM1 * u2;
  uint32_t c0 = L.r1 ^ ((uint32_t)(q1 >> 32) ^ k0b);
  uint32_t c1 = (uint32_t)q1;
  uint32_t c2 = L.h2 ^ (u3 ^ k1b);
  uint32_t c3 = L.l2;
  uint32_t k0 = k0b + kPhiloxW0, k1 = k1b + kPhiloxW1;
  {
    // round 3: word 1 and the key are uniform, word 3 is per lane and fixed,
    // so each new word is one per-lane product high half and one xor
    const uint64_t p0 = (uint64_t)kPhiloxM0 * c0;
    const uint64_t p1 = (uint64_t)kPhiloxM1 * c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ (c1 ^ k0);
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ (c3 ^ k1);
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += kPhiloxW0;
    k1 += kPhiloxW1;
  }
#pragma unroll
  for (int round = 3; round < 10; ++round) {
    philox_round(c0, c1, c2, c3, k0, k1);
    k0 += kPhiloxW0;
    k1 += kPhiloxW1;
  }
  Words4 w;
  w.r[0] = c0; w.r[1] = c1; w.r[2] = c2; w.r[3] = c3;
  return w;
}

// ---------------------------------------------------------------------------
// Uniform variates.  The per-dimension affine map y = A t + B is folded into
// each family; t is
//   FP64: u = (r + 1/2) 2^-32 exactly, A = hi - lo, B = lo (y = fma(A, u, B));
//   FP32: v = 1 + (r >> 9) 2^-23 in [1, 2) built from the bits (one
//         v_alignbit_b32), A = hi - lo, B = lo - A (1 - 2^-24), so that
//         A v + B = lo + A ((r >> 9) + 1/2) 2^-23.
// ---------------------------------------------------------------------------
template <typename T> struct Unif;

// FP64: the variate is the word itself, t = r (exact), and the affine
// constants carry the scale and the half-step offset of u = (r + 1/2) 2^-32:
// y = lo + h u = (h 2^-32) r + (lo + h 2^-33).  The power-of-two scalings are
// exact; the one rounding of B moves y by at most half an ulp from
// fma(h, u, lo), and the map costs a conversion and one fma per coordinate.
template <> struct Unif<double> {
  static __device__ __forceinline__ double t(uint32_t r) { return (double)r; }
  static __host__ __device__ inline void affine(double lo, double hi, double* A, double* B) {
    const double h = hi - lo;
    *A = h * 0x1p-32;
    *B = lo + h * 0x1p-33;
  }
};

template <> struct Unif<float> {
  static __device__ __forceinline__ float t(uint32_t r) {
    // (0x7F : r) >> 9 = 0x3F800000 | (r >> 9): a float in [1, 2)
    return __uint_as_float(__builtin_amdgcn_alignbit(0x7Fu, r, 9u));
  }
  static __host__ __device__ inline void affine(double lo, double hi, double* A, double* B) {
    *A = hi - lo;
    *B = lo - (hi - lo) * (1.0 - 0x1p-24);
  }
};

template <typename T> __device__ __forceinline__ T fmaT(T a, T b, T c);
template <> __device__ __forceinline__ double fmaT(double a, double b, double c) {
  return __builtin_fma(a, b, c);
}
template <> __device__ __forceinline__ float fmaT(float a, float b, float c) {
  return __builtin_fmaf(a, b, c);
}

constexpr double kLog2e = 1.4426950408889634074;

// FP32 sine and cosine through the hardware units, which take their argument
// in revolutions.  The FP32 families carry phases in revolutions throughout:
// the per-point constants are multiplied by 1/(2 pi) in FP64 at set-up, before
// rounding, so a sample's phase r carries the same relative rounding as the
// phase in radians would, and r - rint(r) reduces it to [-1/2, 1/2] exactly
// (for |r| >= 2^23 an FP32 phase no longer resolves a revolution and the
// reduced phase is 0).
constexpr double kInv2Pi = 0.15915494309189533577;

__device__ __forceinline__ float sin_turns(float r) {
  return __builtin_amdgcn_sinf(r - __builtin_rintf(r));
}

__device__ __forceinline__ float cos_turns(float r) {
  return __builtin_amdgcn_cosf(r - __builtin_rintf(r));
}

// FP64 sine and cosine of a phase r in revolutions.  t = r - rint(r) lies in
// [-1/2, 1/2] exactly.  Both reduce to sin(2 pi v) with v in [-1/4, 1/4]:
//   sin: v = t for |t| <= 1/4, else v = copysign(1/2, t) - t (sin(pi - a) =
//        sin a; exact, since 1/4 <= |t| <= 1/2);
//   cos: v = 1/4 - |t| (cos a = sin(pi/2 - a); exact for |t| >= 1/8, else
//        one rounding of at most 2^-55 revolutions).
// sin(2 pi v) = v P(v^2) with P of degree 8, from Chebyshev economization of
// the Taylor series on [-1/4, 1/4] (paper_1910_01965_amd/fp64_poly.py: the
// dropped terms are below 1.7e-19, the FP64 Horner evaluation within 2.2e-16
// relative of a 60-digit reference on a dense grid).  One polynomial serves
// both functions, with no octant selection.
__host__ __device__ __forceinline__ double sin_2pi_quarter(double v) {
  const double v2 = v * v;
  double p = 0.10071467531221244;
  p = __builtin_fma(p, v2, -0.7176853699001249);
  p = __builtin_fma(p, v2, 3.8199227975201033);
  p = __builtin_fma(p, v2, -15.094641368684599);
  p = __builtin_fma(p, v2, 42.05869391526577);
  p = __builtin_fma(p, v2, -76.70585975263434);
  p = __builtin_fma(p, v2, 81.60524927607172);
  p = __builtin_fma(p, v2, -41.34170224039975);
  p = __builtin_fma(p, v2, 6.283185307179586);
  return v * p;
}

// FP64 2^t.  k = rint(t) and f = t - k in [-1/2, 1/2] (exact); 2^f by a
// degree-11 polynomial from Chebyshev economization of the Taylor series of
// e^(f ln 2) on [-1/2, 1/2] (fp64_poly.py: dropped terms below 3.2e-18,
// Horner within 1.2e-16 relative); 2^k applied by ldexp.  t is first clamped
// to [-2100, 2100], beyond which 2^t is 0 or inf in double: -inf then gives
// 0 and +inf gives inf, as exp does, and k always fits an int (a NaN t is
// clamped too and gives 0; the parameter values it would come from must be
// finite).  kNonPositive: the caller guarantees t <= 0 (or NaN), so only the
// lower clamp is needed.
template <bool kNonPositive = false>
__host__ __device__ __forceinline__ double exp2_fp64(double t) {
  t = __builtin_fmax(t, -2100.0);
  if constexpr (!kNonPositive) t = __builtin_fmin(t, 2100.0);
  const double k = __builtin_rint(t);
  const double f = t - k;
  double p = 4.456675463639861e-10;
  p = __builtin_fma(p, f, 7.074194562613105e-09);
  p = __builtin_fma(p, f, 1.0178051192117847e-07);
  p = __builtin_fma(p, f, 1.3215432534254118e-06);
  p = __builtin_fma(p, f, 1.5252733856295574e-05);
  p = __builtin_fma(p, f, 0.00015403530463727982);
  p = __builtin_fma(p, f, 0.001333355814639035);
  p = __builtin_fma(p, f, 0.009618129107587253);
  p = __builtin_fma(p, f, 0.0555041086648217);
  p = __builtin_fma(p, f, 0.24022650695910158);
  p = __builtin_fma(p, f, 0.6931471805599453);
  p = __builtin_fma(p, f, 1.0);
  return __builtin_ldexp(p, (int)k);
}

__host__ __device__ __forceinline__ double sin_turns(double r) {
  const double t = r - __builtin_rint(r);
  return sin_2pi_quarter(__builtin_fabs(t) > 0.25 ? __builtin_copysign(0.5, t) - t : t);
}

__host__ __device__ __forceinline__ double cos_turns(double r) {
  const double t = r - __builtin_rint(r);
  return sin_2pi_quarter(0.25 - __builtin_fabs(t));
}

// Parameter x_l of grid point g (C order: stride_l = prod_{j>l} L_j).
__device__ __forceinline__ double param_x(const ScanParams& p, uint64_t g, int l) {
  const uint64_t i = (g / p.axis_stride[l]) % (uint64_t)p.axis_len[l];
  return p.axis[p.axis_off[l] + (int64_t)i];
}

// ---------------------------------------------------------------------------
// Integrand families.  Each one holds the per-point constants (set up once
// per point in FP64, then rounded to T) and evaluates one sample from its N
// variates t[0..N-1].
// ---------------------------------------------------------------------------

// sin(sum_l x_l + sum_k y_k): the paper's test integrand, Eq. (2) and Eq. (4).
template <typename T, int N> struct SinSum {
  static constexpr int kMinDims = 1;
  T A[N], B[N];
  T sx;        // FP64: sum of x; FP32: sum x + sum B (all in revolutions)
  __device__ void setup(const ScanParams& p, uint64_t g) {
    double s = 0.0, sb = 0.0;
    for (int l = 0; l < p.M; ++l) s += param_x(p, g, l);
#pragma unroll
    for (int k = 0; k < N; ++k) {
      double a, b;
      Unif<T>::affine(p.lo[k], p.hi[k], &a, &b);
      A[k] = (T)(a * kInv2Pi);
      B[k] = (T)(b * kInv2Pi);
      sb += b;
    }
    sx = sizeof(T) == 8 ? (T)(s * kInv2Pi) : (T)((s + sb) * kInv2Pi);
  }
  __device__ __forceinline__ T value(const T* t) const {
    if constexpr (sizeof(T) == 8) {
      double sy = 0.0;
#pragma unroll
      for (int k = 0; k < N; ++k) sy += fmaT(A[k], t[k], B[k]);
      return sin_turns(sx + sy);
    } else {
      float ph = sx;
#pragma unroll
      for (int k = 0; k < N; ++k) ph = fmaT(A[k], t[k], ph);
      return sin_turns(ph);
    }
  }
};

// exp(-(sum_{k<=M} x_k y_k^2 + sum_{k>M} y_k^2)).
// With every coefficient c_k of a point finite and >= 0 (c_k = x_k for k <= M,
// 1 beyond; times log2(e) in FP32), sqrt(c_k) is folded into that point's
// affine map, z_k = sqrt(c_k) y_k, and the point stores c_k = 1, so that the
// one formula fma(c_k y, y, q) gives sum_k z_k^2.  The tile loops run waves
// whose points are all folded on GaussUnit, which drops the product with
// c_k = 1 and so changes no bit: a point's value depends on that point alone.
template <typename T, int N> struct GaussUnit {
  T A[N], B[N];
  __device__ __forceinline__ T value(const T* t) const {
    // the first square is a plain product: fma(z, z, +0) would be the same
    // value but a three-operand instruction, which cannot dual-issue
    T q;
#pragma unroll
    for (int k = 0; k < N; ++k) {
      const T z = fmaT(A[k], t[k], B[k]);
      q = k == 0 ? z * z : fmaT(z, z, q);
    }
    if constexpr (sizeof(T) == 8) {
      return exp2_fp64<true>(q * -kLog2e);  // q, a sum of squares, is >= 0
    } else {
      return __builtin_amdgcn_exp2f(-q);
    }
  }
};

template <typename T, int N> struct Gauss {
  static constexpr int kMinDims = 1;
  using UnitForm = GaussUnit<T, N>;
  T A[N], B[N], c[N];   // FP32: c carries log2(e) for exp2
  bool unit;            // wave-uniform: c_k = 1 on every active lane of the wave
  __device__ void setup(const ScanParams& p, uint64_t g) {
    double x[N];
    bool fold = true;
#pragma unroll
    for (int k = 0; k < N; ++k) {
      x[k] = (k < p.M) ? param_x(p, g, k) : 1.0;
      fold = fold && x[k] >= 0.0 && x[k] <= 0x1.fffffffffffffp+1023;
    }
#pragma unroll
    for (int k = 0; k < N; ++k) {
      double a, b;
      Unif<T>::affine(p.lo[k], p.hi[k], &a, &b);
      const double ck = sizeof(T) == 8 ? x[k] : x[k] * kLog2e;
      const double s = fold ? sqrt(ck) : 1.0;
      A[k] = (T)(a * s);
      B[k] = (T)(b * s);
      c[k] = fold ? (T)1 : (T)ck;
    }
    unit = __builtin_amdgcn_ballot_w64(!fold) == 0;
  }
  __device__ __forceinline__ UnitForm unit_form() const {
    UnitForm u;
#pragma unroll
    for (int k = 0; k < N; ++k) {
      u.A[k] = A[k];
      u.B[k] = B[k];
    }
    return u;
  }
  __device__ __forceinline__ T value(const T* t) const {
    T q;
#pragma unroll
    for (int k = 0; k < N; ++k) {
      const T y = fmaT(A[k], t[k], B[k]);
      q = k == 0 ? (c[k] * y) * y : fmaT(c[k] * y, y, q);
    }
    if constexpr (sizeof(T) == 8) {
      return exp2_fp64(q * -kLog2e);
    } else {
      return __builtin_amdgcn_exp2f(-q);
    }
  }
};

// cos(x1 y1 + x2 y2 + sum_{k>=3} y_k) exp(-x3^2 y1 y2) + x4.
template <typename T, int N> struct CosExp {
  static constexpr int kMinDims = 2;
  T A[N], B[N];
  T x1, x2, nx3sq, x4;  // nx3sq = -x3^2 log2(e): the exponential is evaluated as 2^t
  T rest;               // FP32: sum of B_k for k >= 3, folded into the phase
  // x1, x2, rest and A_k, B_k (k >= 3) in revolutions (times 1/(2 pi))
  __device__ void setup(const ScanParams& p, uint64_t g) {
    const double turn = kInv2Pi;
    double sb = 0.0;
#pragma unroll
    for (int k = 0; k < N; ++k) {
      double a, b;
      Unif<T>::affine(p.lo[k], p.hi[k], &a, &b);
      A[k] = (T)(k >= 2 ? a * turn : a);
      B[k] = (T)(k >= 2 && sizeof(T) == 8 ? b * turn : b);
      if (k >= 2) sb += b;
    }
    x1 = (T)(param_x(p, g, 0) * turn);
    x2 = (T)(param_x(p, g, 1) * turn);
    const double x3 = param_x(p, g, 2);
    nx3sq = (T)(-(x3 * x3) * kLog2e);
    x4 = (T)param_x(p, g, 3);
    rest = (T)(sb * turn);
  }
  __device__ __forceinline__ T value(const T* t) const {
    const T y1 = fmaT(A[0], t[0], B[0]);
    const T y2 = fmaT(A[1], t[1], B[1]);
    if constexpr (sizeof(T) == 8) {
      double ph = x1 * y1 + x2 * y2;
#pragma unroll
      for (int k = 2; k < N; ++k) ph += fmaT(A[k], t[k], B[k]);
      return __builtin_fma(cos_turns(ph), exp2_fp64(nx3sq * y1 * y2), x4);
    } else {
      float ph;
      if constexpr (N == 2) {
        ph = fmaT(x1, y1, x2 * y2);  // no further terms: no zero addend
      } else {
        ph = rest;
#pragma unroll
        for (int k = 2; k < N; ++k) ph = fmaT(A[k], t[k], ph);
        ph = fmaT(x1, y1, fmaT(x2, y2, ph));
      }
      const float e = __builtin_amdgcn_exp2f(nx3sq * y1 * y2);
      return fmaT(cos_turns(ph), e, x4);
    }
  }
};

// 1: the sampler must reproduce the box volume exactly.
template <typename T, int N> struct Const {
  static constexpr int kMinDims = 1;
  __device__ void setup(const ScanParams&, uint64_t) {}
  __device__ __forceinline__ T value(const T*) const { return (T)1; }
};

// sum_k y_k.
template <typename T, int N> struct Linear {
  static constexpr int kMinDims = 1;
  T A[N], B[N];
  __device__ void setup(const ScanParams& p, uint64_t) {
#pragma unroll
    for (int k = 0; k < N; ++k) {
      double a, b;
      Unif<T>::affine(p.lo[k], p.hi[k], &a, &b);
      A[k] = (T)a;
      B[k] = (T)b;
    }
  }
  __device__ __forceinline__ T value(const T* t) const {
    T s = (T)0;
#pragma unroll
    for (int k = 0; k < N; ++k) s += fmaT(A[k], t[k], B[k]);
    return s;
  }
};

// ---------------------------------------------------------------------------
// One group of four consecutive samples s = 4j .. 4j+3 of point g uses the N
// Philox blocks b = jN .. jN+N-1 (words 4Nj .. 4Nj+4N-1, word i of the group
// being coordinate i mod N of sample 4j + i / N).
// ---------------------------------------------------------------------------
// Word-block generators of one grid point: any counter, or the point-major
// fast path (b < 2^32, g < 2^32, b shared by the wave).
struct GenAny {
  uint64_t g, seed;
  __device__ __forceinline__ Words4 block(uint64_t b) const { return philox_block(b, g, seed); }
};

struct GenPointMajor {
  PhiloxLane L;
  __device__ __forceinline__ Words4 block(uint64_t b) const {
    return philox_block_pm((uint32_t)b, L);
  }
};

template <class Fam, typename T, int N, class Gen>
__device__ __forceinline__ void eval_group(const Fam& fam, uint64_t j, const Gen& gen, T v[4]) {
  T t[4 * N];
  const uint64_t b0 = j * (uint64_t)N;
  if constexpr (N <= kAnyMaxDims) {
#pragma unroll
    for (int c = 0; c < N; ++c) {
      const Words4 w = gen.block(b0 + c);
#pragma unroll
      for (int i = 0; i < 4; ++i) t[4 * c + i] = Unif<T>::t(w.r[i]);
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) v[s] = fam.value(t + s * N);
  } else {
    // many dimensions: sample s is evaluated right after the block that holds
    // its last word (word sN + N - 1), so that only the variates of about one
    // sample are live at a time; the values are the same
#pragma unroll
    for (int c = 0; c < N; ++c) {
      const Words4 w = gen.block(b0 + c);
#pragma unroll
      for (int i = 0; i < 4; ++i) t[4 * c + i] = Unif<T>::t(w.r[i]);
#pragma unroll
      for (int s = 0; s < 4; ++s)
        if ((s * N + N - 1) / 4 == c) v[s] = fam.value(t + s * N);
    }
  }
}

// Runs body(f) with f = the family's reduced form (Fam::UnitForm) when the
// family has one and its wave-uniform `unit` flag is set, else with fam
// itself; the two give the same bits, the reduced form in fewer instructions.
template <class Fam, class = void> struct HasUnitForm : std::false_type {};
template <class Fam>
struct HasUnitForm<Fam, std::void_t<typename Fam::UnitForm>> : std::true_type {};

template <class Fam, class Body>
__device__ __forceinline__ void with_form(const Fam& fam, Body&& body) {
  if constexpr (HasUnitForm<Fam>::value) {
    if (fam.unit) {
      body(fam.unit_form());
      return;
    }
  }
  body(fam);
}

// ---------------------------------------------------------------------------
// Per-lane accumulation: shifted sums of d = v - c and d^2 in T, each with a
// Kahan compensation term, four samples at a time.  c is one of the lane's own
// samples, which keeps the final M2 = S2 - S1^2 / n well conditioned.
// ---------------------------------------------------------------------------
template <typename T> struct LaneAcc {
  T c;
  T s1, e1, s2, e2;
  __device__ __forceinline__ void init(T shift) {
    c = shift;
    s1 = e1 = s2 = e2 = (T)0;
  }
  __device__ __forceinline__ static void kahan(T& s, T& e, T x) {
    const T y = x - e;
    const T tt = s + y;
    e = (tt - s) - y;
    s = tt;
  }
  __device__ __forceinline__ void add4(const T v[4]) {
    const T d0 = v[0] - c, d1 = v[1] - c, d2 = v[2] - c, d3 = v[3] - c;
    const T s = (d0 + d1) + (d2 + d3);
    const T q = fmaT(d0, d0, d1 * d1) + fmaT(d2, d2, d3 * d3);
    kahan(s1, e1, s);
    kahan(s2, e2, q);
  }
  // the first `valid` of the four values count (ragged last group)
  __device__ __forceinline__ void add_partial(const T v[4], int valid) {
    T w[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) w[i] = (i < valid) ? v[i] : c;
    add4(w);
  }
};

// Welford state (count, mean, M2) in FP64.
struct Moments {
  double n, mean, m2;
};

template <typename T>
__device__ __forceinline__ Moments to_moments(const LaneAcc<T>& a, double count) {
  Moments m;
  m.n = count;
  if (count > 0.0) {
    const double S1 = (double)a.s1 - (double)a.e1;
    const double S2 = (double)a.s2 - (double)a.e2;
    m.mean = (double)a.c + S1 / count;
    m.m2 = S2 - S1 * (S1 / count);
    if (m.m2 < 0.0) m.m2 = 0.0;
  } else {
    m.mean = 0.0;
    m.m2 = 0.0;
  }
  return m;
}

// Chan, Golub, LeVeque pairwise merge; `a` is always the lower-indexed part
// so that every merge order is fixed.
__device__ __forceinline__ Moments merge(const Moments& a, const Moments& b) {
  if (b.n == 0.0) return a;
  if (a.n == 0.0) return b;
  Moments m;
  m.n = a.n + b.n;
  const double d = b.mean - a.mean;
  const double wb = b.n / m.n;
  m.mean = a.mean + d * wb;
  m.m2 = a.m2 + b.m2 + d * d * a.n * wb;
  return m;
}

// Butterfly over the 64 lanes; every lane ends with the merge of all 64,
// combined in lane order at every level.
__device__ __forceinline__ Moments wave_merge(Moments m) {
  const int lane = (int)(threadIdx.x & 63u);
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    Moments o;
    o.n = __shfl_xor(m.n, off, 64);
    o.mean = __shfl_xor(m.mean, off, 64);
    o.m2 = __shfl_xor(m.m2, off, 64);
    m = (lane & off) ? merge(o, m) : merge(m, o);
  }
  return m;
}

// Samples in split sp (groups [sp*gps, min((sp+1)*gps, n_groups)), the last
// group of the scan possibly short).
__host__ __device__ __forceinline__ uint64_t split_samples(uint64_t n, uint64_t n_groups,
                                                           uint64_t gps, uint64_t sp) {
  const uint64_t j0 = sp * gps;
  uint64_t j1 = j0 + gps;
  if (j1 > n_groups) j1 = n_groups;
  if (j0 >= j1) return 0;
  uint64_t s1 = 4 * j1;
  if (s1 > n) s1 = n;
  return s1 - 4 * j0;
}

__device__ __forceinline__ void finalize(const ScanParams& p, uint64_t g, const Moments& m) {
  p.f[g] = p.vol * m.mean;
  p.sigma[g] = p.vol * sqrt(m.m2 / (m.n * (m.n - 1.0)));
}

}  // namespace zmc
