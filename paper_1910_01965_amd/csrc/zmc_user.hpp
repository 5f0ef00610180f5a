// zmc_user.hpp -- the integrand family of a user function, for the kernels
// that the library builds at run time (hipRTC) from the user's source.  The
// program that includes this header first defines, at global scope,
//
//   template <typename T> __device__ T integrand(const T* y, const T* x, const T* p);
//
// where y holds the sample's N coordinates in the box, x the grid point's M
// parameters and p the scan's constant parameters (n_params <= 16 of them),
// all in the working precision T.  This is the paper's user-defined integrand
// of a parameter scan (Sec. 2; Sec. 4), compiled for the device instead of by
// Numba.
#pragma once

#include "zmc_scan.hpp"

namespace zmc {

template <typename T, int N, int M>
struct UserFamily {
  static constexpr int kMinDims = 1;
  T A[N], B[N];
  T x[M > 0 ? M : 1];
  T q[kMaxUserParams];
  __device__ void setup(const ScanParams& p, uint64_t g) {
#pragma unroll
    for (int k = 0; k < N; ++k) {
      double a, b;
      Unif<T>::affine(p.lo[k], p.hi[k], &a, &b);
      A[k] = (T)a;
      B[k] = (T)b;
    }
#pragma unroll
    for (int l = 0; l < M; ++l) x[l] = (T)param_x(p, g, l);
#pragma unroll
    for (int i = 0; i < kMaxUserParams; ++i) q[i] = (T)p.params[i];
  }
  __device__ __forceinline__ T value(const T* t) const {
    T y[N];
#pragma unroll
    for (int k = 0; k < N; ++k) y[k] = fmaT(A[k], t[k], B[k]);
    return ::integrand<T>(y, x, q);
  }
};

}  // namespace zmc
