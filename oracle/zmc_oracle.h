/*
 * zmc_oracle.h -- plain single-threaded FP64 reference for the direct Monte
 * Carlo parameter scan (ZMCintegral-v5, arXiv:1910.01965).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU library.
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it; the product path never does.  It shares no source,
 * header, table or helper with the GPU library.
 *
 * What it computes (paper, Sec. 2, Eq. (1)): for every point x of an
 * M-dimensional parameter grid, f(x) = integral over an N-dimensional box of
 * g(y; x) dy, estimated by direct (crude) Monte Carlo (paper, Sec. 1 and
 * Sec. 2: no stratified sampling, no heuristic tree search).  The paper names
 * no random number generator and no error estimate; the readings taken here
 * are:
 *   - random words: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel
 *     Random Numbers: As Easy as 1, 2, 3", SC'11), key = seed, counter =
 *     (word block b, grid index g), words packed as w = s*N + k;
 *   - uniform: u = (r + 1/2) * 2^-32, exact in FP64 and inside (0,1);
 *   - estimate: f = V * mean, sigma = V * sqrt(M2 / (n (n-1))) with V the
 *     box volume and M2 the sum of squared deviations (Bessel-corrected
 *     standard error of the mean).
 * Grid flattening is C order: the last parameter varies fastest.
 */
#ifndef ZMC_ORACLE_H
#define ZMC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Integrand families.  SIN_SUM is the paper's test integrand, Eq. (2) and
 * Eq. (4); GAUSS and COSEXP are the two further workload integrands;
 * CONST and LINEAR exist to test the sampler and the estimator. */
enum {
  ZMC_ORACLE_SIN_SUM = 0, /* sin(sum_l x_l + sum_k y_k)                      */
  ZMC_ORACLE_GAUSS = 1,   /* exp(-(sum_{k<=M} x_k y_k^2 + sum_{k>M} y_k^2))  */
  ZMC_ORACLE_COSEXP = 2,  /* cos(x1 y1 + x2 y2 + sum_{k>=3} y_k)
                             * exp(-x3^2 y1 y2) + x4                          */
  ZMC_ORACLE_CONST = 3,   /* 1                                               */
  ZMC_ORACLE_LINEAR = 4,  /* sum_k y_k                                       */
  ZMC_ORACLE_USER = 5     /* user(y, x, p): a user-defined integrand         */
};

/* A user-defined integrand g(y; x) with constants p[0..15] (zero-filled
 * beyond n_params): the paper's user function of a parameter scan (Sec. 2). */
typedef double (*zmc_oracle_user_fn)(const double* y, const double* x,
                                     const double* p);

/* One scan.  All arrays are host memory owned by the caller and read only
 * during a call.  axis_vals holds the M value lists back to back
 * (axis_len[0] values of x_1, then axis_len[1] values of x_2, ...). */
typedef struct zmc_oracle_spec {
  int32_t M;                /* number of parameters, 0..16                  */
  int32_t N;                /* integration dimensions, 1..16                */
  const int64_t* axis_len;  /* [M] list lengths, each >= 1                  */
  const double* axis_vals;  /* [sum axis_len] parameter values              */
  const double* lo;         /* [N] lower box edges                          */
  const double* hi;         /* [N] upper box edges, hi > lo                 */
  int32_t family;           /* ZMC_ORACLE_*                                 */
  uint64_t samples;         /* samples per grid point, >= 2                 */
  uint64_t seed;            /* Philox key                                   */
  zmc_oracle_user_fn user;  /* ZMC_ORACLE_USER only                         */
  const double* params;     /* [n_params] constants for `user`              */
  int32_t n_params;         /* 0..16                                        */
} zmc_oracle_spec;

/* Return codes: 0 = ok, 1 = invalid spec, 2 = out of memory. */

/* One Philox4x32-10 block: out = Philox(ctr, key). */
void zmc_oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                              uint32_t out[4]);

/* Word w of the stream of grid point g: block b = w / 4 with counter
 * (b mod 2^32, b / 2^32, g mod 2^32, g / 2^32), lane w mod 4. */
uint32_t zmc_oracle_word(uint64_t seed, uint64_t g, uint64_t w);

/* Number of grid points G = prod axis_len (1 when M = 0); 0 if invalid. */
uint64_t zmc_oracle_grid_size(const zmc_oracle_spec* spec);

/* Integrand values g(y_s; x) for samples s = s0 .. s0+count-1 of point g. */
int zmc_oracle_values(const zmc_oracle_spec* spec, uint64_t g, uint64_t s0,
                      int64_t count, double* out);

/* Sample mean and M2 = sum (v - mean)^2 of the integrand at point g. */
int zmc_oracle_moments(const zmc_oracle_spec* spec, uint64_t g, double* mean,
                       double* m2);

/* Estimates f and sigma at the n_idx flat grid indices idx[] (all G points
 * in order when idx is NULL, n_idx is then ignored). */
int zmc_oracle_scan(const zmc_oracle_spec* spec, const uint64_t* idx,
                    int64_t n_idx, double* f, double* sigma);

#ifdef __cplusplus
}
#endif

#endif /* ZMC_ORACLE_H */
