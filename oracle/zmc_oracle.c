/*
 * zmc_oracle.c -- plain single-threaded FP64 reference for the direct Monte
 * Carlo parameter scan (ZMCintegral-v5, arXiv:1910.01965, Sec. 2).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg, never by the product path.  No blocking,
 * fusion or reordering: each function takes the steps of the definition in
 * order so that it can be read against the paper.
 *
 * Build: cc -std=c99 -O2 -fPIC -shared (ISO mode: no FMA contraction, so
 * every fma below is the only fused operation).
 */
#include "zmc_oracle.h"

#include <math.h>
#include <stdlib.h>

#define ORACLE_OK 0
#define ORACLE_INVALID 1
#define ORACLE_NOMEM 2

/* ------------------------------------------------------------------------
 * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11, Sec. 4.2).
 * A round multiplies words 0 and 2 by the two Philox multipliers, and the
 * new state is (hi(M1*R2) ^ R1 ^ k0, lo(M1*R2), hi(M0*R0) ^ R3 ^ k1,
 * lo(M0*R0)).  The key is bumped by the two Weyl constants between rounds.
 * ---------------------------------------------------------------------- */
static const uint32_t PHILOX_M0 = 0xD2511F53u;
static const uint32_t PHILOX_M1 = 0xCD9E8D57u;
static const uint32_t PHILOX_W0 = 0x9E3779B9u; /* golden ratio           */
static const uint32_t PHILOX_W1 = 0xBB67AE85u; /* sqrt(3) - 1            */

void zmc_oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                              uint32_t out[4]) {
  uint32_t r0 = ctr[0], r1 = ctr[1], r2 = ctr[2], r3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  int round;
  for (round = 0; round < 10; ++round) {
    uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)r0;
    uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)r2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ r1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ r3 ^ k1;
    uint32_t n3 = lo0;
    r0 = n0; r1 = n1; r2 = n2; r3 = n3;
    if (round < 9) {
      k0 += PHILOX_W0;
      k1 += PHILOX_W1;
    }
  }
  out[0] = r0; out[1] = r1; out[2] = r2; out[3] = r3;
}

uint32_t zmc_oracle_word(uint64_t seed, uint64_t g, uint64_t w) {
  uint64_t b = w / 4u;
  uint32_t ctr[4], key[2], out[4];
  ctr[0] = (uint32_t)b;
  ctr[1] = (uint32_t)(b >> 32);
  ctr[2] = (uint32_t)g;
  ctr[3] = (uint32_t)(g >> 32);
  key[0] = (uint32_t)seed;
  key[1] = (uint32_t)(seed >> 32);
  zmc_oracle_philox4x32_10(ctr, key, out);
  return out[w % 4u];
}

/* ------------------------------------------------------------------------
 * Scan description checks.
 * ---------------------------------------------------------------------- */
uint64_t zmc_oracle_grid_size(const zmc_oracle_spec* spec) {
  uint64_t G = 1;
  int l;
  if (spec == NULL || spec->M < 0 || spec->M > 16) return 0;
  if (spec->M > 0 && (spec->axis_len == NULL || spec->axis_vals == NULL))
    return 0;
  for (l = 0; l < spec->M; ++l) {
    int64_t L = spec->axis_len[l];
    if (L < 1) return 0;
    if (G > ((uint64_t)1 << 62) / (uint64_t)L) return 0;
    G *= (uint64_t)L;
  }
  return G;
}

static int spec_ok(const zmc_oracle_spec* spec) {
  int k;
  if (zmc_oracle_grid_size(spec) == 0) return 0;
  if (spec->N < 1 || spec->N > 16) return 0;
  if (spec->lo == NULL || spec->hi == NULL) return 0;
  for (k = 0; k < spec->N; ++k) {
    if (!isfinite(spec->lo[k]) || !isfinite(spec->hi[k])) return 0;
    if (!(spec->lo[k] < spec->hi[k])) return 0;
  }
  if (spec->samples < 2) return 0;
  switch (spec->family) {
    case ZMC_ORACLE_SIN_SUM: break;
    case ZMC_ORACLE_GAUSS: if (spec->M > spec->N) return 0; break;
    case ZMC_ORACLE_COSEXP: if (spec->M != 4 || spec->N < 2) return 0; break;
    case ZMC_ORACLE_CONST: break;
    case ZMC_ORACLE_LINEAR: break;
    case ZMC_ORACLE_USER:
      if (spec->user == NULL) return 0;
      if (spec->n_params < 0 || spec->n_params > 16) return 0;
      if (spec->n_params > 0 && spec->params == NULL) return 0;
      break;
    default: return 0;
  }
  return 1;
}

/* Grid point g -> parameter vector x, C order (last parameter fastest),
 * x_l taken from the l-th value list (paper, Sec. 2: each parameter runs over
 * its own list; the result is a multi-dimensional grid). */
static void decode_point(const zmc_oracle_spec* spec, uint64_t g, double* x) {
  int64_t off[16];
  int64_t acc = 0;
  int l;
  for (l = 0; l < spec->M; ++l) {
    off[l] = acc;
    acc += spec->axis_len[l];
  }
  for (l = spec->M - 1; l >= 0; --l) {
    uint64_t L = (uint64_t)spec->axis_len[l];
    uint64_t i = g % L;
    g = g / L;
    x[l] = spec->axis_vals[off[l] + (int64_t)i];
  }
}

/* ------------------------------------------------------------------------
 * The integrand g(y; x).  y and x are 0-based arrays: y[0] is y_1.
 * ---------------------------------------------------------------------- */
static double integrand(const zmc_oracle_spec* spec, const double* x,
                        const double* y) {
  const int M = spec->M, N = spec->N;
  int k, l;
  switch (spec->family) {
    case ZMC_ORACLE_SIN_SUM: {
      /* paper Eq. (2) / Eq. (4): sin(sum_j y_j + sum_l x_l) */
      double sx = 0.0, sy = 0.0;
      for (l = 0; l < M; ++l) sx += x[l];
      for (k = 0; k < N; ++k) sy += y[k];
      return sin(sx + sy);
    }
    case ZMC_ORACLE_GAUSS: {
      double q = 0.0;
      for (k = 0; k < N; ++k) {
        double c = (k < M) ? x[k] : 1.0;
        q += c * y[k] * y[k];
      }
      return exp(-q);
    }
    case ZMC_ORACLE_COSEXP: {
      double phase = x[0] * y[0] + x[1] * y[1];
      for (k = 2; k < N; ++k) phase += y[k];
      return cos(phase) * exp(-(x[2] * x[2]) * y[0] * y[1]) + x[3];
    }
    case ZMC_ORACLE_CONST:
      return 1.0;
    case ZMC_ORACLE_LINEAR: {
      double s = 0.0;
      for (k = 0; k < N; ++k) s += y[k];
      return s;
    }
    case ZMC_ORACLE_USER: {
      double p[16];
      for (k = 0; k < 16; ++k) p[k] = (k < spec->n_params) ? spec->params[k] : 0.0;
      return spec->user(y, x, p);
    }
    default:
      return NAN;
  }
}

/* ------------------------------------------------------------------------
 * Samples: word w = s*N + k of point g gives coordinate k of sample s,
 * u = (r + 1/2) 2^-32 in (0,1), y_k = lo_k + (hi_k - lo_k) u as one fma.
 * ---------------------------------------------------------------------- */
int zmc_oracle_values(const zmc_oracle_spec* spec, uint64_t g, uint64_t s0,
                      int64_t count, double* out) {
  double x[16], y[16];
  uint32_t ctr[4], key[2], block[4];
  uint64_t cached_b = 0;
  int have_block = 0;
  int64_t i;
  int k;
  if (!spec_ok(spec) || out == NULL || count < 0) return ORACLE_INVALID;
  if (g >= zmc_oracle_grid_size(spec)) return ORACLE_INVALID;
  decode_point(spec, g, x);
  key[0] = (uint32_t)spec->seed;
  key[1] = (uint32_t)(spec->seed >> 32);
  for (i = 0; i < count; ++i) {
    uint64_t s = s0 + (uint64_t)i;
    for (k = 0; k < spec->N; ++k) {
      uint64_t w = s * (uint64_t)spec->N + (uint64_t)k;
      uint64_t b = w / 4u;
      uint32_t r;
      /* same word as zmc_oracle_word(seed, g, w); one block serves four
       * consecutive words */
      if (!have_block || b != cached_b) {
        ctr[0] = (uint32_t)b;
        ctr[1] = (uint32_t)(b >> 32);
        ctr[2] = (uint32_t)g;
        ctr[3] = (uint32_t)(g >> 32);
        zmc_oracle_philox4x32_10(ctr, key, block);
        cached_b = b;
        have_block = 1;
      }
      r = block[w % 4u];
      double u = ((double)r + 0.5) * 0x1p-32;
      double h = spec->hi[k] - spec->lo[k];
      y[k] = fma(h, u, spec->lo[k]);
    }
    out[i] = integrand(spec, x, y);
  }
  return ORACLE_OK;
}

/* ------------------------------------------------------------------------
 * Estimator: Neumaier-compensated sums; mean = sum(v) / n, then the
 * corrected two-pass sum of squares M2 = sum (v-mean)^2 - (sum (v-mean))^2/n
 * (Chan, Golub, LeVeque, "Algorithms for computing the sample variance",
 * Am. Stat. 1983).
 * ---------------------------------------------------------------------- */
typedef struct { double s, c; } neumaier;

static void nsum_add(neumaier* a, double v) {
  double t = a->s + v;
  if (fabs(a->s) >= fabs(v))
    a->c += (a->s - t) + v;
  else
    a->c += (v - t) + a->s;
  a->s = t;
}

static double nsum_value(const neumaier* a) { return a->s + a->c; }

int zmc_oracle_moments(const zmc_oracle_spec* spec, uint64_t g, double* mean,
                       double* m2) {
  uint64_t n, s;
  double* v;
  neumaier sum = {0.0, 0.0}, dev = {0.0, 0.0}, sq = {0.0, 0.0};
  double mu, d, corr;
  int rc;
  if (!spec_ok(spec)) return ORACLE_INVALID;
  n = spec->samples;
  v = (double*)malloc(sizeof(double) * (size_t)n);
  if (v == NULL) return ORACLE_NOMEM;
  rc = zmc_oracle_values(spec, g, 0, (int64_t)n, v);
  if (rc != ORACLE_OK) { free(v); return rc; }
  for (s = 0; s < n; ++s) nsum_add(&sum, v[s]);
  mu = nsum_value(&sum) / (double)n;
  for (s = 0; s < n; ++s) {
    d = v[s] - mu;
    nsum_add(&dev, d);
    nsum_add(&sq, d * d);
  }
  corr = nsum_value(&dev);
  *mean = mu;
  *m2 = nsum_value(&sq) - corr * corr / (double)n;
  if (*m2 < 0.0) *m2 = 0.0;
  free(v);
  return ORACLE_OK;
}

int zmc_oracle_scan(const zmc_oracle_spec* spec, const uint64_t* idx,
                    int64_t n_idx, double* f, double* sigma) {
  uint64_t G, n;
  double V = 1.0;
  int64_t i, count;
  int k, rc;
  if (!spec_ok(spec) || f == NULL || sigma == NULL) return ORACLE_INVALID;
  G = zmc_oracle_grid_size(spec);
  n = spec->samples;
  for (k = 0; k < spec->N; ++k) V *= spec->hi[k] - spec->lo[k];
  count = (idx == NULL) ? (int64_t)G : n_idx;
  for (i = 0; i < count; ++i) {
    uint64_t g = (idx == NULL) ? (uint64_t)i : idx[i];
    double mean, m2;
    if (g >= G) return ORACLE_INVALID;
    rc = zmc_oracle_moments(spec, g, &mean, &m2);
    if (rc != ORACLE_OK) return rc;
    f[i] = V * mean;
    sigma[i] = V * sqrt(m2 / ((double)n * (double)(n - 1)));
  }
  return ORACLE_OK;
}
