/* zmc_abi_check.c -- the C ABI of libzmc used from plain C: no Python, no
 * torch, only include/zmc.h and libzmc.so.  TEST INFRASTRUCTURE: it also
 * links the oracle (oracle/zmc_oracle.c) to check the results.
 *
 * Without arguments it runs the host-only calls (version, validation,
 * error messages).  With --gpu it also runs, on the current device:
 *   - zmc_scan (host buffers) in both precisions against the oracle;
 *   - zmc_scan_range over a slice, bitwise equal to that slice of zmc_scan;
 *   - a run-time-compiled user integrand, against the same function in C.
 * Exit status 0 when every check holds. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "zmc.h"
#include "zmc_oracle.h"

#define L1 40
#define L2 30
#define G_ALL (L1 * L2)

static int failures = 0;

static void expect(int ok, const char* what) {
  printf("%s %s\n", ok ? "ok  " : "FAIL", what);
  if (!ok) ++failures;
}

/* err_f = |f - f_ref| / max(|f_ref|, sigma_ref sqrt(n)); err_sigma relative */
static void compare(const char* what, const double* f, const double* s, const double* fr,
                    const double* sr, int n, double samples, double tf, double ts) {
  double ef = 0.0, es = 0.0;
  for (int i = 0; i < n; ++i) {
    double scale = fmax(fabs(fr[i]), sr[i] * sqrt(samples));
    double a = fabs(f[i] - fr[i]) / scale, b = fabs(s[i] - sr[i]) / sr[i];
    if (!(a <= ef)) ef = a;
    if (!(b <= es)) es = b;
  }
  char line[256];
  snprintf(line, sizeof(line), "%s: max err_f %.2e (tol %.0e), max err_sigma %.2e (tol %.0e)", what,
           ef, tf, es, ts);
  expect(ef <= tf && es <= ts, line);
}

/* the user integrand of the run-time check, once as HIP source and once in C */
static const char* kSource =
    "template <typename T> __device__ T integrand(const T* y, const T* x, const T* p) {\n"
    "  return exp(-p[0] * x[0] * y[0] * y[0]) * cos(x[1] * y[1] + y[2]);\n"
    "}\n";
static double user_c(const double* y, const double* x, const double* p) {
  return exp(-p[0] * x[0] * y[0] * y[0]) * cos(x[1] * y[1] + y[2]);
}

int main(int argc, char** argv) {
  const int gpu = argc > 1 && strcmp(argv[1], "--gpu") == 0;
  int64_t len[2] = {L1, L2};
  double vals[L1 + L2];
  for (int i = 0; i < L1; ++i) vals[i] = 0.1 + 9.9 * i / (L1 - 1);
  for (int j = 0; j < L2; ++j) vals[L1 + j] = 0.1 + 9.9 * j / (L2 - 1);
  double lo[3] = {0.0, 0.0, 0.0}, hi[3] = {1.0, 1.0, 1.0};
  zmc_scan_desc d;
  memset(&d, 0, sizeof(d));
  d.M = 2;
  d.N = 3;
  d.axis_len = len;
  d.axis_vals = vals;
  d.lo = lo;
  d.hi = hi;
  d.family = ZMC_GAUSS;
  d.precision = ZMC_FP64;
  d.samples = 4099;
  d.seed = 42;

  printf("library: %s\n", zmc_version());
  uint64_t G = 0;
  expect(zmc_validate(&d, &G) == ZMC_OK && G == G_ALL, "zmc_validate: a 40 x 30 GAUSS grid");
  zmc_scan_desc bad = d;
  double hi_bad[3] = {0.0, 1.0, 1.0};
  bad.hi = hi_bad;
  expect(zmc_validate(&bad, NULL) == ZMC_E_INVALID && strstr(zmc_last_error(), "lo >= hi") != NULL,
         "zmc_validate: lo >= hi is ZMC_E_INVALID with a message");
  bad = d;
  bad.samples = 1;
  expect(zmc_validate(&bad, NULL) == ZMC_E_INVALID, "zmc_validate: one sample is ZMC_E_INVALID");
  expect(zmc_scan(NULL, NULL, NULL) == ZMC_E_INVALID, "zmc_scan: NULL descriptor");
  if (!gpu) {
    printf("%s (host-only part)\n", failures ? "FAILED" : "passed");
    return failures ? 1 : 0;
  }

  static double f[G_ALL], s[G_ALL], fr[G_ALL], sr[G_ALL], f2[G_ALL], s2[G_ALL];
  zmc_oracle_spec o;
  memset(&o, 0, sizeof(o));
  o.M = 2;
  o.N = 3;
  o.axis_len = len;
  o.axis_vals = vals;
  o.lo = lo;
  o.hi = hi;
  o.family = ZMC_ORACLE_GAUSS;
  o.samples = d.samples;
  o.seed = d.seed;
  expect(zmc_oracle_scan(&o, NULL, G_ALL, fr, sr) == 0, "oracle scan");

  expect(zmc_scan(&d, f, s) == ZMC_OK, "zmc_scan FP64");
  compare("zmc_scan FP64 vs oracle", f, s, fr, sr, G_ALL, (double)d.samples, 1e-12, 1e-12);
  d.precision = ZMC_FP32_MERGE64;
  expect(zmc_scan(&d, f, s) == ZMC_OK, "zmc_scan FP32");
  compare("zmc_scan FP32 vs oracle", f, s, fr, sr, G_ALL, (double)d.samples, 2e-5, 1e-3);
  expect(zmc_scan_range(&d, 100, 1100, f2, s2, 256) == ZMC_OK, "zmc_scan_range [100, 1100)");
  expect(memcmp(f2, f + 100, 1000 * sizeof(double)) == 0 &&
             memcmp(s2, s + 100, 1000 * sizeof(double)) == 0,
         "zmc_scan_range equals that slice of zmc_scan bit for bit");

  zmc_integrand* h = NULL;
  expect(zmc_integrand_create(kSource, &h) == ZMC_OK && h != NULL, "zmc_integrand_create");
  double p[1] = {0.5};
  d.family = ZMC_USER;
  d.integrand = h;
  d.params = p;
  d.n_params = 1;
  d.precision = ZMC_FP64;
  o.family = ZMC_ORACLE_USER;
  o.user = user_c;
  o.params = p;
  o.n_params = 1;
  expect(zmc_oracle_scan(&o, NULL, G_ALL, fr, sr) == 0, "oracle scan, user function");
  expect(zmc_scan(&d, f, s) == ZMC_OK, "zmc_scan, user integrand FP64");
  compare("user integrand FP64 vs oracle", f, s, fr, sr, G_ALL, (double)d.samples, 1e-12, 1e-12);
  expect(zmc_integrand_destroy(h) == ZMC_OK, "zmc_integrand_destroy");
  printf("%s\n", failures ? "FAILED" : "passed");
  return failures ? 1 : 0;
}
