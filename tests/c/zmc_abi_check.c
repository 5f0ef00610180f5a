/* zmc_abi_check.c -- the C ABI of libzmc used from plain C: no Python, no
 * torch, only include/zmc.h and libzmc.so.  TEST INFRASTRUCTURE: it also
 * links the oracle (oracle/zmc_oracle.c) to check the results.
 *
 * Without arguments it runs the host-only calls (version, validation,
 * error messages).  With --gpu it also runs, on the current device:
 *   - zmc_scan (host buffers) in both precisions against the oracle;
 *   - zmc_scan_range over a slice, bitwise equal to that slice of zmc_scan;
 *   - a run-time-compiled user integrand, against the same function in C;
 *   - with device buffers from hipMalloc: zmc_scan_device (bitwise equal to
 *     zmc_scan), zmc_scan_batch over three scans of different families and
 *     precisions (against the oracle), and the server on the same three
 *     (bitwise equal to the batch).
 * Exit status 0 when every check holds. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

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

#define NS 3

/* Three scans: the Gaussian grid in FP32, a one-parameter SIN_SUM scan in
 * FP64 on [0,1]^4, and a 5^4-point COSEXP grid in FP32 with a ragged sample
 * count; all through device buffers. */
static void device_checks(const double* gauss_vals, const int64_t* gauss_len) {
  static double sin_vals[50], cos_vals[20];
  static int64_t sin_len[1] = {50}, cos_len[4] = {5, 5, 5, 5};
  for (int i = 0; i < 50; ++i) sin_vals[i] = i / 49.0;
  for (int l = 0; l < 4; ++l)
    for (int i = 0; i < 5; ++i) cos_vals[5 * l + i] = -1.0 + 0.5 * i;
  static double lo3[3] = {0, 0, 0}, hi3[3] = {1, 1, 1}, lo4[4] = {0, 0, 0, 0}, hi4[4] = {1, 1, 1, 1};
  static double lo2[2] = {0, 0}, hi2[2] = {2, 1};
  zmc_scan_desc sc[NS];
  memset(sc, 0, sizeof(sc));
  sc[0].M = 2; sc[0].N = 3; sc[0].axis_len = gauss_len; sc[0].axis_vals = gauss_vals;
  sc[0].lo = lo3; sc[0].hi = hi3; sc[0].family = ZMC_GAUSS; sc[0].precision = ZMC_FP32_MERGE64;
  sc[0].samples = 4099; sc[0].seed = 42;
  sc[1].M = 1; sc[1].N = 4; sc[1].axis_len = sin_len; sc[1].axis_vals = sin_vals;
  sc[1].lo = lo4; sc[1].hi = hi4; sc[1].family = ZMC_SIN_SUM; sc[1].precision = ZMC_FP64;
  sc[1].samples = 2048; sc[1].seed = 7;
  sc[2].M = 4; sc[2].N = 2; sc[2].axis_len = cos_len; sc[2].axis_vals = cos_vals;
  sc[2].lo = lo2; sc[2].hi = hi2; sc[2].family = ZMC_COSEXP; sc[2].precision = ZMC_FP32_MERGE64;
  sc[2].samples = 1001; sc[2].seed = 9;
  const int fam_o[NS] = {ZMC_ORACLE_GAUSS, ZMC_ORACLE_SIN_SUM, ZMC_ORACLE_COSEXP};
  uint64_t G[NS];
  double *d_f[NS], *d_s[NS], *d_f2[NS], *d_s2[NS];
  double *h_f[NS], *h_s[NS], *h_f2[NS], *h_s2[NS], *r_f[NS], *r_s[NS];
  for (int i = 0; i < NS; ++i) {
    expect(zmc_validate(&sc[i], &G[i]) == ZMC_OK, "device scans: valid descriptor");
    const size_t b = G[i] * sizeof(double);
    expect(hipMalloc((void**)&d_f[i], b) == hipSuccess && hipMalloc((void**)&d_s[i], b) == hipSuccess &&
               hipMalloc((void**)&d_f2[i], b) == hipSuccess && hipMalloc((void**)&d_s2[i], b) == hipSuccess,
           "hipMalloc of the outputs");
    h_f[i] = malloc(b); h_s[i] = malloc(b); h_f2[i] = malloc(b); h_s2[i] = malloc(b);
    r_f[i] = malloc(b); r_s[i] = malloc(b);
    zmc_oracle_spec o;
    memset(&o, 0, sizeof(o));
    o.M = sc[i].M; o.N = sc[i].N; o.axis_len = sc[i].axis_len; o.axis_vals = sc[i].axis_vals;
    o.lo = sc[i].lo; o.hi = sc[i].hi; o.family = fam_o[i]; o.samples = sc[i].samples;
    o.seed = sc[i].seed;
    expect(zmc_oracle_scan(&o, NULL, (int64_t)G[i], r_f[i], r_s[i]) == 0, "oracle scan");
  }
  /* one batch, the library staging the lists */
  expect(zmc_scan_batch(sc, NS, NULL, d_f, d_s, NULL) == ZMC_OK, "zmc_scan_batch of three scans");
  for (int i = 0; i < NS; ++i) {
    hipMemcpy(h_f[i], d_f[i], G[i] * 8, hipMemcpyDeviceToHost);
    hipMemcpy(h_s[i], d_s[i], G[i] * 8, hipMemcpyDeviceToHost);
    const int fp64 = sc[i].precision == ZMC_FP64;
    char what[64];
    snprintf(what, sizeof(what), "batched scan %d vs oracle", i);
    compare(what, h_f[i], h_s[i], r_f[i], r_s[i], (int)G[i], (double)sc[i].samples,
            fp64 ? 1e-12 : 2e-5, fp64 ? 1e-12 : 1e-3);
  }
  /* the server on the same scans: bitwise the batch's results */
  zmc_server* srv = NULL;
  expect(zmc_server_create(NULL, &srv) == ZMC_OK, "zmc_server_create");
  uint64_t t[NS];
  for (int i = 0; i < NS; ++i)
    expect(zmc_server_submit(srv, &sc[i], NULL, d_f2[i], d_s2[i], &t[i]) == ZMC_OK, "zmc_server_submit");
  double lat_max = 0.0;
  for (int i = 0; i < NS; ++i) {
    zmc_status st = ZMC_E_DEVICE;
    double lat = -1.0;
    expect(zmc_server_wait(srv, t[i], &st, &lat) == ZMC_OK && st == ZMC_OK && lat >= 0.0,
           "zmc_server_wait: done");
    if (lat > lat_max) lat_max = lat;
  }
  zmc_server_stats ss;
  memset(&ss, 0, sizeof(ss));
  expect(zmc_server_get_stats(srv, &ss) == ZMC_OK && ss.completed == (uint64_t)NS &&
             ss.latency_max_s == lat_max && ss.latency_p50_s > 0.0 &&
             ss.latency_p50_s <= ss.latency_p99_s && ss.latency_p99_s <= ss.latency_max_s &&
             ss.samples_per_s > 0.0,
         "zmc_server_get_stats: counts, latency percentiles, throughput");
  expect(ss.tickets == (uint64_t)NS, "zmc_server_get_stats: every ticket still tracked");
  expect(ss.slice_samples_now == 4000000000ull, "zmc_server_get_stats: default slice budget");
  for (int i = 0; i < NS; ++i)
    expect(zmc_server_release(srv, t[i]) == ZMC_OK, "zmc_server_release of a finished request");
  {
    int32_t done = 0;
    expect(zmc_server_poll(srv, t[0], &done, NULL, NULL) == ZMC_E_INVALID &&
               zmc_server_release(srv, t[0]) == ZMC_E_INVALID,
           "a released ticket is unknown");
    memset(&ss, 0, sizeof(ss));
    expect(zmc_server_get_stats(srv, &ss) == ZMC_OK && ss.tickets == 0 && ss.completed == (uint64_t)NS,
           "zmc_server_get_stats: no ticket tracked after release");
  }
  expect(zmc_server_destroy(srv) == ZMC_OK, "zmc_server_destroy");
  int same = 1;
  for (int i = 0; i < NS; ++i) {
    hipMemcpy(h_f2[i], d_f2[i], G[i] * 8, hipMemcpyDeviceToHost);
    hipMemcpy(h_s2[i], d_s2[i], G[i] * 8, hipMemcpyDeviceToHost);
    same = same && memcmp(h_f2[i], h_f[i], G[i] * 8) == 0 && memcmp(h_s2[i], h_s[i], G[i] * 8) == 0;
  }
  expect(same, "server results equal the batch's bit for bit");
  /* zmc_scan_device with lists on the device: bitwise zmc_scan */
  double* d_axis = NULL;
  expect(hipMalloc((void**)&d_axis, 50 * 8) == hipSuccess &&
             hipMemcpy(d_axis, sin_vals, 50 * 8, hipMemcpyHostToDevice) == hipSuccess,
         "lists on the device");
  expect(zmc_scan_device(&sc[1], d_axis, d_f2[1], d_s2[1], NULL) == ZMC_OK &&
             hipDeviceSynchronize() == hipSuccess, "zmc_scan_device");
  hipMemcpy(h_f2[1], d_f2[1], G[1] * 8, hipMemcpyDeviceToHost);
  hipMemcpy(h_s2[1], d_s2[1], G[1] * 8, hipMemcpyDeviceToHost);
  expect(zmc_scan(&sc[1], h_f[1], h_s[1]) == ZMC_OK, "zmc_scan of the same scan");
  expect(memcmp(h_f2[1], h_f[1], G[1] * 8) == 0 && memcmp(h_s2[1], h_s[1], G[1] * 8) == 0,
         "zmc_scan_device equals zmc_scan bit for bit");
  (void)hipFree(d_axis);
  for (int i = 0; i < NS; ++i) {
    (void)hipFree(d_f[i]); (void)hipFree(d_s[i]); (void)hipFree(d_f2[i]); (void)hipFree(d_s2[i]);
    free(h_f[i]); free(h_s[i]); free(h_f2[i]); free(h_s2[i]); free(r_f[i]); free(r_s[i]);
  }
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
  /* the layouts a binding must mirror */
  printf("sizeof: scan_desc %zu launch_opts %zu plan_info %zu batch_opts %zu batch_info %zu "
         "server_opts %zu server_stats %zu\n",
         sizeof(zmc_scan_desc), sizeof(zmc_launch_opts), sizeof(zmc_plan_info),
         sizeof(zmc_batch_opts), sizeof(zmc_batch_info), sizeof(zmc_server_opts),
         sizeof(zmc_server_stats));
  expect(zmc_server_cancel(NULL, 1) == ZMC_E_INVALID, "zmc_server_cancel: NULL server");
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
  /* the same function with approximate FP32 transcendentals */
  zmc_integrand* hf = NULL;
  expect(zmc_integrand_create_ex(kSource, 2u, &hf) == ZMC_E_INVALID && hf == NULL,
         "zmc_integrand_create_ex refuses unknown flags");
  expect(zmc_integrand_create_ex(kSource, ZMC_INTEGRAND_FAST_MATH, &hf) == ZMC_OK && hf != NULL,
         "zmc_integrand_create_ex, fast math");
  d.integrand = hf;
  d.precision = ZMC_FP32_MERGE64;
  expect(zmc_scan(&d, f, s) == ZMC_OK, "zmc_scan, fast-math user integrand FP32");
  compare("fast-math user integrand FP32 vs oracle", f, s, fr, sr, G_ALL, (double)d.samples, 2e-5,
          1e-3);
  expect(zmc_integrand_destroy(hf) == ZMC_OK, "zmc_integrand_destroy (fast math)");
  expect(zmc_integrand_destroy(h) == ZMC_OK, "zmc_integrand_destroy");
  device_checks(vals, len);
  printf("%s\n", failures ? "FAILED" : "passed");
  return failures ? 1 : 0;
}
