/* zmc_oracle_cli.c -- command-line front end of the FP64 oracle.
 *
 * TEST INFRASTRUCTURE ONLY: a way to run the oracle (zmc_oracle.c) without
 * Python, e.g. to check single grid points by hand.
 *
 * usage: zmc_oracle_cli SPEC_FILE [G_INDEX ...]
 *
 * SPEC_FILE holds one directive per line ('#' starts a comment):
 *   family  sin_sum | gauss | cosexp | const | linear
 *   samples N                 samples per grid point (>= 2)
 *   seed    S                 Philox key (decimal, 64 bits)
 *   box     LO HI             one line per integration dimension, in order
 *   axis    V1 V2 ...         one line per parameter list, in order
 * It prints "g f sigma" for every grid point, or for the listed flat indices
 * (C order, the last parameter fastest), with 17 significant digits.
 * Exit status: 0 on success, 1 on a malformed spec or argument, 2 when the
 * oracle rejects the scan. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "zmc_oracle.h"

#define MAX_DIMS 16
#define MAX_PARAMS 16

static int family_id(const char* s) {
  static const char* names[] = {"sin_sum", "gauss", "cosexp", "const", "linear"};
  int i;
  for (i = 0; i < 5; ++i)
    if (strcmp(s, names[i]) == 0) return i;
  return -1;
}

int main(int argc, char** argv) {
  FILE* fh;
  char line[1 << 16];
  double lo[MAX_DIMS], hi[MAX_DIMS];
  int64_t axis_len[MAX_PARAMS];
  double* vals = NULL;
  int64_t n_vals = 0, cap = 0;
  zmc_oracle_spec spec;
  uint64_t G, i, n_out;
  uint64_t* idx = NULL;
  double *f, *sigma;
  int rc;

  if (argc < 2) {
    fprintf(stderr, "usage: %s SPEC_FILE [G_INDEX ...]\n", argv[0]);
    return 1;
  }
  memset(&spec, 0, sizeof(spec));
  spec.family = -1;
  fh = fopen(argv[1], "r");
  if (fh == NULL) {
    perror(argv[1]);
    return 1;
  }
  while (fgets(line, sizeof(line), fh) != NULL) {
    char* hash = strchr(line, '#');
    char* tok;
    if (hash) *hash = '\0';
    tok = strtok(line, " \t\r\n");
    if (tok == NULL) continue;
    if (strcmp(tok, "family") == 0) {
      tok = strtok(NULL, " \t\r\n");
      spec.family = tok ? family_id(tok) : -1;
    } else if (strcmp(tok, "samples") == 0) {
      tok = strtok(NULL, " \t\r\n");
      spec.samples = tok ? strtoull(tok, NULL, 10) : 0;
    } else if (strcmp(tok, "seed") == 0) {
      tok = strtok(NULL, " \t\r\n");
      spec.seed = tok ? strtoull(tok, NULL, 10) : 0;
    } else if (strcmp(tok, "box") == 0) {
      char *a = strtok(NULL, " \t\r\n"), *b = strtok(NULL, " \t\r\n");
      if (a == NULL || b == NULL || spec.N >= MAX_DIMS) {
        fprintf(stderr, "bad box line\n");
        return 1;
      }
      lo[spec.N] = strtod(a, NULL);
      hi[spec.N] = strtod(b, NULL);
      spec.N++;
    } else if (strcmp(tok, "axis") == 0) {
      int64_t L = 0;
      if (spec.M >= MAX_PARAMS) {
        fprintf(stderr, "more than %d axes\n", MAX_PARAMS);
        return 1;
      }
      while ((tok = strtok(NULL, " \t\r\n")) != NULL) {
        if (n_vals == cap) {
          cap = cap ? 2 * cap : 1024;
          vals = (double*)realloc(vals, (size_t)cap * sizeof(double));
          if (vals == NULL) return 1;
        }
        vals[n_vals++] = strtod(tok, NULL);
        ++L;
      }
      axis_len[spec.M++] = L;
    } else {
      fprintf(stderr, "unknown directive '%s'\n", tok);
      return 1;
    }
  }
  fclose(fh);
  spec.axis_len = axis_len;
  spec.axis_vals = vals;
  spec.lo = lo;
  spec.hi = hi;
  G = zmc_oracle_grid_size(&spec);
  if (G == 0 || spec.family < 0) {
    fprintf(stderr, "malformed spec (family, axes)\n");
    return 1;
  }
  n_out = argc > 2 ? (uint64_t)(argc - 2) : G;
  if (argc > 2) {
    idx = (uint64_t*)malloc((size_t)n_out * sizeof(uint64_t));
    if (idx == NULL) return 1;
    for (i = 0; i < n_out; ++i) idx[i] = strtoull(argv[2 + i], NULL, 10);
  }
  f = (double*)malloc((size_t)n_out * sizeof(double));
  sigma = (double*)malloc((size_t)n_out * sizeof(double));
  if (f == NULL || sigma == NULL) return 1;
  rc = zmc_oracle_scan(&spec, idx, (int64_t)n_out, f, sigma);
  if (rc != 0) {
    fprintf(stderr, "the oracle rejected the scan (code %d)\n", rc);
    return 2;
  }
  for (i = 0; i < n_out; ++i)
    printf("%llu %.17g %.17g\n", (unsigned long long)(idx ? idx[i] : i), f[i], sigma[i]);
  free(f);
  free(sigma);
  free(idx);
  free(vals);
  return 0;
}
