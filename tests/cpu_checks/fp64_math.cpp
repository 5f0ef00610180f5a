// Host build of the FP64 2^t, sine and cosine of the scan kernels against
// long-double libm on dense grids and at the edges (-inf, +inf, NaN, huge
// arguments, exact powers of two).  Prints "<max rel err exp2> <max rel err sin> <max abs err cos>
// <edge failures>".
#include <math.h>
#include <stdio.h>

#include "zmc_device.hpp"

int main() {
  double worst_e = 0, worst_s = 0, worst_c = 0;
  for (int i = -300000; i <= 300000; ++i) {
    const double t = i * (60.0 / 300000.0);  // 2^t over [-60, 60]
    const long double ref = exp2l((long double)t);
    const double got = zmc::exp2_fp64(t);
    const double e = (double)fabsl(((long double)got - ref) / ref);
    if (e > worst_e) worst_e = e;
    const double r = i * (7.3 / 300000.0);  // phases over +-7.3 revolutions
    // the reference phase in long double after the exact identities
    // sin(2 pi (r - m)) = sin(2 pi r) for whole m and sin(pi - a) = sin(a), so
    // that 2 pi t with |t| <= 1/4 carries no rounding worth counting near the
    // zeros of sin
    long double q = (long double)r - rintl(r);
    if (fabsl(q) > 0.25L) q = copysignl(0.5L, q) - q;
    const long double x = 2.0L * 3.141592653589793238462643383279502884L * q;
    const long double xc = 2.0L * 3.141592653589793238462643383279502884L * ((long double)r - rintl(r));
    const long double rs = sinl(x), rc = cosl(xc);
    const double gs = zmc::sin_turns(r), gc = zmc::cos_turns(r);
    const long double tol = fabsl(rs) > 1e-6L ? fabsl(rs) : 1e-6L;
    const double es = (double)(fabsl((long double)gs - rs) / tol);
    if (es > worst_s) worst_s = es;
    const double ec = (double)fabsl((long double)gc - rc);
    if (ec > worst_c) worst_c = ec;
  }
  int bad = 0;
  bad += !(zmc::exp2_fp64(-INFINITY) == 0.0);
  bad += !(zmc::exp2_fp64(INFINITY) == INFINITY);
  bad += !(zmc::exp2_fp64(NAN) == 0.0);  // the clamp maps NaN to -2100
  bad += !(zmc::exp2_fp64(-1.0e300) == 0.0);
  bad += !(zmc::exp2_fp64(1.0e300) == INFINITY);
  bad += !(zmc::exp2_fp64(0.0) == 1.0);
  bad += !(zmc::exp2_fp64(10.0) == 1024.0);
  bad += !(zmc::exp2_fp64(-1074.0) == ldexp(1.0, -1074));
  bad += !(zmc::exp2_fp64(1023.0) == ldexp(1.0, 1023));
  bad += !(zmc::sin_turns(0.25) == 1.0 && zmc::cos_turns(0.0) == 1.0);
  // the variant for t <= 0 (the Gaussian's -q log2 e)
  for (int i = 0; i <= 100000; ++i) {
    const double t = -i * (60.0 / 100000.0);
    bad += !(zmc::exp2_fp64<true>(t) == zmc::exp2_fp64(t));
  }
  bad += !(zmc::exp2_fp64<true>(-INFINITY) == 0.0 && zmc::exp2_fp64<true>(-1.0e300) == 0.0);
  printf("%.3e %.3e %.3e %d\n", worst_e, worst_s, worst_c, bad);
  return 0;
}
