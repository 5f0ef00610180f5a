"""Coefficients of the FP64 polynomials in csrc/zmc_device.hpp.

Both come from Chebyshev economization (Lanczos) of a Taylor series: the
series is taken to degree 34 in exact rational arithmetic (pi and ln 2 to 60
digits), rewritten in the Chebyshev basis of the interval, cut after the
stated degree (the dropped Chebyshev coefficients bound the truncation
error), rewritten in powers of the argument and rounded to double.

  exp2:  2^f = sum_{n=0..11} e_n f^n          for f in [-1/2, 1/2]
  sin:   sin(2 pi v) = v sum_{k=0..8} s_k v^(2k)  for v in [-1/4, 1/4]

Run `python -m paper_1910_01965_amd.fp64_poly` to print the constants and
the largest relative error of the double-precision Horner evaluation on a
dense grid against a 60-digit reference.
"""
import math
from decimal import Decimal, getcontext
from fractions import Fraction as Fr

getcontext().prec = 60
LN2 = Fr(Decimal(2).ln())
PI = Fr(Decimal("3.14159265358979323846264338327950288419716939937510582097494459"))
DEGREE_TAYLOR = 34


def _economize(a, d):
    """Power coefficients a (argument x in [-1, 1]) cut to degree d through the
    Chebyshev basis; returns (power coefficients of degree d, bound on the
    dropped part)."""
    D = len(a) - 1
    c = [Fr(0)] * (D + 1)
    for n, an in enumerate(a):  # x^n = 2^(1-n) sum_j C(n, j) T_(n-2j), T_0 halved
        if an == 0:
            continue
        for j in range(n // 2 + 1):
            k = n - 2 * j
            w = Fr(math.comb(n, j), 2 ** (n - 1)) if n > 0 else Fr(1)
            if k == 0 and n > 0:
                w /= 2
            c[k] += an * w
    dropped = sum(abs(x) for x in c[d + 1:])
    T = [[Fr(1)], [Fr(0), Fr(1)]]
    for k in range(2, d + 1):
        t = [Fr(0)] * (k + 1)
        for i, v in enumerate(T[k - 1]):
            t[i + 1] += 2 * v
        for i, v in enumerate(T[k - 2]):
            t[i] -= v
        T.append(t)
    p = [Fr(0)] * (d + 1)
    for k in range(d + 1):
        for i, v in enumerate(T[k]):
            p[i] += c[k] * v
    return p, dropped


def exp2_coefficients(degree=11):
    """e_0..e_degree of 2^f on [-1/2, 1/2] (f = x / 2)."""
    a = [(LN2 / 2) ** n / math.factorial(n) for n in range(DEGREE_TAYLOR + 1)]
    p, dropped = _economize(a, degree)
    return [float(pn * 2 ** n) for n, pn in enumerate(p)], float(dropped)


def sin_coefficients(degree=17):
    """s_0..s_(degree//2) of sin(2 pi v) = v sum_k s_k v^(2k) on [-1/4, 1/4]
    (v = x / 4, sin(pi x / 2))."""
    a = [Fr(0)] * (DEGREE_TAYLOR + 1)
    for n in range(1, DEGREE_TAYLOR + 1, 2):
        a[n] = (-1) ** ((n - 1) // 2) * (PI / 2) ** n / math.factorial(n)
    p, dropped = _economize(a, degree)
    return [float(p[2 * k + 1] * 4 ** (2 * k + 1)) for k in range(degree // 2 + 1)], float(dropped)


def _fma(a, b, c):
    """a * b + c rounded once to double, as the device's fma."""
    return float(Fr(a) * Fr(b) + Fr(c))


def _horner(coef, x):
    r = coef[-1]
    for c in reversed(coef[:-1]):
        r = _fma(r, x, c)
    return r


def main():
    e, de = exp2_coefficients()
    s, ds = sin_coefficients()
    print(f"// exp2: degree {len(e) - 1}, dropped Chebyshev terms {de:.2e}")
    for n, c in enumerate(e):
        print(f"  e{n} = {c!r}")
    print(f"// sin(2 pi v) / v: {len(s)} terms, dropped Chebyshev terms {ds:.2e}")
    for k, c in enumerate(s):
        print(f"  s{k} = {c!r}")
    worst_e = worst_s = 0.0
    pi = Decimal(PI.numerator) / Decimal(PI.denominator)
    for i in range(-4000, 4001):
        f = i / 8000.0
        ref = Decimal(2) ** Decimal(f)
        got = _horner(e, f)
        worst_e = max(worst_e, abs((Decimal(got) - ref) / ref))
        v = i / 16000.0
        if v != 0.0:
            ref_s = _dsin(2 * pi * Decimal(v))
            got_s = v * _horner(s, v * v)
            worst_s = max(worst_s, abs((Decimal(got_s) - ref_s) / ref_s))
    print(f"max relative error: exp2 {float(worst_e):.3e}, sin {float(worst_s):.3e}")


def _dsin(x):
    """sin of a Decimal by its Taylor series (|x| <= pi / 2)."""
    term, total, n = x, x, 1
    while abs(term) > Decimal(10) ** -55:
        term = -term * x * x / ((2 * n) * (2 * n + 1))
        total += term
        n += 1
    return total


if __name__ == "__main__":
    main()
