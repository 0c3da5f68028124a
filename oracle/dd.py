"""Double-double arithmetic for the oracle's phase and node evaluation.

Oracle (test infrastructure only).

Why it is needed.  An entry of K or of a butterfly factor is exp(2 pi i Phi)
with |Phi| up to about 0.6 N, and it depends on Phi only modulo 1.  Plain
float64 carries Phi to about eps |Phi|, i.e. 2e-11 at N = 2^18, which would be
the oracle's own error in every entry.  Here a quantity is carried as a pair
(hi, lo) of float64 arrays whose exact sum is the value to about 2^-104
relative, the integer part of Phi is dropped exactly, and only the final
fraction is rounded to float64.  The entries then carry the rounding of an
O(1) quantity whatever N is.

Methods (published, written here from their definitions):
  two_sum      Knuth's error-free sum (TAOCP vol. 2, 4.2.2): a + b = s + e exactly.
  two_prod     Dekker's error-free product with Veltkamp's splitting
               (Dekker 1971): a * b = p + e exactly (no FMA needed).
  add, mul     double-double sum and product built from those two.
  div, sqrt    one correction step of the quotient / root (Dekker 1971).
  sincos_pi    sin(pi x), cos(pi x): reduction by exact multiples of 1/2, then the
               Taylor series of sin and cos on |theta| <= pi/4, summed by Horner's
               rule in double-double with reciprocal factorials exact to 2^-106.

numpy applies every ufunc elementwise with IEEE round-to-nearest and never
fuses a multiply and an add, which these transformations assume.
"""
from fractions import Fraction
from math import factorial

import numpy as np

_SPLITTER = 134217729.0          # 2^27 + 1

# pi to 64 decimal digits (a published constant), split into a double-double
_PI_DIGITS = "3.1415926535897932384626433832795028841971693993751058209749445923"


def _dd_of_fraction(fr):
    hi = float(fr)
    return hi, float(fr - Fraction(hi))


PI = _dd_of_fraction(Fraction(_PI_DIGITS))

# 1/k! for the Taylor series; (pi/4)^27 / 27! < 1e-33, so 28 terms reach 2^-106
_NTERMS = 28
_INV_FACT = [_dd_of_fraction(Fraction(1, factorial(k))) for k in range(_NTERMS)]


def two_sum(a, b):
    s = a + b
    bb = s - a
    e = (a - (s - bb)) + (b - bb)
    return s, e


def _split(a):
    t = _SPLITTER * a
    hi = t - (t - a)
    return hi, a - hi


def two_prod(a, b):
    p = a * b
    ah, al = _split(a)
    bh, bl = _split(b)
    e = ((ah * bh - p) + ah * bl + al * bh) + al * bl
    return p, e


def as_dd(x):
    """A float64 array (taken as exact) or a (hi, lo) pair -> (hi, lo) pair of float64 arrays."""
    if isinstance(x, tuple):
        return np.asarray(x[0], np.float64), np.asarray(x[1], np.float64)
    x = np.asarray(x, np.float64)
    return x, np.zeros_like(x)


def _norm(s, e):
    return two_sum(s, e)


def add(a, b):
    s, e = two_sum(a[0], b[0])
    return _norm(s, e + (a[1] + b[1]))


def neg(a):
    return -a[0], -a[1]


def sub(a, b):
    return add(a, neg(b))


def mul(a, b):
    p, e = two_prod(a[0], b[0])
    return _norm(p, e + (a[0] * b[1] + a[1] * b[0]))


def scale(a, s):
    """a * s for a power of two s (exact)."""
    return a[0] * s, a[1] * s


def div(a, b):
    q1 = a[0] / b[0]
    r = sub(a, mul((q1, np.zeros_like(q1)), b))
    q2 = r[0] / b[0]
    return _norm(q1, q2)


def sqrt(a):
    """sqrt of a non-negative double-double: s = sqrt(hi), corrected by (a - s^2) / (2 s)."""
    s = np.sqrt(a[0])
    p, e = two_prod(s, s)
    r = ((a[0] - p) - e) + a[1]                 # a[0] - p is exact (p is within an ulp of a[0])
    with np.errstate(divide="ignore", invalid="ignore"):
        corr = np.where(s > 0, r / (2.0 * s), 0.0)
    return two_sum(s, corr)


def absolute(a):
    sgn = np.where(a[0] < 0, -1.0, 1.0)
    return a[0] * sgn, a[1] * sgn


def frac(a):
    """a minus the integer nearest to its high part: a pair in about [-1/2, 1/2].
    hi - rint(hi) is exact in float64 (Sterbenz), so no information is lost."""
    n = np.rint(a[0])
    return two_sum(a[0] - n, a[1])


def to_float(a):
    return a[0] + a[1]


def from_fraction(fr):
    """A Python Fraction (or int) as a double-double scalar pair."""
    hi, lo = _dd_of_fraction(Fraction(fr))
    return np.float64(hi), np.float64(lo)


def sincos_pi(x):
    """(sin(pi x), cos(pi x)) as double-double pairs, for x a double-double pair."""
    x = as_dd(x)
    m = np.rint(2.0 * x[0])                     # x = m/2 + r, |r| <= 1/4
    r = two_sum(x[0] - 0.5 * m, x[1])           # x[0] - m/2 is exact (Sterbenz)
    th = mul(PI, r)
    t2 = mul(th, th)
    zero = np.zeros_like(t2[0])
    # sin th = th * sum_k (-1)^k th^2k / (2k+1)!, cos th = sum_k (-1)^k th^2k / (2k)!
    ks = (_NTERMS - 1) // 2
    s = (zero + _INV_FACT[2 * ks + 1][0] * (-1) ** ks, zero + _INV_FACT[2 * ks + 1][1] * (-1) ** ks)
    c = (zero + _INV_FACT[2 * ks][0] * (-1) ** ks, zero + _INV_FACT[2 * ks][1] * (-1) ** ks)
    for k in range(ks - 1, -1, -1):
        sg = (-1) ** k
        s = add((zero + sg * _INV_FACT[2 * k + 1][0], zero + sg * _INV_FACT[2 * k + 1][1]), mul(s, t2))
        c = add((zero + sg * _INV_FACT[2 * k][0], zero + sg * _INV_FACT[2 * k][1]), mul(c, t2))
    s = mul(s, th)
    q = np.mod(m, 4.0)
    # sin(th + q pi/2), cos(th + q pi/2)
    sin_hi = np.select([q == 0, q == 1, q == 2], [s[0], c[0], -s[0]], -c[0])
    sin_lo = np.select([q == 0, q == 1, q == 2], [s[1], c[1], -s[1]], -c[1])
    cos_hi = np.select([q == 0, q == 1, q == 2], [c[0], -s[0], -c[0]], s[0])
    cos_lo = np.select([q == 0, q == 1, q == 2], [c[1], -s[1], -c[1]], s[1])
    return (sin_hi, sin_lo), (cos_hi, cos_lo)
