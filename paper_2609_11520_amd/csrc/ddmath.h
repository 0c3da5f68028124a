// Double-double arithmetic for the factor generation (Section 2.2 entries at any N).
//
// A factor entry is exp(2 pi i Phi) times a Lagrange value, and it depends on Phi only
// modulo 1 while |Phi| grows like N (1.6e5 at N = 2^18).  The generators therefore carry
// phases, Chebyshev nodes, c(x) and Lagrange products as unevaluated sums hi + lo of two
// doubles (about 106 bits), drop the integer part of a phase exactly and round once at the
// end, so an entry carries a few roundings of O(1) quantities whatever N is.
//
// Methods: Knuth's error-free sum, the FMA form of the error-free product, one correction
// step for quotients and square roots (Dekker 1971), and sin/cos(pi x) by reduction to
// |x| <= 1/4 followed by their Taylor series summed term by term, each term obtained from the
// previous one by a multiplication and an exact-integer division.  All functions are
// __host__ __device__: the host fills small node tables with the same code.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>

namespace fio {

struct dd {
    double hi, lo;
};

#define FIO_DD_FN __host__ __device__ __forceinline__

FIO_DD_FN dd dd_two_sum(double a, double b) {
#pragma clang fp contract(off)
    const double s = a + b;
    const double bb = s - a;
    return dd{s, (a - (s - bb)) + (b - bb)};
}

FIO_DD_FN dd dd_of(double a) { return dd{a, 0.0}; }
FIO_DD_FN double dd_val(dd a) { return a.hi + a.lo; }
FIO_DD_FN dd dd_neg(dd a) { return dd{-a.hi, -a.lo}; }
// exact scaling by a power of two
FIO_DD_FN dd dd_ldexp(dd a, double p2) { return dd{a.hi * p2, a.lo * p2}; }

FIO_DD_FN dd dd_add(dd a, dd b) {
#pragma clang fp contract(off)
    const dd s = dd_two_sum(a.hi, b.hi);
    return dd_two_sum(s.hi, s.lo + (a.lo + b.lo));
}

FIO_DD_FN dd dd_sub(dd a, dd b) { return dd_add(a, dd_neg(b)); }

FIO_DD_FN dd dd_mul(dd a, dd b) {
#pragma clang fp contract(off)
    const double p = a.hi * b.hi;
    const double e = fma(a.hi, b.hi, -p);          // a.hi * b.hi = p + e exactly
    return dd_two_sum(p, e + (a.hi * b.lo + a.lo * b.hi));
}

FIO_DD_FN dd dd_mul_d(dd a, double b) { return dd_mul(a, dd_of(b)); }

// a / d for a double d
FIO_DD_FN dd dd_div_d(dd a, double d) {
#pragma clang fp contract(off)
    const double q1 = a.hi / d;
    const double p = q1 * d;
    const double e = fma(q1, d, -p);
    const double r = ((a.hi - p) - e) + a.lo;       // a - q1 d
    return dd_two_sum(q1, r / d);
}

FIO_DD_FN dd dd_div(dd a, dd b) {
#pragma clang fp contract(off)
    const double q1 = a.hi / b.hi;
    const dd r = dd_sub(a, dd_mul_d(b, q1));
    return dd_two_sum(q1, r.hi / b.hi);
}

FIO_DD_FN dd dd_sqrt(dd a) {
#pragma clang fp contract(off)
    if (!(a.hi > 0.0)) return dd{0.0, 0.0};
    const double s = sqrt(a.hi);
    const double p = s * s;
    const double e = fma(s, s, -p);
    const double r = ((a.hi - p) - e) + a.lo;       // a - s^2
    return dd_two_sum(s, r / (2.0 * s));
}

FIO_DD_FN dd dd_abs(dd a) { return a.hi < 0.0 ? dd_neg(a) : a; }

// a minus the integer nearest to a.hi (hi - rint(hi) is exact): a value in about [-1/2, 1/2]
FIO_DD_FN dd dd_frac(dd a) {
#pragma clang fp contract(off)
    const double n = rint(a.hi);
    return dd_two_sum(a.hi - n, a.lo);
}

// pi to 106 bits: hi = the double nearest pi, lo = the double nearest pi - hi
constexpr double kPiHi = 3.141592653589793116e+00;
constexpr double kPiLo = 1.224646799147353207e-16;

// sin(pi x) and cos(pi x) for a double-double x
FIO_DD_FN void dd_sincospi(dd x, dd &s, dd &c) {
#pragma clang fp contract(off)
    const double m = rint(2.0 * x.hi);                 // x = m/2 + r, |r| <= 1/4 (+ rounding)
    const dd r = dd_two_sum(x.hi - 0.5 * m, x.lo);     // x.hi - m/2 is exact
    const dd th = dd_mul(dd{kPiHi, kPiLo}, r);
    const dd t2 = dd_mul(th, th);
    // sin th = sum_k (-1)^k th^(2k+1) / (2k+1)!,  cos th = sum_k (-1)^k th^(2k) / (2k)!;
    // |th| <= pi/4 + tiny, so 14 terms each reach 2^-106 relative
    dd ts = th, ss = th, tc = dd_of(1.0), sc = dd_of(1.0);
    for (int k = 1; k <= 14; ++k) {
        ts = dd_div_d(dd_neg(dd_mul(ts, t2)), (double)((2 * k) * (2 * k + 1)));
        tc = dd_div_d(dd_neg(dd_mul(tc, t2)), (double)((2 * k - 1) * (2 * k)));
        ss = dd_add(ss, ts);
        sc = dd_add(sc, tc);
    }
    long long qd = (long long)m % 4;
    if (qd < 0) qd += 4;
    switch (qd) {                                       // sin/cos of th + qd pi/2
        case 0: s = ss; c = sc; break;
        case 1: s = sc; c = dd_neg(ss); break;
        case 2: s = dd_neg(ss); c = dd_neg(sc); break;
        default: s = dd_neg(sc); c = ss; break;
    }
}

FIO_DD_FN dd dd_sinpi(dd x) {
    dd s, c;
    dd_sincospi(x, s, c);
    return s;
}

FIO_DD_FN dd dd_cospi(dd x) {
    dd s, c;
    dd_sincospi(x, s, c);
    return c;
}

// exp(2 pi i f) for a double-double f, rounded once per component
FIO_DD_FN double2 dd_expi2pi(dd f) {
    dd s, c;
    dd_sincospi(dd_ldexp(dd_frac(f), 2.0), s, c);
    double2 e;
    e.x = dd_val(c);
    e.y = dd_val(s);
    return e;
}

// Chebyshev nodes t_i = cos((2i + 1) pi / (2q)) of the first kind on [-1, 1], to 106 bits
constexpr int kMaxQ = 16;
struct Nodes {
    int q;
    double hi[kMaxQ], lo[kMaxQ];
    FIO_DD_FN dd t(int i) const { return dd{hi[i], lo[i]}; }
};

inline Nodes make_nodes(int q) {
    Nodes n{};
    n.q = q;
    for (int i = 0; i < q && i < kMaxQ; ++i) {
        // (2i + 1) / (2q) as a double-double: the quotient and its exact remainder
        const double num = 2.0 * i + 1.0, den = 2.0 * q;
        const dd a = dd_div_d(dd_of(num), den);
        const dd t = dd_cospi(a);
        n.hi[i] = t.hi;
        n.lo[i] = t.lo;
    }
    return n;
}

// Lagrange basis function of node t of the first-kind grid on [-1, 1] at reference coordinate u:
// prod_{k != t} (u - t_k) / (t_t - t_k), all in double-double, rounded once
FIO_DD_FN double dd_lagrange(dd u, int t, const Nodes &n) {
    dd num = dd_of(1.0), den = dd_of(1.0);
    for (int k = 0; k < n.q; ++k) {
        if (k == t) continue;
        num = dd_mul(num, dd_sub(u, n.t(k)));
        den = dd_mul(den, dd_sub(n.t(t), n.t(k)));
    }
    return dd_val(dd_div(num, den));
}

#undef FIO_DD_FN
}  // namespace fio
