// rhg_dd.h -- double-double ("dd") arithmetic for the RHG library.
//
// A dd value is the unevaluated sum hi + lo of two binary64 numbers with
// |lo| <= ulp(hi)/2, about 106 significant bits.  The library uses it where
// binary64 cannot settle a question exactly:
//   * host planning: Eq. (22) is compared with the target degree, and
//     cosh(R), cosh(alpha R) - 1 are formed, to ~1e-30 relative;
//   * the device fallback of the edge test: pairs whose binary64 value lies
//     within a relative 2^-30 of cosh(R) are re-evaluated here.
// The error-free transformations are Knuth's TwoSum and the FMA-based
// TwoProduct; the algorithms follow the standard double-double literature
// (Dekker 1971; Hida, Li, Bailey, "Library for double-double and quad-double
// arithmetic", 2000).  All functions are usable on host and device.  The file
// must be compiled without floating-point contraction (-ffp-contract=off):
// the error-free transformations depend on every operation being rounded.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

namespace rhg {

struct dd {
    double hi, lo;
};

#define RHG_HD __host__ __device__ __forceinline__

RHG_HD dd dd_make(double h, double l = 0.0) { dd r; r.hi = h; r.lo = l; return r; }

RHG_HD dd two_sum(double a, double b)
{
    double s = a + b;
    double bb = s - a;
    double e = (a - (s - bb)) + (b - bb);
    return dd_make(s, e);
}

RHG_HD dd quick_two_sum(double a, double b)  // requires |a| >= |b| or a == 0
{
    double s = a + b;
    double e = b - (s - a);
    return dd_make(s, e);
}

RHG_HD dd two_prod(double a, double b)
{
    double p = a * b;
    double e = fma(a, b, -p);
    return dd_make(p, e);
}

RHG_HD dd dd_add(dd a, dd b)
{
    dd s = two_sum(a.hi, b.hi);
    dd t = two_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = quick_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return quick_two_sum(s.hi, s.lo);
}

RHG_HD dd dd_neg(dd a) { return dd_make(-a.hi, -a.lo); }
RHG_HD dd dd_sub(dd a, dd b) { return dd_add(a, dd_neg(b)); }

RHG_HD dd dd_add_d(dd a, double b)
{
    dd s = two_sum(a.hi, b);
    s.lo += a.lo;
    return quick_two_sum(s.hi, s.lo);
}

RHG_HD dd dd_mul(dd a, dd b)
{
    dd p = two_prod(a.hi, b.hi);
    p.lo += a.hi * b.lo + a.lo * b.hi;
    return quick_two_sum(p.hi, p.lo);
}

RHG_HD dd dd_mul_d(dd a, double b)
{
    dd p = two_prod(a.hi, b);
    p.lo += a.lo * b;
    return quick_two_sum(p.hi, p.lo);
}

RHG_HD dd dd_mul_pow2(dd a, double p2) { return dd_make(a.hi * p2, a.lo * p2); }

RHG_HD dd dd_div(dd a, dd b)
{
    double q1 = a.hi / b.hi;
    dd r = dd_sub(a, dd_mul_d(b, q1));
    double q2 = r.hi / b.hi;
    r = dd_sub(r, dd_mul_d(b, q2));
    double q3 = r.hi / b.hi;
    dd q = quick_two_sum(q1, q2);
    return dd_add_d(q, q3);
}

RHG_HD dd dd_div_d(dd a, double b) { return dd_div(a, dd_make(b)); }

RHG_HD dd dd_sqrt(dd a)
{
    if (a.hi <= 0.0) return dd_make(0.0);
    double x = sqrt(a.hi);
    dd x2 = two_prod(x, x);
    dd d = dd_sub(a, x2);
    return dd_add_d(dd_make(x), d.hi / (2.0 * x));
}

RHG_HD int dd_cmp(dd a, dd b)  // sign of a - b
{
    dd d = dd_sub(a, b);
    return (d.hi > 0.0) - (d.hi < 0.0);
}

// ln 2 and 2*pi to ~160 bits, each split into three binary64 parts.
#define RHG_LN2_0 0.6931471805599453
#define RHG_LN2_1 2.3190468138462996e-17
#define RHG_LN2_2 5.707708438416212e-34
#define RHG_TWO_PI_0 6.283185307179586
#define RHG_TWO_PI_1 2.4492935982947064e-16
#define RHG_TWO_PI_2 (-5.989539619436679e-33)
#define RHG_PI_0 3.141592653589793

// e^x - 1 for |x| <= 2^-9 by its Taylor series, Horner form in dd.
RHG_HD dd dd_expm1_small(dd x)
{
    // 1 + x/2 (1 + x/3 (1 + ... (1 + x/12)))
    dd p = dd_make(1.0);
    for (int k = 12; k >= 2; --k) p = dd_add_d(dd_mul(p, dd_div_d(x, (double)k)), 1.0);
    return dd_mul(p, x);
}

// e^x for |x| < 700: x = k ln2 + t, |t| <= ln2/2, then e^t = (1 + m)^(2^9)
// with m = expm1(t / 2^9), squared nine times as m <- m (2 + m).
RHG_HD dd dd_exp(dd x)
{
    double k = rint(x.hi / RHG_LN2_0);
    dd t = dd_sub(x, two_prod(k, RHG_LN2_0));
    t = dd_sub(t, two_prod(k, RHG_LN2_1));
    t = dd_add_d(t, -k * RHG_LN2_2);
    dd m = dd_expm1_small(dd_mul_pow2(t, 1.0 / 512.0));
    for (int i = 0; i < 9; ++i) m = dd_mul(m, dd_add_d(m, 2.0));
    dd e = dd_add_d(m, 1.0);
    return dd_mul_pow2(e, ldexp(1.0, (int)k));
}

RHG_HD dd dd_cosh(dd x)
{
    dd e = dd_exp(x);
    dd ei = dd_div(dd_make(1.0), e);
    return dd_mul_pow2(dd_add(e, ei), 0.5);
}

// sinh x for x >= 0: series below 1/2 (no cancellation), exponentials above.
RHG_HD dd dd_sinh(dd x)
{
    if (x.hi == 0.0) return dd_make(0.0);
    if (x.hi < 0.5) {
        dd x2 = dd_mul(x, x);
        dd p = dd_make(1.0);  // 1 + x^2/(2*3) (1 + x^2/(4*5) (1 + ...))
        for (int k = 30; k >= 2; k -= 2) p = dd_add_d(dd_mul(p, dd_div_d(x2, (double)(k * (k + 1)))), 1.0);
        return dd_mul(p, x);
    }
    dd e = dd_exp(x);
    dd ei = dd_div(dd_make(1.0), e);
    return dd_mul_pow2(dd_sub(e, ei), 0.5);
}

// sin x for 0 <= x <= pi/2 + tiny by its Taylor series (x^35/35! < 1e-33).
RHG_HD dd dd_sin(dd x)
{
    dd x2 = dd_mul(x, x);
    dd p = dd_make(1.0);
    for (int k = 34; k >= 2; k -= 2) p = dd_sub(dd_make(1.0), dd_mul(p, dd_div_d(x2, (double)(k * (k + 1)))));
    return dd_mul(p, x);
}

// 2 atanh(s) / s - 2 = 2 (s^2/3 + s^4/5 + ...), the first `terms` terms, in
// double-double; the reciprocals 1/(2k+1) are correctly rounded hi/lo pairs.
template <int TERMS>
RHG_HD dd atanh_series(dd s)
{
    constexpr double inv_hi[24] = {
        0x1.0000000000000p+0, 0x1.5555555555555p-2, 0x1.999999999999ap-3, 0x1.2492492492492p-3,
        0x1.c71c71c71c71cp-4, 0x1.745d1745d1746p-4, 0x1.3b13b13b13b14p-4, 0x1.1111111111111p-4,
        0x1.e1e1e1e1e1e1ep-5, 0x1.af286bca1af28p-5, 0x1.8618618618618p-5, 0x1.642c8590b2164p-5,
        0x1.47ae147ae147bp-5, 0x1.2f684bda12f68p-5, 0x1.1a7b9611a7b96p-5, 0x1.0842108421084p-5,
        0x1.f07c1f07c1f08p-6, 0x1.d41d41d41d41dp-6, 0x1.bacf914c1bad0p-6, 0x1.a41a41a41a41ap-6,
        0x1.8f9c18f9c18fap-6, 0x1.7d05f417d05f4p-6, 0x1.6c16c16c16c17p-6, 0x1.5c9882b931057p-6};
    constexpr double inv_lo[24] = {
        0x0.0p+0, 0x1.5555555555555p-56, -0x1.999999999999ap-57, 0x1.2492492492492p-57,
        0x1.c71c71c71c71cp-58, -0x1.745d1745d1746p-59, -0x1.3b13b13b13b14p-58, 0x1.1111111111111p-60,
        0x1.e1e1e1e1e1e1ep-61, 0x1.af286bca1af28p-59, 0x1.8618618618618p-59, 0x1.642c8590b2164p-60,
        -0x1.eb851eb851eb8p-61, 0x1.2f684bda12f68p-59, 0x1.1a7b9611a7b96p-61, 0x1.0842108421084p-60,
        -0x1.f07c1f07c1f08p-61, 0x1.0750750750750p-60, -0x1.bacf914c1bad0p-60, 0x1.0690690690690p-60,
        -0x1.f3831f3831f38p-61, 0x1.7d05f417d05f4p-62, -0x1.f49f49f49f49fp-61, 0x1.310572620ae4cp-61};
    static_assert(TERMS >= 1 && TERMS <= 24, "series length");
    const dd s2 = dd_mul(s, s);
    dd p = dd_make(inv_hi[TERMS - 1], inv_lo[TERMS - 1]);
#pragma unroll
    for (int i = TERMS - 2; i >= 0; --i) p = dd_add(dd_mul(p, s2), dd_make(inv_hi[i], inv_lo[i]));
    return dd_mul_pow2(dd_mul(p, s), 2.0);  // 2 atanh(s)
}

// log(1 + y) for y >= 0 as 2 atanh((z - 1)/(z + 1)), z = 1 + y.  For small y
// the quotient y / (y + 2) keeps full relative accuracy (|s| <= 0.172, 24
// terms).  Otherwise z is scaled by a power of two into [1/sqrt2, sqrt2)
// and its eighth root is taken (three double-double square roots), so that
// |s| <= 0.0217 and 11 terms reach the double-double precision.
RHG_HD dd dd_log1p(dd y)
{
    if (y.hi <= 0.41421356237309503) return atanh_series<24>(dd_div(y, dd_add_d(y, 2.0)));
    dd z = dd_add_d(y, 1.0);
    int e;
    frexp(z.hi, &e);  // z.hi = f * 2^e, f in [1/2, 1)
    dd m = dd_mul_pow2(z, ldexp(1.0, -e));
    if (m.hi < 0.70710678118654757) { m = dd_mul_pow2(m, 2.0); e -= 1; }
    m = dd_sqrt(dd_sqrt(dd_sqrt(m)));
    dd r = dd_mul_pow2(atanh_series<11>(dd_div(dd_add_d(m, -1.0), dd_add_d(m, 1.0))), 8.0);
    const double k = (double)e;
    if (k != 0.0) {
        dd kl = two_prod(k, RHG_LN2_0);
        kl = dd_add(kl, two_prod(k, RHG_LN2_1));
        kl = dd_add_d(kl, k * RHG_LN2_2);
        r = dd_add(r, kl);
    }
    return r;
}

}  // namespace rhg
