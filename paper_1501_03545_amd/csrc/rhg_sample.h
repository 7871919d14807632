// rhg_sample.h -- the per-point draw of the sampler (Algorithm 1, angular
// and radial draws), shared by the sampling kernel and the batch kernel that
// generates small graphs in one workgroup.
//
// Vertex i draws its two uniforms from Philox4x32-10 (Salmon, Moraes, Dror,
// Shaw, SC'11) with counter (i_lo, i_hi, 0, 0) and key (seed_lo, seed_hi):
// one 128-bit block gives two 53-bit uniforms.  The angle is uniform on
// [0, 2 pi) and the radius follows Eq. (1) by inverting its CDF
// F(r) = (cosh(alpha r) - 1) / (cosh(alpha R) - 1) (Appendix C with the full
// angular range): r = acosh(1 + u (cosh(alpha R) - 1)) / alpha, evaluated as
// log1p(x + sqrt(x (x + 2))) / alpha with x = u (cosh(alpha R) - 1), which
// keeps full relative accuracy for small u.  The radius is evaluated in
// double-double (about 104 bits: log1p by a table of log(k / 128) and a short
// atanh series) and rounded once, so it is the correctly rounded binary64
// value unless the exact radius lies within about 2^-100 (relative) of a
// rounding boundary.
#pragma once
#include "rhg_internal.h"
#include "rhg_philox.h"

namespace rhg {

// log(1 + y) for y >= 0 in double-double with a table: 1 + y = 2^e m with m
// in [1/sqrt2, sqrt2), m = t (1 + s') for the nearest t = k / 128, and
// log m = log t + 2 atanh(s), s = (m - t) / (m + t), |s| < 2^-8.5, so seven
// terms of the series reach the double-double precision.  The table
// log(k / 128), k = 90 .. 181, is computed by each workgroup with the
// series routine (dd_log1p) before it samples.
constexpr int LOGT_K0 = 90, LOGT_N = 92;

__device__ __forceinline__ dd log1p_table(dd y, const dd *tab)
{
    if (y.hi <= 0.41421356237309503) return dd_log1p(y);
    dd z = dd_add_d(y, 1.0);
    int e;
    frexp(z.hi, &e);
    dd m = dd_mul_pow2(z, ldexp(1.0, -e));
    if (m.hi < 0.70710678118654757) {
        m = dd_mul_pow2(m, 2.0);
        e -= 1;
    }
    int k = (int)rint(m.hi * 128.0);
    k = min(max(k, LOGT_K0), LOGT_K0 + LOGT_N - 1);
    const double t = (double)k * 0.0078125;  // exact
    const dd sq = dd_div(dd_add_d(m, -t), dd_add_d(m, t));
    dd r = dd_add(tab[k - LOGT_K0], atanh_series<7>(sq));
    const double kk = (double)e;
    if (kk != 0.0) {
        dd kl = two_prod(kk, RHG_LN2_0);
        kl = dd_add(kl, two_prod(kk, RHG_LN2_1));
        kl = dd_add_d(kl, kk * RHG_LN2_2);
        r = dd_add(r, kl);
    }
    return r;
}

// The table log(k / 128), k = LOGT_K0 .. LOGT_K0 + LOGT_N - 1, filled by the
// threads of a workgroup (the caller synchronises before using it).
__device__ __forceinline__ void fill_log_table(dd *tab, int tid, int nthreads)
{
    for (int k = tid; k < LOGT_N; k += nthreads)
        tab[k] = dd_log1p(dd_make((double)(k + LOGT_K0) * 0.0078125 - 1.0));  // log(k / 128), exact argument
}

// Point i of the graph with Philox key (k0, k1), alpha, R and
// cosh(alpha R) - 1 = c + c_lo.
__device__ __forceinline__ void sample_point(int64_t i, uint32_t k0, uint32_t k1, double alpha, double R, double c,
                                             double c_lo, const dd *tab, double *r_out, double *theta_out)
{
    uint32_t x0 = (uint32_t)(uint64_t)i, x1 = (uint32_t)((uint64_t)i >> 32), x2 = 0u, x3 = 0u;
    philox4x32_10(x0, x1, x2, x3, k0, k1);
    const uint64_t a = ((uint64_t)x1 << 32) | x0;
    const uint64_t b = ((uint64_t)x3 << 32) | x2;
    const double ut = (double)(a >> 11) * 0x1p-53;
    const double ur = (double)(b >> 11) * 0x1p-53;
    *theta_out = RHG_TWO_PI_D * ut;
    const dd x = dd_mul_d(dd_make(c, c_lo), ur);
    const dd y = dd_add(x, dd_sqrt(dd_mul(x, dd_add_d(x, 2.0))));
    const dd ri = dd_div_d(log1p_table(y, tab), alpha);
    *r_out = fmin(ri.hi, R);  // the exact value is <= R
}

}  // namespace rhg
