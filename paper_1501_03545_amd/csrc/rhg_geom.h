// rhg_geom.h -- device helpers shared by the threshold and temperature
// searches: the angle key of the sort, the angle between two points, the
// sorted-position runs of an angular window (through a band's cell
// directory), cosh of the hyperbolic distance in binary64 and in
// double-double, and the keys of the set of pairs decided after a count
// pass.
//
// The distance law is that of Sec. 2.1 in the native representation,
//     cosh d = cosh r_q cosh r_c - sinh r_q sinh r_c cos(dtheta),
// evaluated in the form with non-negative terms
//     cosh d = cosh(r_q - r_c) + 2 sinh r_q sinh r_c sin^2(dtheta/2),
// which has no cancellation.
#pragma once
#include "rhg_internal.h"

namespace rhg {

// The top 32 bits of theta / (2 pi) (the angle part of a sort key).
__device__ __forceinline__ uint32_t angle_key_s(double t)
{
    const double k = t * (4294967296.0 / RHG_TWO_PI_D);
    if (!(k > 0.0)) return 0u;
    if (k >= 4294967295.0) return 4294967295u;
    return (uint32_t)k;
}

// Band of radius r: the largest j with E[j] <= r (exact comparisons).
__device__ __forceinline__ int band_of_r(const double *E, int B, double r)
{
    int lo = 0, hi = B - 1;  // answer in [lo, hi]
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (E[mid] <= r) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Sort key of a point: its band in the top band_bits bits, then the top
// angle bits.  Sorted (key, id) pairs order the index by band, then angle.
__device__ __forceinline__ uint32_t point_key(const double *E, int B, int band_bits, double r, double t)
{
    const uint32_t b = (uint32_t)band_of_r(E, B, r);
    const uint32_t ak = angle_key_s(t);
    return band_bits ? ((b << (32 - band_bits)) | (ak >> band_bits)) : ak;
}

// The FP32 screen record of a point: e^r / sqrt(2 cosh R), e^-r /
// sqrt(2 cosh R), sinh r sqrt(2 / cosh R) (inv = 1 / sqrt(2 cosh R),
// sc = sqrt(2 / cosh R)) and the id as raw bits.
__device__ __forceinline__ float4 point_record(double r, uint32_t id, double inv, double sc)
{
    return make_float4((float)(exp(r) * inv), (float)(exp(-r) * inv), (float)(sinh(r) * sc), __int_as_float((int)id));
}

// Angle between two points the short way round, in [0, pi].
__device__ __forceinline__ double short_angle(double ta, double tb)
{
    double d = fabs(ta - tb);
    if (d > RHG_PI_0) {
        // the long way round: TWO_PI_D - tmax is exact (tmax > pi)
        const double tmax = fmax(ta, tb), tmin = fmin(ta, tb);
        d = ((RHG_TWO_PI_D - tmax) + tmin) + RHG_TWO_PI_RES_D;
    }
    return d;
}

// Sorted-position runs of a band (positions [s, e), 2^cb angular cells whose
// starts are dir[0 .. 2^cb]) covering the angular window [lo, hi] (lo may be
// < 0 and hi >= 2 pi: the window wraps).  Whole cells are taken, so the runs
// may hold points just outside the window.  Returns the number of runs (0,
// 1 or 2) in ascending position order.
__device__ __forceinline__ int cell_runs(const int32_t *dir, int cb, double lo, double hi, int64_t s, int64_t e,
                                         int64_t *ra, int64_t *rb)
{
    if (hi - lo >= RHG_TWO_PI_D) {
        ra[0] = s; rb[0] = e;
        return 1;
    }
    const int shift = 32 - cb;
    const int64_t nc = (int64_t)1 << cb;
    auto cell = [&](double t) -> int64_t { return cb ? (int64_t)(angle_key_s(t) >> shift) : 0; };
    int64_t a0, a1, b0 = 1, b1 = 0;
    if (lo < 0.0) {
        a0 = 0; a1 = cell(hi);
        b0 = cell(lo + RHG_TWO_PI_D); b1 = nc - 1;
    } else if (hi >= RHG_TWO_PI_D) {
        a0 = 0; a1 = cell(hi - RHG_TWO_PI_D);
        b0 = cell(lo); b1 = nc - 1;
    } else {
        a0 = cell(lo); a1 = cell(hi);
    }
    if (b1 >= b0 && b0 <= a1 + 1) {  // the two runs meet
        ra[0] = s; rb[0] = e;
        return 1;
    }
    ra[0] = dir[a0]; rb[0] = dir[a1 + 1];
    if (b1 >= b0) {
        ra[1] = dir[b0]; rb[1] = dir[b1 + 1];
        return 2;
    }
    return 1;
}

// cosh d in binary64 (a few ulps relative).
__device__ __forceinline__ double cosh_dist64(double rq, double tq, double rc, double tc)
{
    const double x = 0.5 * short_angle(tq, tc);
    double s;
    if (x < 0x1p-7) {
        const double x2 = x * x;
        s = x * (1.0 - x2 * (1.0 / 6.0 - x2 * (1.0 / 120.0)));
    } else {
        s = sin(x);
    }
    const double ch = 0.5 * (exp(rq) * exp(-rc) + exp(-rq) * exp(rc));
    return ch + 2.0 * (sinh(rq) * sinh(rc)) * (s * s);
}

// cosh d in double-double, the angle difference formed exactly.
__device__ __forceinline__ dd cosh_dist_dd(double rq, double tq, double rc, double tc)
{
    const double tmax = fmax(tq, tc), tmin = fmin(tq, tc);
    dd d = two_sum(tmax, -tmin);  // exact
    if (dd_cmp(d, dd_make(RHG_PI_0, 1.2246467991473532e-16)) > 0) {
        d = two_sum(RHG_TWO_PI_0 - tmax, tmin);  // RHG_TWO_PI_0 - tmax is exact
        d = dd_add(d, dd_make(RHG_TWO_PI_1, RHG_TWO_PI_2));
    }
    const dd s = dd_sin(dd_mul_pow2(d, 0.5));
    const dd dr = two_sum(rq, -rc);
    return dd_add(dd_cosh(dr),
                  dd_mul_pow2(dd_mul(dd_mul(dd_sinh(dd_make(rq)), dd_sinh(dd_make(rc))), dd_mul(s, s)), 2.0));
}

// A listed pair (query and candidate sorted positions) as a set key: never
// 0, the empty slot.
__device__ __forceinline__ uint64_t pair_key(int64_t q, int64_t c)
{
    return (1ull << 63) | ((uint64_t)(uint32_t)q << 32) | (uint32_t)c;
}

// Slot of a key in the open-addressing set: SplitMix64's finaliser (Steele,
// Lea and Flood, OOPSLA 2014) as the hash.
__device__ __forceinline__ uint64_t slot_hash(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// Exclusive prefix sum of v over the wavefront's 64 lanes (every lane takes
// part); *total is the wavefront's sum.
__device__ __forceinline__ int wave_excl_sum(int v, int lane, int *total)
{
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    *total = __shfl(x, 63, 64);
    return x - v;
}

// The staging slot of a light query at radius r in band j, in units of 4
// words: its row's length, then room for f (mu + 5 sqrt(mu) + 8) entries
// (at most 2^24), mu the query's expected degree (log-linear in r between
// the band's edges E[j], E[j+1] through the plan's log2 values lin[j],
// lout[j]).  The same single-precision hardware steps wherever a slot is
// sized, so that every kernel finds the same slots (the plan's estimate of
// their total allows for the steps' rounding); a wavefront's 64 slots fit
// a 32-bit sum.
__device__ __forceinline__ int stage_slot_quads(const double *E, const float *lin, const float *lout, float f, int j,
                                                double r)
{
    const float w = (float)(E[j + 1] - E[j]);
    const float t = w > 0.0f ? fminf(fmaxf((float)(r - E[j]) * __builtin_amdgcn_rcpf(w), 0.0f), 1.0f) : 0.0f;
    const float mu = __builtin_amdgcn_exp2f(fmaf(t, lout[j] - lin[j], lin[j]));
    const float e = fminf(f * (mu + 5.0f * __builtin_amdgcn_sqrtf(mu) + 8.0f), 16777216.0f);
    return ((int)ceilf(e) + 1 + 3) >> 2;
}

// A staged row's entry whose decision the resolving kernel makes: the
// candidate's id with this bit set, until it becomes the id or
// STAGE_REJECT.
constexpr uint32_t STAGE_PENDING = 0x80000000u;
constexpr int32_t STAGE_REJECT = -1;

}  // namespace rhg
