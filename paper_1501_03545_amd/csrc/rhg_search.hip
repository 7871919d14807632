// rhg_search.hip -- the neighbour search (Algorithm 1, the parallel query
// loop over vertices; range query of Sec. 3.2).
//
// For a query q and a radial band j the paper's Euclidean query circle of
// Proposition 1 becomes, in native coordinates, an angular window around
// theta_q: a point at radius r and angle difference dtheta is a neighbour iff
//     sin^2(dtheta/2) <= (cosh R - cosh(r_q - r)) / (2 sinh r_q sinh r),
// and the right side decreases in r (its derivative has the sign of
// cosh R cosh r - cosh r_q >= 0), so the window computed at the band's inner
// edge E[j] covers every point of the band.  Bands with r_q + E[j+1] <= R lie
// wholly inside the circle (triangle inequality) and are taken without tests.
//
// Each candidate is decided exactly on its binary64 coordinates:
//   1. FP64: cosh d = cosh(r_q - r_c) + 2 sinh r_q sinh r_c sin^2(dtheta/2)
//      from per-point e^r, e^-r, sinh r and a per-pair half-angle sine (a
//      Taylor polynomial below 2^-7, where sin x / x is within 5e-17 of it);
//      every term is non-negative, so the relative error is a few ulp.
//      Values further than a relative 2^-30 from cosh R are final.
//   2. Double-double re-evaluation of the same formula from r and theta for
//      the rest (expected: a handful of pairs per graph).
#include "rhg_internal.h"

namespace rhg {

struct SearchArgs {
    double E[RHG_MAX_BANDS + 1];       // band edges
    double e_lo[RHG_MAX_BANDS];        // e^{E[j]}
    double em_lo[RHG_MAX_BANDS];       // e^{-E[j]}
    double sh_lo[RHG_MAX_BANDS];       // sinh(E[j])
    int64_t dir_base[RHG_MAX_BANDS + 1];
    int cbits[RHG_MAX_BANDS];
    int B;
    int band_bits;
    int64_t n;
    double R;
    double C;        // cosh R (binary64)
    double C_lo;     // double-double tail of cosh R
    double acc_thr;  // C (1 - 2^-30): below is certainly an edge
    double rej_thr;  // C (1 + 2^-30): above is certainly not
    const int32_t *band_start;
    const int32_t *dir;
    const double *sr, *st, *sep, *sem, *ssh;
    const int32_t *sid;
    unsigned long long *stats;
};

__device__ __forceinline__ uint32_t angle_key_s(double t)
{
    const double k = t * (4294967296.0 / RHG_TWO_PI_D);
    if (!(k > 0.0)) return 0u;
    if (k >= 4294967295.0) return 4294967295u;
    return (uint32_t)k;
}

// Angle between two points taken the short way round, in [0, pi].
__device__ __forceinline__ double short_angle(double ta, double tb)
{
    const double tmax = fmax(ta, tb), tmin = fmin(ta, tb);
    double d = tmax - tmin;
    // the long way round: TWO_PI_D - tmax is exact (tmax > pi)
    if (d > RHG_PI_0) d = ((RHG_TWO_PI_D - tmax) + tmin) + RHG_TWO_PI_RES_D;
    return d;
}

__device__ __noinline__ int edge_dd(double rq, double tq, double rc, double tc, double C, double C_lo,
                                    unsigned long long *stats)
{
    atomicAdd(&stats[ST_DD], 1ull);
    const double tmax = fmax(tq, tc), tmin = fmin(tq, tc);
    dd d = two_sum(tmax, -tmin);  // exact
    if (dd_cmp(d, dd_make(RHG_PI_0, 1.2246467991473532e-16)) > 0) {
        d = two_sum(RHG_TWO_PI_0 - tmax, tmin);  // RHG_TWO_PI_0 - tmax is exact
        d = dd_add(d, dd_make(RHG_TWO_PI_1, RHG_TWO_PI_2));
    }
    const dd s = dd_sin(dd_mul_pow2(d, 0.5));
    const dd dr = two_sum(rq, -rc);
    const dd L = dd_add(dd_cosh(dr), dd_mul_pow2(dd_mul(dd_mul(dd_sinh(dd_make(rq)), dd_sinh(dd_make(rc))),
                                                        dd_mul(s, s)),
                                                 2.0));
    const dd diff = dd_sub(L, dd_make(C, C_lo));
    if (fabs(diff.hi) <= 1e-26 * C) atomicAdd(&stats[ST_TIES], 1ull);
    return diff.hi <= 0.0;
}

struct Query {
    double r, t, ep, em, sh;
    int64_t p;
};

__device__ __forceinline__ int edge_test(const SearchArgs &A, const Query &q, int64_t c)
{
    const double tc = A.st[c];
    const double d = short_angle(q.t, tc);
    const double x = 0.5 * d;
    double s;
    if (x < 0x1p-7) {
        const double x2 = x * x;
        s = x * (1.0 - x2 * (1.0 / 6.0 - x2 * (1.0 / 120.0)));
    } else {
        s = sin(x);
    }
    const double ch = 0.5 * (q.ep * A.sem[c] + q.em * A.sep[c]);
    const double L = ch + 2.0 * (q.sh * A.ssh[c]) * (s * s);
    if (L < A.acc_thr) return 1;
    if (L > A.rej_thr) return 0;
    return edge_dd(q.r, q.t, A.sr[c], tc, A.C, A.C_lo, A.stats);
}

// Does every point of band j (r < E[j+1], or r <= R for the last band) lie
// within distance R of q?  Exact: r_q + E[j+1] <= R tested with TwoSum.
__device__ __forceinline__ bool band_inside(const SearchArgs &A, double rq, int j)
{
    const dd s = two_sum(rq, A.E[j + 1]);
    return s.hi < A.R || (s.hi == A.R && s.lo <= 0.0);
}

// Half-width of the angular window of band j for query q (conservative),
// or a value >= pi when the whole band must be scanned.
__device__ __forceinline__ double window_half_width(const SearchArgs &A, const Query &q, int j)
{
    if (A.sh_lo[j] == 0.0 || q.sh == 0.0) return 4.0;
    const double chd = 0.5 * (q.ep * A.em_lo[j] + q.em * A.e_lo[j]);  // cosh(r_q - E[j])
    const double X = (A.C - chd) / (2.0 * q.sh * A.sh_lo[j]);
    if (X >= 0.999999) return 4.0;
    const double tm = 2.0 * asin(sqrt(fmax(X, 0.0)));
    return tm * (1.0 + 0x1p-20) + 0x1p-40;
}

// Tests candidates [a, b) in sorted order.  In the emit pass `lim` is the
// row length found by the count pass; writes beyond it are dropped (and
// reported) instead of running past the row.
template <bool EMIT>
__device__ __forceinline__ void scan_range(const SearchArgs &A, const Query &q, int64_t a, int64_t b,
                                           int64_t &cnt, int32_t *out, int64_t lim)
{
    for (int64_t c = a; c < b; ++c) {
        if (c == q.p) continue;
        if (edge_test(A, q, c)) {
            if (EMIT && cnt < lim) out[cnt] = A.sid[c];
            ++cnt;
        }
    }
}

template <bool EMIT>
__global__ void __launch_bounds__(256) search_kernel(SearchArgs A, int64_t *__restrict__ row_ptr,
                                                     int32_t *__restrict__ col_idx)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < A.n; p += stride) {
        Query q;
        q.p = p;
        q.r = A.sr[p];
        q.t = A.st[p];
        q.ep = A.sep[p];
        q.em = A.sem[p];
        q.sh = A.ssh[p];
        const int32_t id = A.sid[p];
        int32_t *out = nullptr;
        int64_t lim = 0;
        if (EMIT) {
            out = col_idx + row_ptr[id];
            lim = row_ptr[id + 1] - row_ptr[id];
        }
        int64_t cnt = 0;
        for (int j = 0; j < A.B; ++j) {
            const int64_t s = A.band_start[j], e = A.band_start[j + 1];
            if (s == e) continue;
            if (band_inside(A, q.r, j)) {
                if (EMIT) {
                    for (int64_t c = s; c < e; ++c) {
                        if (c == p) continue;
                        if (cnt < lim) out[cnt] = A.sid[c];
                        ++cnt;
                    }
                } else {
                    cnt += (e - s) - ((p >= s && p < e) ? 1 : 0);
                }
                continue;
            }
            const double w = window_half_width(A, q, j);
            if (w >= 3.0) {
                scan_range<EMIT>(A, q, s, e, cnt, out, lim);
                continue;
            }
            const int cb = A.cbits[j];
            const int64_t nc = (int64_t)1 << cb;
            const int32_t *dir = A.dir + A.dir_base[j];
            const int shift = 32 - cb;
            double lo = q.t - w, hi = q.t + w;
            // cells [c0, c1] (and a second run when the window wraps)
            int64_t a0, a1, b0 = 0, b1 = -1;
            if (lo < 0.0) {
                lo += RHG_TWO_PI_D;
                a0 = 0;
                a1 = cb ? (int64_t)(angle_key_s(hi) >> shift) : 0;
                b0 = cb ? (int64_t)(angle_key_s(lo) >> shift) : 0;
                b1 = nc - 1;
            } else if (hi >= RHG_TWO_PI_D) {
                hi -= RHG_TWO_PI_D;
                a0 = 0;
                a1 = cb ? (int64_t)(angle_key_s(hi) >> shift) : 0;
                b0 = cb ? (int64_t)(angle_key_s(lo) >> shift) : 0;
                b1 = nc - 1;
            } else {
                a0 = cb ? (int64_t)(angle_key_s(lo) >> shift) : 0;
                a1 = cb ? (int64_t)(angle_key_s(hi) >> shift) : 0;
            }
            if (b1 >= b0 && b0 <= a1 + 1) {  // the two runs meet: whole band
                scan_range<EMIT>(A, q, s, e, cnt, out, lim);
                continue;
            }
            scan_range<EMIT>(A, q, dir[a0], dir[a1 + 1], cnt, out, lim);
            if (b1 >= b0) scan_range<EMIT>(A, q, dir[b0], dir[b1 + 1], cnt, out, lim);
        }
        if (EMIT) {
            if (cnt != lim) atomicAdd(&A.stats[ST_EMIT_MISMATCH], 1ull);
        } else {
            row_ptr[id + 1] = cnt;
            if (p == 0) row_ptr[0] = 0;
        }
    }
}

hipError_t launch_search(rhg_index *idx, int64_t *row_ptr, int32_t *col_idx, int emit, hipStream_t s)
{
    const Layout &L = idx->L;
    SearchArgs A;
    for (int j = 0; j <= L.B; ++j) {
        A.E[j] = L.E[j];
        A.dir_base[j] = L.dir_base[j];
    }
    for (int j = 0; j < L.B; ++j) {
        A.e_lo[j] = exp(L.E[j]);
        A.em_lo[j] = exp(-L.E[j]);
        A.sh_lo[j] = sinh(L.E[j]);
        A.cbits[j] = L.cbits[j];
    }
    A.B = L.B;
    A.band_bits = L.band_bits;
    A.n = idx->n;
    A.R = idx->p.R;
    A.C = idx->p.cosh_R;
    A.C_lo = idx->p.cosh_R_lo;
    A.acc_thr = A.C * (1.0 - 0x1p-30);
    A.rej_thr = A.C * (1.0 + 0x1p-30);
    A.band_start = idx->band_start;
    A.dir = idx->dir;
    A.sr = idx->sr;
    A.st = idx->st;
    A.sep = idx->sep;
    A.sem = idx->sem;
    A.ssh = idx->ssh;
    A.sid = idx->sid;
    A.stats = idx->stats;
    const int64_t n = idx->n;
    if (n <= 0) {
        if (!emit) return hipMemsetAsync(row_ptr, 0, sizeof(int64_t), s);
        return hipSuccess;
    }
    int64_t blocks = (n + 255) / 256;
    if (emit)
        hipLaunchKernelGGL(search_kernel<true>, dim3((unsigned)blocks), dim3(256), 0, s, A, row_ptr, col_idx);
    else
        hipLaunchKernelGGL(search_kernel<false>, dim3((unsigned)blocks), dim3(256), 0, s, A, row_ptr, col_idx);
    return hipGetLastError();
}

}  // namespace rhg
