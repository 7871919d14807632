// rhg_search.hip -- the neighbour search (Algorithm 1, the parallel query
// loop; range query of Sec. 3.2), as count and emit passes over the index.
//
// Query region.  For a query q and a radial band j the Euclidean query circle
// of Proposition 1 is, in native coordinates, an angular window around
// theta_q: a point at radius r and angle difference dtheta is a neighbour iff
//     sin^2(dtheta/2) <= X(r) = (cosh R - cosh(r_q - r)) / (2 sinh r_q sinh r),
// and X decreases in r (the derivative has the sign of cosh R cosh r -
// cosh r_q >= 0) and, symmetrically, in r_q.  The window computed at the
// band's inner edge E[j] therefore covers the band, and the window of the
// innermost query of a group covers the whole group.  A band with
// r_q + E[j+1] <= R lies inside the circle (triangle inequality).
//
// Exact decision per candidate, on the binary64 coordinates:
//   P32  cosh d / cosh R = e'_q m'_c + m'_q e'_c + s'_q s'_c sin^2(dtheta/2)
//        with per-point FP32 values e' = e^r/sqrt(2 cosh R),
//        m' = e^-r/sqrt(2 cosh R), s' = sinh r sqrt(2/cosh R) and dtheta
//        formed in FP64 then rounded; every term is non-negative, so the
//        value is within 19 * 2^-24 (relative) of the exact ratio.  Values
//        outside 1 -/+ 2^-18 are final.
//   P64  the same sum in FP64 from r and theta (margin 2^-30), and
//   DD   double-double for the rest.
//
// Work split.  The first positions of the sorted index (the innermost
// points, the hubs) are "heavy": each (heavy query, band) pair is a work item
// for a whole workgroup (one block each, so the block dispatcher balances
// them).  Every other query is
// "light": a wavefront takes 64 consecutive queries (same band, adjacent
// angles); per band it either shares one window -- the union of its lanes'
// windows -- when those windows overlap, broadcasting each candidate to all
// lanes, or gives each lane its own window when they are narrow.
#include <string.h>

#include "rhg_internal.h"

namespace rhg {

struct SearchArgs {
    double E[RHG_MAX_BANDS + 1];      // band edges
    float ep_lo[RHG_MAX_BANDS];       // e'(E[j]), m'(E[j]), s'(E[j])
    float em_lo[RHG_MAX_BANDS];
    float sh_lo[RHG_MAX_BANDS];
    int64_t dir_base[RHG_MAX_BANDS + 1];
    int cbits[RHG_MAX_BANDS];
    int B;
    int64_t n;
    int64_t heavy_cap;                // heavy queries at most
    double R;
    double C, C_lo;                   // cosh R as double-double
    int use_p32;                      // FP32 screen valid (R small enough)
    const int32_t *band_start;
    const int32_t *dir;
    const double *sr, *st;
    const float4 *rec;                // (e', m', s', id bits)
    const int32_t *heavy_end;         // first light position
    int32_t *heavy_cnt;               // per (heavy query, band): count, then offset
    unsigned long long *stats;
};

constexpr float P32_ACC = 1.0f - 0x1p-18f;
constexpr float P32_REJ = 1.0f + 0x1p-18f;

__device__ __forceinline__ uint32_t angle_key_s(double t)
{
    const double k = t * (4294967296.0 / RHG_TWO_PI_D);
    if (!(k > 0.0)) return 0u;
    if (k >= 4294967295.0) return 4294967295u;
    return (uint32_t)k;
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

// ------------------------------------------------------------ exact tests

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

// FP64 evaluation from the coordinates; double-double inside the margin.
__device__ __noinline__ int edge_p64(double rq, double tq, double rc, double tc, double C, double C_lo,
                                     unsigned long long *stats)
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
    const double L = ch + 2.0 * (sinh(rq) * sinh(rc)) * (s * s);
    if (L < C * (1.0 - 0x1p-30)) return 1;
    if (L > C * (1.0 + 0x1p-30)) return 0;
    return edge_dd(rq, tq, rc, tc, C, C_lo, stats);
}

// FP32 screen: 1 edge, 0 no edge, 2 undecided.  `full_poly` selects the
// degree-11 Taylor polynomial of sin (any angle); otherwise the angle is
// known to be below 2^-5 and two terms suffice (x^4/120 < 2^-27).
__device__ __forceinline__ int p32(double tq, float eq, float mq, float sq, double tc, float ec, float mc, float sc,
                                   bool full_poly)
{
    const float x = (float)(0.5 * short_angle(tq, tc));
    const float x2 = x * x;
    float s;
    if (full_poly) {
        float p = -1.0f / 39916800.0f;
        p = fmaf(p, x2, 1.0f / 362880.0f);
        p = fmaf(p, x2, -1.0f / 5040.0f);
        p = fmaf(p, x2, 1.0f / 120.0f);
        p = fmaf(p, x2, -1.0f / 6.0f);
        p = fmaf(p, x2, 1.0f);
        s = x * p;
    } else {
        s = x * fmaf(x2, -1.0f / 6.0f, 1.0f);
    }
    float L = fmaf(eq, mc, mq * ec);
    L = fmaf(sq * sc, s * s, L);
    return L < P32_ACC ? 1 : (L > P32_REJ ? 0 : 2);
}

__device__ __forceinline__ int decide(const SearchArgs &A, double rq, double tq, float eq, float mq, float sq,
                                      int64_t c, double tc, float ec, float mc, float sc, bool full_poly)
{
    int v = 2;
    if (A.use_p32) v = p32(tq, eq, mq, sq, tc, ec, mc, sc, full_poly);
    if (v == 2) {
        if (A.use_p32) atomicAdd(&A.stats[ST_FP32_UNDECIDED], 1ull);
        v = edge_p64(rq, tq, A.sr[c], tc, A.C, A.C_lo, A.stats);
    }
    return v;
}

// ------------------------------------------------------------ windows

// Every point of band j (r < E[j+1], or r <= R for the last band) is within
// distance R of a query at radius rq: rq + E[j+1] <= R, tested exactly.
__device__ __forceinline__ bool band_inside(const SearchArgs &A, double rq, int j)
{
    const dd s = two_sum(rq, A.E[j + 1]);
    return s.hi < A.R || (s.hi == A.R && s.lo <= 0.0);
}

// Conservative half-width of band j's window for a query with FP32 record
// (eq, mq, sq); >= 3 means "scan the whole band".  X = (1 - cosh(r_q -
// E[j])/C) / (2 sinh r_q sinh E[j] / C) from the normalised record; for
// X <= 1/4, 2 asin(sqrt X) <= 2 sqrt(X) (1 + X/5).  The FP32 rounding of X
// (a few 1e-7 relative; the band edges keep cosh(r_q - E[j]) / C <= e^-E[1])
// is covered by the factor 1 + 2^-12 and the 2^-40 absolute pad.
__device__ __forceinline__ double window_w(const SearchArgs &A, float eq, float mq, float sq, int j)
{
    const float shl = A.sh_lo[j];
    if (A.E[j] < 0.25 || shl == 0.0f || sq == 0.0f) return 4.0;  // ill-conditioned near the centre
    const float num = 1.0f - fmaf(eq, A.em_lo[j], mq * A.ep_lo[j]);
    const float X = num / (sq * shl);
    if (!(X < 0.25f)) {
        if (!(X < 0.999f)) return 4.0;  // also catches NaN
        return 2.0 * asin(sqrt((double)X * (1.0 + 0x1p-12))) * (1.0 + 0x1p-12) + 0x1p-40;
    }
    const float Xp = fmaxf(X, 0.0f);
    return (double)(2.0f * sqrtf(Xp) * fmaf(Xp, 0.2f, 1.0f)) * (1.0 + 0x1p-12) + 0x1p-40;
}

// Sorted-position runs of band j covering the angular window [lo, hi]
// (lo may be < 0 and hi >= 2 pi: the window wraps).  Returns the number of
// runs (0, 1 or 2) in ascending position order.
__device__ __forceinline__ int window_runs(const SearchArgs &A, int j, double lo, double hi, int64_t s, int64_t e,
                                           int64_t *ra, int64_t *rb)
{
    if (hi - lo >= RHG_TWO_PI_D) {
        ra[0] = s; rb[0] = e;
        return 1;
    }
    const int cb = A.cbits[j];
    const int32_t *dir = A.dir + A.dir_base[j];
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

// Values every lane of the wave holds equally, made visibly uniform so that
// branches and loops on them compile to scalar control flow.
__device__ __forceinline__ int64_t uni64(int64_t v)
{
    const int lo = __builtin_amdgcn_readfirstlane((int)(uint32_t)(uint64_t)v);
    const int hi = __builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// ------------------------------------------------------------ heavy path

// One (heavy query, band) item per workgroup iteration.  Count pass: the
// item's count goes to heavy_cnt; emit pass: heavy_cnt holds the item's
// offset inside the row, and the workgroup writes its accepted candidates in
// position order (block-wide ballot prefix).
template <bool EMIT>
__device__ void heavy_item(const SearchArgs &A, int64_t q, int j, const int64_t *row_ptr, int32_t *col)
{
    __shared__ int wave_cnt[4];
    __shared__ int64_t running_sh;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t s = uni64(A.band_start[j]), e = uni64(A.band_start[j + 1]);
    const double rq = A.sr[q], tq = A.st[q];
    const float4 fq = A.rec[q];
    const int32_t id = __float_as_int(fq.w);
    int64_t out_base = 0, row_end = 0;
    if (EMIT) {
        out_base = row_ptr[id] + A.heavy_cnt[q * A.B + j];
        row_end = row_ptr[id + 1];
    }
    int64_t total = 0;
    if (s == e) {
        if (!EMIT && threadIdx.x == 0) A.heavy_cnt[q * A.B + j] = 0;
        return;
    }
    if (__builtin_amdgcn_readfirstlane((int)band_inside(A, rq, j))) {
        const bool self_in = (q >= s && q < e);
        if (EMIT) {
            for (int64_t c = s + threadIdx.x; c < e; c += 256) {
                if (c == q) continue;
                const int64_t k = (self_in && c > q) ? c - s - 1 : c - s;
                if (out_base + k < row_end) col[out_base + k] = __float_as_int(A.rec[c].w);
            }
        } else if (threadIdx.x == 0) {
            A.heavy_cnt[q * A.B + j] = (int32_t)((e - s) - (self_in ? 1 : 0));
        }
        return;
    }
    const double w = window_w(A, fq.x, fq.y, fq.z, j);
    int64_t ra[2], rb[2];
    int nr;
    if (w >= 3.0) { ra[0] = s; rb[0] = e; nr = 1; }
    else nr = window_runs(A, j, tq - w, tq + w, s, e, ra, rb);
    nr = __builtin_amdgcn_readfirstlane(nr);
    const bool full_poly = !(w + RHG_TWO_PI_D * ldexp(1.0, -A.cbits[j]) < 0x1p-5);
    if (threadIdx.x == 0) running_sh = 0;
    __syncthreads();
    for (int k = 0; k < nr; ++k) {
        const int64_t lo_k = uni64(ra[k]), hi_k = uni64(rb[k]);
        for (int64_t base = lo_k; base < hi_k; base += 256) {
            const int64_t c = base + threadIdx.x;
            int acc = 0;
            float4 fc = make_float4(0.f, 0.f, 0.f, 0.f);
            if (c < hi_k && c != q) {
                fc = A.rec[c];
                acc = decide(A, rq, tq, fq.x, fq.y, fq.z, c, A.st[c], fc.x, fc.y, fc.z, full_poly);
            }
            const uint64_t bal = __ballot(acc);
            if (lane == 0) wave_cnt[wave] = __popcll(bal);
            __syncthreads();
            int before = 0, blk = 0;
#pragma unroll
            for (int w2 = 0; w2 < 4; ++w2) {
                const int v = wave_cnt[w2];
                if (w2 < wave) before += v;
                blk += v;
            }
            if (EMIT && acc) {
                const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
                const int64_t o = out_base + running_sh + before + __popcll(bal & lt);
                if (o < row_end) col[o] = __float_as_int(fc.w);
            }
            __syncthreads();
            if (threadIdx.x == 0) running_sh += blk;
            total += blk;
            __syncthreads();
        }
    }
    if (!EMIT && threadIdx.x == 0) A.heavy_cnt[q * A.B + j] = (int32_t)total;
    __syncthreads();
}

// ------------------------------------------------------------ light path

// Test candidate runs [ra, rb) against the lane's query, every lane seeing
// every candidate: each lane loads one candidate per 64-step, and the step
// broadcasts them lane by lane through scalar registers.
template <bool EMIT>
__device__ __forceinline__ void shared_runs(const SearchArgs &A, int nr, const int64_t *ra, const int64_t *rb,
                                            bool need, int64_t p, double rq, double tq, float4 fq, bool full_poly,
                                            int64_t &cnt, int32_t *out, int64_t lim)
{
    const int lane = threadIdx.x & 63;
    for (int k = 0; k < nr; ++k) {
        for (int64_t base = ra[k]; base < rb[k]; base += 64) {
            const int64_t c = base + lane;
            double tcl = 0.0;
            float4 fcl = make_float4(0.f, 0.f, 0.f, 0.f);
            if (c < rb[k]) {
                tcl = A.st[c];
                fcl = A.rec[c];
            }
            const int m = (int)min((int64_t)64, rb[k] - base);
            const int tlo = __double2loint(tcl), thi = __double2hiint(tcl);
            const int ex = __float_as_int(fcl.x), mx = __float_as_int(fcl.y), sx = __float_as_int(fcl.z);
            const int idx = __float_as_int(fcl.w);
            for (int t = 0; t < m; ++t) {
                const double tc = __hiloint2double(__builtin_amdgcn_readlane(thi, t),
                                                   __builtin_amdgcn_readlane(tlo, t));
                const float ec = __int_as_float(__builtin_amdgcn_readlane(ex, t));
                const float mc = __int_as_float(__builtin_amdgcn_readlane(mx, t));
                const float sc = __int_as_float(__builtin_amdgcn_readlane(sx, t));
                const int idt = EMIT ? __builtin_amdgcn_readlane(idx, t) : 0;
                const int64_t ct = base + t;
                if (need && ct != p) {
                    if (decide(A, rq, tq, fq.x, fq.y, fq.z, ct, tc, ec, mc, sc, full_poly)) {
                        if (EMIT && cnt < lim) out[cnt] = idt;
                        ++cnt;
                    }
                }
            }
        }
    }
}

// The lane's own window: candidates loaded by each lane from memory.
template <bool EMIT>
__device__ __forceinline__ void lane_runs(const SearchArgs &A, int j, int64_t s, int64_t e, int64_t p, double rq,
                                          double tq, float4 fq, int64_t &cnt, int32_t *out, int64_t lim)
{
    const double w = window_w(A, fq.x, fq.y, fq.z, j);
    int64_t ra[2], rb[2];
    int nr;
    if (w >= 3.0) { ra[0] = s; rb[0] = e; nr = 1; }
    else nr = window_runs(A, j, tq - w, tq + w, s, e, ra, rb);
    // candidates of the boundary cells lie up to one cell width outside
    const bool full_poly = !(w + RHG_TWO_PI_D * ldexp(1.0, -A.cbits[j]) < 0x1p-5);
    for (int k = 0; k < nr; ++k) {
        for (int64_t c = ra[k]; c < rb[k]; ++c) {
            if (c == p) continue;
            const float4 fc = A.rec[c];
            if (decide(A, rq, tq, fq.x, fq.y, fq.z, c, A.st[c], fc.x, fc.y, fc.z, full_poly)) {
                if (EMIT && cnt < lim) out[cnt] = __float_as_int(fc.w);
                ++cnt;
            }
        }
    }
}

__device__ __forceinline__ double wave_min(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

template <bool EMIT>
__device__ void light_wave(const SearchArgs &A, int64_t base, int64_t *row_ptr, int32_t *col)
{
    const int lane = threadIdx.x & 63;
    const int64_t p = base + lane;
    const int64_t hend = *A.heavy_end;
    const bool active = p < A.n && p >= hend;
    if (__ballot(active) == 0) return;
    double rq = 0.0, tq = 0.0;
    float4 fq = make_float4(0.f, 0.f, 0.f, 0.f);
    if (active) {
        rq = A.sr[p];
        tq = A.st[p];
        fq = A.rec[p];
    }
    const int32_t id = __float_as_int(fq.w);
    int32_t *out = nullptr;
    int64_t lim = 0;
    if (EMIT && active) {
        out = col + row_ptr[id];
        lim = row_ptr[id + 1] - row_ptr[id];
    }
    // the innermost query of the wave has the widest windows
    const double rmin = wave_min(active ? rq : 1e300);
    const uint64_t is_min = __ballot(active && rq == rmin);
    const int lmin = __ffsll((unsigned long long)is_min) - 1;
    const float eqm = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(fq.x), lmin));
    const float mqm = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(fq.y), lmin));
    const float sqm = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(fq.z), lmin));
    const double tmin = wave_min(active ? tq : 1e300), tmax = wave_max(active ? tq : -1e300);
    int64_t cnt = 0;
    for (int j = 0; j < A.B; ++j) {
        const int64_t s = A.band_start[j], e = A.band_start[j + 1];
        if (s == e) continue;
        const bool full = active && band_inside(A, rq, j);
        if (full) {
            const bool self_in = (p >= s && p < e);
            if (EMIT) {
                for (int64_t c = s; c < e; ++c) {
                    if (c == p) continue;
                    if (cnt < lim) out[cnt] = __float_as_int(A.rec[c].w);
                    ++cnt;
                }
            } else {
                cnt += (e - s) - (self_in ? 1 : 0);
            }
        }
        const bool need = active && !full;
        if (__ballot(need) == 0) continue;
        const double W = window_w(A, eqm, mqm, sqm, j);
        if (W >= 3.0 || 2.0 * W >= tmax - tmin) {
            int64_t ra[2], rb[2];
            int nr;
            if (W >= 3.0) { ra[0] = s; rb[0] = e; nr = 1; }
            else nr = window_runs(A, j, tmin - W, tmax + W, s, e, ra, rb);
            const bool full_poly = !(W + (tmax - tmin) + RHG_TWO_PI_D * ldexp(1.0, -A.cbits[j]) < 0x1p-5);
            shared_runs<EMIT>(A, nr, ra, rb, need, p, rq, tq, fq, full_poly, cnt, out, lim);
        } else if (need) {
            lane_runs<EMIT>(A, j, s, e, p, rq, tq, fq, cnt, out, lim);
        }
    }
    if (!active) return;
    if (EMIT) {
        if (cnt != lim) atomicAdd(&A.stats[ST_EMIT_MISMATCH], 1ull);
    } else {
        row_ptr[id + 1] = cnt;
    }
}

// ------------------------------------------------------------ kernels

template <bool EMIT>
__global__ void __launch_bounds__(256) search_kernel(SearchArgs A, int64_t *__restrict__ row_ptr,
                                                     int32_t *__restrict__ col_idx)
{
    // blocks [0, heavy_cap * B): one (heavy query, band) item each, in query
    // order so the hubs start first; the rest: 256 light queries each
    const int64_t nhb = A.heavy_cap * A.B;
    if ((int64_t)blockIdx.x < nhb) {
        const int64_t hend = uni64(*A.heavy_end);
        const int64_t q = (int64_t)blockIdx.x / A.B;
        if (q >= hend) return;
        heavy_item<EMIT>(A, q, (int)((int64_t)blockIdx.x % A.B), row_ptr, col_idx);
        return;
    }
    const int64_t base = ((int64_t)blockIdx.x - nhb) * 256 + (threadIdx.x & ~63);
    light_wave<EMIT>(A, base, row_ptr, col_idx);
}

// Before the count pass: heavy_end = the first light position (the end of
// the heavy bands, capped).
__global__ void search_prologue(SearchArgs A, int jh, int32_t *heavy_end, int64_t *row_ptr, int emit)
{
    if (threadIdx.x == 0) {
        if (!emit) {
            int64_t h = jh > 0 ? (int64_t)A.band_start[jh] : 0;
            if (h > A.heavy_cap) h = A.heavy_cap;
            *heavy_end = (int32_t)h;
            row_ptr[0] = 0;
        }
    }
}

// After the count pass: heavy row degrees and per-item offsets.
__global__ void heavy_finalize(SearchArgs A, int64_t *__restrict__ row_ptr)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= *A.heavy_end) return;
    int64_t run = 0;
    for (int j = 0; j < A.B; ++j) {
        const int32_t c = A.heavy_cnt[q * A.B + j];
        A.heavy_cnt[q * A.B + j] = (int32_t)run;
        run += c;
    }
    row_ptr[__float_as_int(A.rec[q].w) + 1] = run;
}

hipError_t launch_search(rhg_index *idx, int64_t *row_ptr, int32_t *col_idx, int emit, hipStream_t s)
{
    const Layout &L = idx->L;
    const rhg_params &p = idx->p;
    SearchArgs A;
    memset(&A, 0, sizeof(A));
    const double inv = 1.0 / sqrt(2.0 * p.cosh_R), sc = sqrt(2.0 / p.cosh_R);
    for (int j = 0; j <= L.B; ++j) {
        A.E[j] = L.E[j];
        A.dir_base[j] = L.dir_base[j];
    }
    for (int j = 0; j < L.B; ++j) {
        A.ep_lo[j] = (float)(exp(L.E[j]) * inv);
        A.em_lo[j] = (float)(exp(-L.E[j]) * inv);
        A.sh_lo[j] = (float)(sinh(L.E[j]) * sc);
        A.cbits[j] = L.cbits[j];
    }
    A.B = L.B;
    A.n = idx->n;
    A.heavy_cap = idx->heavy_cap;
    A.R = p.R;
    A.C = p.cosh_R;
    A.C_lo = p.cosh_R_lo;
    A.use_p32 = 1;  // R < 80 (rhg_plan_radius): the FP32 record neither overflows nor loses range
    A.band_start = idx->band_start;
    A.dir = idx->dir;
    A.sr = idx->sr;
    A.st = idx->st;
    A.rec = idx->rec;
    A.heavy_end = idx->heavy_end;
    A.heavy_cnt = idx->heavy_cnt;
    A.stats = idx->stats;
    const int64_t n = idx->n;
    hipLaunchKernelGGL(search_prologue, dim3(1), dim3(64), 0, s, A, L.heavy_band, idx->heavy_end, row_ptr, emit);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || n <= 0) return e;
    const int64_t blocks = idx->heavy_cap * L.B + (n + 255) / 256;
    if (emit)
        hipLaunchKernelGGL(search_kernel<true>, dim3((unsigned)blocks), dim3(256), 0, s, A, row_ptr, col_idx);
    else
        hipLaunchKernelGGL(search_kernel<false>, dim3((unsigned)blocks), dim3(256), 0, s, A, row_ptr, col_idx);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (!emit && idx->heavy_cap > 0) {
        hipLaunchKernelGGL(heavy_finalize, dim3((unsigned)((idx->heavy_cap + 255) / 256)), dim3(256), 0, s, A,
                           row_ptr);
        e = hipGetLastError();
    }
    return e;
}

}  // namespace rhg
