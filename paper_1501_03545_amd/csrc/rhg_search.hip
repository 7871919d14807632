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
//        formed in FP64 then rounded.  Every term is non-negative, so the
//        relative error of the sum is the largest of its terms': with
//        u = 2^-24, at most 21 u where the degree-11 sine polynomial runs
//        (record roundings 3 u, angle cast u, five Horner FMAs with rounded
//        coefficients and a rounded x^2 4.7 u at x = pi/2, truncation
//        0.96 u, the products s*s, s'*s' and the final FMAs), and at most
//        12 u on the two-term branch (angle below 2^-5).  Underflow adds at
//        most 2^-34 absolute for R < 80.  Values outside 1 -/+ 2^-18 (64 u)
//        are final.
//   P64  the same sum in FP64 from r and theta (margin 2^-30), and
//   DD   double-double for the rest.
//
// Work split.  The first positions of the sorted index (the innermost
// points, the hubs) are "heavy": each (heavy query, band) pair is split into
// chunks of candidates, each a work item for a whole workgroup.  Every other query is "light": a wavefront takes 64 consecutive
// sorted positions (same band, adjacent angles) and, per band, the union of
// its lanes' windows.  A union that is short, or whose lanes' windows
// overlap, is swept: the unions of all such bands are read in one stream of
// contiguous runs, staged in LDS a chunk at a time, and every lane tests the
// candidates of its own window in the chunk (found by binary search on the
// angle key).  A long union of disjoint narrow windows is instead split into
// the lanes' own windows, worked through as one stream of 64 candidates per
// step.  The emit pass repeats the count pass's search in the same order and
// writes each row in place; or, staged (large graphs), the count pass also
// writes each light row into a slot sized from the query's expected degree,
// and the emit pass searches only the heavy chunks, copies the light rows
// from their slots in id order and searches again the few wavefronts whose
// rows outgrew a slot.
#include <string.h>

#include <algorithm>

#include "rhg_geom.h"
#include "rhg_internal.h"
#include "rhg_sample.h"

namespace rhg {

struct SearchArgs {
    double E[RHG_MAX_BANDS + 1];      // band edges
    float ep_lo[RHG_MAX_BANDS];       // e'(E[j]), m'(E[j]), s'(E[j])
    float em_lo[RHG_MAX_BANDS];
    float sh_lo[RHG_MAX_BANDS];
    float rs_lo[RHG_MAX_BANDS];       // 1 / sqrt(s'(E[j])) (0 for E[j] = 0)
    int64_t dir_base[RHG_MAX_BANDS + 1];
    int cbits[RHG_MAX_BANDS];
    int B;
    int64_t n;
    int64_t heavy_cap;                // heavy queries at most
    int64_t max_chunks;               // capacity of the heavy chunk table
    int heavy_blocks;                 // workgroups striding over heavy chunks
    double R;
    double C, C_lo;                   // cosh R as double-double
    int use_p32;                      // FP32 screen valid (R small enough)
    int stream_stage;                 // per-query streams of <= 64 steps staged in LDS
    int band_bits;                    // top bits of a sort key holding the band
    int sweep_max;                    // unions of at most this many candidates are swept
    int sweep_linear;                 // lanes filter every candidate of a swept chunk
    const uint32_t *keys;             // sorted keys: band, then the top angle bits
    const uint32_t *ids;              // sorted ids (4 bytes where only the id is needed)
    const int32_t *band_start;
    const int32_t *dir;
    const double *sr, *st;
    const float4 *rec;                // (e', m', s', id bits)
    const int32_t *heavy_end;         // first light position
    int64_t *hplan;                   // per heavy item: candidates, then chunks, then their prefix
    int64_t *hcnt;                    // per heavy chunk: count, then its prefix
    int32_t *hitem;                   // per heavy chunk: its item
    int64_t *hscal;                   // [0] candidate total, [1] chunk size
    unsigned long long *stats;
    longlong2 *wstat;                 // count pass, per light wavefront: (tests, candidates swept)
    // pairs the FP32 screen leaves undecided: the count pass lists them
    // (sorted positions q, c; the heavy chunk or -1), a resolving kernel
    // decides them exactly, adds the edges to the degrees and to a hash set,
    // and the emit pass looks them up
    uint64_t *dkeys;
    int32_t *dchunk;
    unsigned long long *dcount;       // [0] pairs listed, [1] the list overflowed
    int64_t dcap;                     // list capacity
    uint64_t *hset;                   // open-addressing set of listed edges (0 = empty slot)
    int64_t hmask;                    // its size - 1 (a power of two, at least twice dcap)
    int64_t col_cap;                  // emit pass: capacity of col_idx (< 0: unchecked)
    // staged count: each light query's row goes to a slot of slot_words
    // words, the slots in sorted-position order (wavefront w's start at
    // wsum[w - 1]), its length first (-1: the wavefront outgrew a slot),
    // then its entries; the count pass leaves each light row's slot start /
    // 4 + 1 in sslot[id] (0: heavy row, ~0: no slot); the emit pass copies
    // the slots out and searches again only the wavefronts flagged in sovf
    float lmu_in[RHG_MAX_BANDS], lmu_out[RHG_MAX_BANDS];
    float stage_f;
    int64_t stage_cap;
    int32_t *stage;
    uint32_t *sslot;
    uint8_t *sovf;
    int64_t *wsum;
    int64_t *dslot;                   // the listed pair's staging entry (-1: none)
    int staged;                       // this count pass stages (its emit pass copies)
    int light_skip;                   // emit pass after a staged count: heavy chunks only
};

// Passes of the search kernels: count, emit.
enum { M_COUNT = 0, M_EMIT = 1, M_STAGE = 2 };


constexpr float P32_ACC = 1.0f - 0x1p-18f;
constexpr float P32_REJ = 1.0f + 0x1p-18f;

// ------------------------------------------------------------ exact tests

__device__ __noinline__ int edge_dd(double rq, double tq, double rc, double tc, double C, double C_lo,
                                    unsigned long long *stats)
{
    atomicAdd(&stats[ST_DD], 1ull);
    const dd diff = dd_sub(cosh_dist_dd(rq, tq, rc, tc), dd_make(C, C_lo));
    if (fabs(diff.hi) <= 1e-26 * C) atomicAdd(&stats[ST_TIES], 1ull);
    return diff.hi <= 0.0;
}

// FP64 evaluation from the coordinates; double-double inside the margin.
__device__ __noinline__ int edge_p64(double rq, double tq, double rc, double tc, double C, double C_lo,
                                     unsigned long long *stats)
{
    const double L = cosh_dist64(rq, tq, rc, tc);
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

// The pair (query at sorted position q, candidate c): the FP32 screen, then
// the exact test.  EXACT decides it here (binary64, then double-double; the
// calls need a stack and spill the caller's registers, so the fast kernels
// keep them out): the count pass instead lists the pair and counts it later
// if it is an edge, and the emit pass finds the resolved edges in the set.
// `chunk` is the heavy chunk the pair belongs to (-1 for a light query).
template <int MODE, bool EXACT>
__device__ __forceinline__ int decide(const SearchArgs &A, int64_t q, double tq, float eq, float mq, float sq,
                                      int64_t c, double tc, float ec, float mc, float sc, bool full_poly,
                                      int64_t chunk)
{
    int v = 2;
    if (A.use_p32) v = p32(tq, eq, mq, sq, tc, ec, mc, sc, full_poly);
    if (v != 2) return v;
    if (EXACT) {
        if (A.use_p32 && MODE != M_EMIT) atomicAdd(&A.stats[ST_FP32_UNDECIDED], 1ull);
        return edge_p64(A.sr[q], tq, A.sr[c], tc, A.C, A.C_lo, A.stats);
    }
    // a staged light row lists the pair itself, with its staging entry
    if (MODE == M_STAGE && chunk < 0) return 2;
    const uint64_t key = pair_key(q, c);
    if (MODE != M_EMIT) {
        const unsigned long long k = atomicAdd(&A.dcount[0], 1ull);
        if ((int64_t)k < A.dcap) {
            A.dkeys[k] = key;
            A.dchunk[k] = (int32_t)chunk;
        }
        return 0;
    }
    for (uint64_t h = slot_hash(key) & (uint64_t)A.hmask;; h = (h + 1) & (uint64_t)A.hmask) {
        const uint64_t x = A.hset[h];
        if (x == key) return 1;
        if (x == 0) return 0;
    }
}

// A staged light row's undecided pair: listed with its staging entry
// (-1: beyond the slot) for the resolving kernel.
__device__ __forceinline__ void list_staged(const SearchArgs &A, int64_t q, int64_t c, int64_t slot)
{
    const unsigned long long k = atomicAdd(&A.dcount[0], 1ull);
    if ((int64_t)k < A.dcap) {
        A.dkeys[k] = pair_key(q, c);
        A.dchunk[k] = -1;
        A.dslot[k] = slot;
    }
}

__device__ __forceinline__ int slot_quads(const SearchArgs &A, int j, double r)
{
    return stage_slot_quads(A.E, A.lmu_in, A.lmu_out, A.stage_f, j, r);
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
// (eq, mq, sq); >= 3 means "scan the whole band".  X = (1 - N) / (s'_q
// s'(E[j])), N = cosh(r_q - E[j]) / C, from the normalised record; for
// X <= 1/4, 2 asin(sqrt X) <= 2 sqrt(X) (1 + X/5).  N carries at most 4 u
// relative error (u = 2^-24), so with 1 - N >= 1/64 (else the whole band)
// the computed X is within 260 u of the exact one and the window within
// about 135 u; the factor 1 + 2^-12 (4096 u) and the 2^-40 absolute pad
// (which also covers the binary64 angle arithmetic of the window ends)
// keep it conservative.
__device__ __forceinline__ double window_w(const SearchArgs &A, float eq, float mq, float sq, int j)
{
    const float shl = A.sh_lo[j];
    if (A.E[j] < 0.25 || shl == 0.0f || sq == 0.0f) return 4.0;  // ill-conditioned near the centre
    const float num = 1.0f - fmaf(eq, A.em_lo[j], mq * A.ep_lo[j]);
    if (!(num >= 0x1p-6f)) return 4.0;  // N near 1: cancellation in 1 - N (also catches NaN)
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
    return cell_runs(A.dir + A.dir_base[j], A.cbits[j], lo, hi, s, e, ra, rb);
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
//
// Every (heavy query, band) pair is an item whose candidates form at most two
// position runs (one window, possibly wrapping round 0 / 2 pi), or the whole
// band when the band lies inside the query's circle.  A planning pass sizes
// each item, then splits it into chunks of at most CH candidates (CH grows
// only if the chunk table would overflow); chunks are numbered in (query,
// band, chunk) order and a fixed pool of workgroups strides over them.  The
// count pass records each chunk's count; their prefix sum places every
// chunk's output inside its row in the emit pass.

struct ItemRuns {
    int64_t a0, b0, a1, b1;  // runs [a0, b0) and [a1, b1)
    int inside;              // whole band, no tests
    int full_poly;
    double w;
};

__device__ __forceinline__ ItemRuns item_runs(const SearchArgs &A, int64_t q, int j)
{
    ItemRuns it;
    it.a0 = it.b0 = it.a1 = it.b1 = 0;
    it.inside = 0;
    it.full_poly = 1;
    it.w = 4.0;
    const int64_t s = A.band_start[j], e = A.band_start[j + 1];
    if (s == e) return it;
    if (band_inside(A, A.sr[q], j)) {
        it.a0 = s; it.b0 = e; it.inside = 1;
        return it;
    }
    const float4 fq = A.rec[q];
    const double tq = A.st[q];
    const double w = window_w(A, fq.x, fq.y, fq.z, j);
    it.w = w;
    int64_t ra[2], rb[2];
    int nr;
    if (w >= 3.0) { ra[0] = s; rb[0] = e; nr = 1; }
    else nr = window_runs(A, j, tq - w, tq + w, s, e, ra, rb);
    it.a0 = ra[0]; it.b0 = rb[0];
    if (nr == 2) { it.a1 = ra[1]; it.b1 = rb[1]; }
    it.full_poly = !(w + RHG_TWO_PI_D * ldexp(1.0, -A.cbits[j]) < 0x1p-5);
    return it;
}

// Plan, step 1: candidates of every heavy item (0 past the heavy queries).
__global__ void __launch_bounds__(256) heavy_plan_len(SearchArgs A)
{
    __shared__ long long part[4];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    long long len = 0;
    if (i < A.heavy_cap * A.B) {
        const int64_t q = i / A.B;
        const int j = (int)(i % A.B);
        if (q < *A.heavy_end) {
            const ItemRuns it = item_runs(A, q, j);
            len = (it.b0 - it.a0) + (it.b1 - it.a1);
        }
        A.hplan[i] = len;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) len += __shfl_xor(len, o, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = len;
    __syncthreads();
    if (threadIdx.x == 0) {
        const long long t = part[0] + part[1] + part[2] + part[3];
        if (t) atomicAdd((unsigned long long *)&A.hscal[0], (unsigned long long)t);
    }
}

// Plan, step 2: chunks per item, with CH chosen so the table cannot overflow.
__global__ void __launch_bounds__(256) heavy_plan_chunks(SearchArgs A)
{
    const int64_t items = A.heavy_cap * A.B;
    const int64_t room = A.max_chunks - items;  // > 0 by construction
    const int64_t total = A.hscal[0];
    int64_t ch = RHG_HEAVY_CHUNK;
    if (total / ch >= room) ch = total / room + 1;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i == 0) A.hscal[1] = ch;
    if (i < items) {
        const int64_t len = A.hplan[i];
        A.hplan[i] = len ? (len + ch - 1) / ch : 0;
    }
}

// One chunk of a heavy item: a workgroup tests its candidates 256 at a
// time.  The count pass records the chunk's count; in the emit pass the
// prefix of the counts places the chunk's neighbours inside the query's row
// (the row order is (band, chunk, candidate)).
template <int MODE, bool EXACT>
__device__ void heavy_chunk(const SearchArgs &A, int64_t c, const int64_t *row_ptr, int32_t *col)
{
    constexpr bool EMIT = MODE == M_EMIT;
    // per-wave acceptance counts, double-buffered so that one barrier per
    // step suffices: a buffer is rewritten two steps later, after every wave
    // has passed the next step's barrier
    __shared__ int wave_cnt[2][4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t item = uni64(A.hitem[c]);  // the item holding chunk c
    const int64_t first = item ? uni64(A.hplan[item - 1]) : 0;
    const int64_t q = item / A.B;
    const int j = (int)(item % A.B);
    const int64_t ch = uni64(A.hscal[1]);
    const ItemRuns it = item_runs(A, q, j);
    const int64_t a0 = uni64(it.a0), b0 = uni64(it.b0), a1 = uni64(it.a1), b1 = uni64(it.b1);
    const int inside = __builtin_amdgcn_readfirstlane(it.inside);
    const bool full_poly = __builtin_amdgcn_readfirstlane(it.full_poly) != 0;
    const int64_t len0 = b0 - a0, len = len0 + (b1 - a1);
    const int64_t v0 = (c - first) * ch, v1 = min(len, v0 + ch);
    const double tq = A.st[q];
    const float4 fq = A.rec[q];
    const int32_t id = __float_as_int(fq.w);
    int64_t out = 0, row_end = 0;
    if (EMIT) {
        // output of this chunk = row start + counts of the row's earlier chunks
        const int64_t qfirst = q ? uni64(A.hplan[q * A.B - 1]) : 0;
        const int64_t base_c = c ? uni64(A.hcnt[c - 1]) : 0;
        const int64_t base_q = qfirst ? uni64(A.hcnt[qfirst - 1]) : 0;
        out = row_ptr[id] + (base_c - base_q);
        row_end = row_ptr[id + 1];
    }
    int64_t total = 0;
    // the candidate of entry v (its id alone inside the circle); the loads of
    // the next 256 entries are issued before this step's tests
    auto fetch = [&](int64_t v, float4 &fc, double &tc) {
        fc = make_float4(0.f, 0.f, 0.f, 0.f);
        tc = 0.0;
        if (v < v1) {
            const int64_t pos = (v < len0) ? a0 + v : a1 + (v - len0);
            if (inside) fc.w = __int_as_float((int32_t)A.ids[pos]);
            else {
                fc = A.rec[pos];
                tc = A.st[pos];
            }
        }
    };
    float4 fn;
    double tn;
    fetch(v0 + threadIdx.x, fn, tn);
    for (int64_t vb = v0; vb < v1; vb += 256) {
        const int64_t v = vb + threadIdx.x;
        const int64_t pos = (v < len0) ? a0 + v : a1 + (v - len0);
        const float4 fc = fn;
        const double tc = tn;
        if (vb + 256 < v1) fetch(v + 256, fn, tn);
        int acc = 0;
        const int32_t cid = __float_as_int(fc.w);
        if (v < v1 && pos != q)
            acc = inside ? 1 : decide<MODE, EXACT>(A, q, tq, fq.x, fq.y, fq.z, pos, tc, fc.x, fc.y, fc.z, full_poly, c);
        const uint64_t bal = __ballot(acc);
        const int buf = (int)(((vb - v0) >> 8) & 1);
        if (lane == 0) wave_cnt[buf][wave] = __popcll(bal);
        __syncthreads();
        int before = 0, blk = 0;
#pragma unroll
        for (int w2 = 0; w2 < 4; ++w2) {
            const int x = wave_cnt[buf][w2];
            if (w2 < wave) before += x;
            blk += x;
        }
        if (EMIT && acc) {
            const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
            const int64_t o = out + total + before + __popcll(bal & lt);
            if (o < row_end) col[o] = cid;
        }
        total += blk;
    }
    // the next chunk starts again at buffer 0: every wave has read this one's
    // counts first
    __syncthreads();
    if (!EMIT && threadIdx.x == 0) A.hcnt[c] = total;
    // the emit pass finds exactly what the count pass counted in this chunk
    if (EMIT && threadIdx.x == 0 && total != A.hcnt[c] - (c ? A.hcnt[c - 1] : 0))
        atomicAdd(&A.stats[ST_EMIT_MISMATCH], 1ull);
}

// ------------------------------------------------------------ light path

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
// Lane l's value, as a wave-uniform scalar.
__device__ __forceinline__ int64_t uni_lane64(int64_t v, int l)
{
    const int lo = __builtin_amdgcn_readlane((int)(uint32_t)(uint64_t)v, l);
    const int hi = __builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), l);
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
__device__ __forceinline__ int64_t wave_excl_sum64(int64_t v, int lane, int64_t *total)
{
    int64_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    *total = __shfl(x, 63, 64);
    return x - v;
}

// Upper bound of band j's window for a query with normalised record
// (e', m', s'): dropping the non-negative cosh(r_q - E[j]) / cosh R term
// gives X <= 1 / (s'_q s'(E[j])), so sqrt X <= rs_q * rs_j with the reciprocal
// square roots computed once per query and per band.  rs_j is raised by
// 2^-20 (16 u), more than the 1-ulp reciprocal square root of the query, the
// record roundings and the product lose, so rs_q * rs_j >= sqrt X; the
// polynomial's roundings (3 u) are covered by the factor 1 + 2^-12.  Above
// X = 1/4 it falls back to window_w.
__device__ __forceinline__ double window_fast(const SearchArgs &A, float rsq, float eq, float mq, float sq, int j)
{
    if (A.rs_lo[j] == 0.0f || A.E[j] < 0.25) return window_w(A, eq, mq, sq, j);
    const float sx = rsq * A.rs_lo[j];
    const float X = sx * sx;
    if (!(X < 0.25f)) return window_w(A, eq, mq, sq, j);
    return (double)(2.0f * sx * fmaf(X, 0.2f, 1.0f)) * (1.0 + 0x1p-12) + 0x1p-40;
}

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The sort key of angle t in band j, as the index computed it (the index
// orders each band's positions by it; points with equal keys stay in id
// order), so a binary search on the staged keys finds where an angle's run
// of positions starts.
__device__ __forceinline__ uint32_t band_key(const SearchArgs &A, int j, double t)
{
    const uint32_t ak = angle_key_s(t);
    return A.band_bits ? (((uint32_t)j << (32 - A.band_bits)) | (ak >> A.band_bits)) : ak;
}

// A wavefront's LDS.  The sweep stages a chunk of candidates; a per-query
// stream keeps its map (one word per step with a bit at each owner's first
// entry, and the owners' runs in lane order) and stages STREAM_CHUNK steps.
constexpr int SWEEP_C = 128;
constexpr int ROWBUF = 16;  // emit pass: row entries each lane gathers in LDS before writing them
constexpr int STREAM_STEPS = 64;
constexpr int STREAM_CHUNK = 4;
struct SweepStage {
    double t[SWEEP_C];
    float4 rec[SWEEP_C];
    uint32_t key[SWEEP_C];
    int32_t row[ROWBUF][64];  // entry i of lane l's buffered row run at row[i][l]
};
// A run of a row written as whole 16-byte stores where the target allows
// dword-aligned ones (the compiler splits them otherwise).
struct __attribute__((aligned(4))) int4a {
    int32_t x, y, z, w;
};
struct StreamStage {
    float4 rec[STREAM_CHUNK][64];
    int32_t tlo[STREAM_CHUNK][64], thi[STREAM_CHUNK][64];
    int2 own[STREAM_CHUNK][64];  // (owner lane, candidate position)
};
struct WaveLds {
    unsigned long long start[STREAM_STEPS];
    int4 run[64];  // owners in lane order: (first entry, first run's length | lane << 16, run starts)
    union {
        SweepStage sw;
        StreamStage ss;
    } u;
};
static_assert(STREAM_STEPS == 64, "one word per lane is cleared");

// Light queries: a wavefront of 64 consecutive sorted positions.  Lane j
// first builds band j's entry of the wave's band table: the union of the
// lanes' windows (the window of the innermost lane, stretched over the
// lanes' angle range) as at most two position runs, and whether the band is
// swept (mode 1) or searched per query (mode 2).
//
// M_COUNT writes the degree, M_EMIT the row.  The row order is the same in
// both: the inside bands in band order, then the swept bands in band order
// (each in position order), then the per-query bands in band order.
template <int MODE, bool EXACT>
__device__ void light_wave(const SearchArgs &A, int64_t base, int64_t *row_ptr, int32_t *col)
{
    // STAGE: counted like the count pass, written like the emit pass into
    // the query's staging slot
    constexpr bool STAGE = MODE == M_STAGE;
    constexpr bool EMIT = MODE == M_EMIT || STAGE;
    constexpr bool COUNTING = MODE != M_EMIT;
    __shared__ WaveLds lds[4];
    WaveLds &SM = lds[threadIdx.x >> 6];
    const int lane = threadIdx.x & 63;
    const int64_t p = base + lane;
    // the query's loads do not wait for the heavy/light boundary
    const bool inb = p < A.n;
    double rq = 0.0, tq = 0.0;
    float4 fq = make_float4(0.f, 0.f, 0.f, 1.f);
    if (inb) {
        rq = A.sr[p];
        tq = A.st[p];
        fq = A.rec[p];
    }
    const int64_t hend = uni64(*A.heavy_end);
    const bool active = inb && p >= hend;
    if (__ballot(active) == 0) {
        if (COUNTING && lane == 0 && base < A.n) A.wstat[base >> 6] = make_longlong2(0, 0);
        return;
    }
    if (!active) {
        rq = 0.0;
        tq = 0.0;
        fq = make_float4(0.f, 0.f, 0.f, 1.f);
    }
    const int32_t id = __float_as_int(fq.w);
    int32_t *out = nullptr;  // EMIT: entry k of the row goes to out[k] while k < lim
    int64_t lim = 0;
    if (MODE == M_EMIT && active) {
        out = col + row_ptr[id];
        lim = row_ptr[id + 1] - row_ptr[id];
    }
    if (STAGE) {
        // the slot: after the wavefront's earlier lanes' slots; word 0 holds
        // the row's length
        int quads = 0;
        if (active) quads = slot_quads(A, A.band_bits ? (int)(A.keys[p] >> (32 - A.band_bits)) : 0, rq);
        int wt;
        const int64_t wv = base >> 6;
        const int64_t sb = (wv ? A.wsum[wv - 1] : 0) + 4 * (int64_t)wave_excl_sum(quads, lane, &wt);
        out = A.stage + sb + 1;
        lim = active ? max<int64_t>(0, min<int64_t>(4 * (int64_t)quads - 1, A.stage_cap - sb - 1)) : 0;
    }
    int64_t pend = 0;  // STAGE: entries of the row still pending
    const int B = A.B;
    // the innermost query of the wave has the widest windows
    const double rmin = wave_min(active ? rq : 1e300);
    const uint64_t is_min = __ballot(active && rq == rmin);
    const int lmin = __ffsll((unsigned long long)is_min) - 1;
    const float eqm = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(fq.x), lmin));
    const float mqm = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(fq.y), lmin));
    const float sqm = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(fq.z), lmin));
    const double tmin = wave_min(active ? tq : 1e300), tmax = wave_max(active ? tq : -1e300);
    const double span = tmax - tmin;

    // bands lying wholly inside this lane's circle: taken without tests.  The
    // test is exact and monotone in the band's outer edge, so the inside
    // bands are the first J of them.
    int64_t cnt = 0;
    int J = 64;  // inactive lanes: neutral in the wave's minimum below
    if (active) {
        J = 0;
        while (J < B && band_inside(A, rq, J)) ++J;
        if (EMIT) {
            for (int j = 0; j < J; ++j) {
                const int64_t s = A.band_start[j], e = A.band_start[j + 1];
                for (int64_t c = s; c < e; ++c) {
                    if (c == p) continue;
                    if (cnt < lim) out[cnt] = (int32_t)A.ids[c];
                    ++cnt;
                }
            }
        } else {
            const int64_t s = A.band_start[0], e = A.band_start[J];
            cnt = (e - s) - ((p >= s && p < e) ? 1 : 0);
        }
    }
    const uint64_t lt_mask = lane ? (~0ull >> (64 - lane)) : 0ull;
    int tests = 0, swept = 0;

    // band table: lane j describes band j
    int mode = 0;  // 0 nothing, 1 swept, 2 per-query windows
    int32_t a0 = 0, b0 = 0, a1 = 0, b1 = 0;
    if (lane < B) {
        const int j = lane;
        const int64_t s = A.band_start[j], e = A.band_start[j + 1];
        if (s < e) {
            const double W = window_w(A, eqm, mqm, sqm, j);
            if (W >= 3.0) {
                a0 = (int32_t)s; b0 = (int32_t)e;
                mode = 1;
            } else {
                int64_t ra[2], rb[2];
                const int nr = window_runs(A, j, tmin - W, tmax + W, s, e, ra, rb);
                a0 = (int32_t)ra[0]; b0 = (int32_t)rb[0];
                if (nr == 2) { a1 = (int32_t)ra[1]; b1 = (int32_t)rb[1]; }
                const int U = (b0 - a0) + (b1 - a1);
                mode = (2.0 * W >= span || U <= A.sweep_max) ? 1 : 2;
            }
        }
    }
    // a band every active lane takes whole needs no tests: the bands below
    // the wave's minimum J (found bit by bit with ballots)
    {
        uint64_t cand = __ballot(active);
        int mj = 0;
#pragma unroll
        for (int b = 6; b >= 0; --b) {
            const uint64_t zero = __ballot(((J >> b) & 1) == 0) & cand;
            if (zero) cand = zero;
            else mj |= 1 << b;
        }
        if (lane < mj) mode = 0;
    }
    if ((b0 - a0) + (b1 - a1) == 0) mode = 0;
    const float rsq = active && fq.z > 0.0f ? rsqrtf(fq.z) : 0.0f;

    // EMIT: the swept bands' entries of this lane's row gather in LDS,
    // ROWBUF at a time, and leave as whole runs; row entries [fl, fl + nb)
    // are buffered.
    int64_t fl = cnt;
    int nb = 0;

    // The pair (this lane's query, candidate at sorted position c): the
    // exact decision, counted and (EMIT) put into the row.
    auto take = [&](int64_t c, double tc, float4 fc, bool fp, SweepStage &S) {
        ++tests;
        const int v = decide<MODE, EXACT>(A, p, tq, fq.x, fq.y, fq.z, c, tc, fc.x, fc.y, fc.z, fp, -1);
        if (v) {
            if (STAGE && v == 2) {
                list_staged(A, p, c, cnt < lim ? (int64_t)(out - A.stage) + cnt : -1);
                ++pend;
            }
            if (EMIT && cnt < lim) {
                S.row[nb][lane] = __float_as_int(fc.w) | (STAGE && v == 2 ? (int)STAGE_PENDING : 0);
                if (++nb == ROWBUF) {
                    // a full buffer: fl + ROWBUF <= lim
#pragma unroll
                    for (int i = 0; i < ROWBUF; i += 4)
                        *(int4a *)(out + fl + i) = int4a{S.row[i][lane], S.row[i + 1][lane], S.row[i + 2][lane],
                                                          S.row[i + 3][lane]};
                    fl += ROWBUF;
                    nb = 0;
                }
            }
            ++cnt;
        }
    };

    // ---- swept bands: the unions of every band with mode 1, in band order,
    // as one stream of position runs, staged SWEEP_C candidates at a time
    const uint64_t swm = __ballot(lane < B && mode == 1);
    if (swm) {
        SweepStage &S = SM.u.sw;
        const int T = (lane < B && mode == 1) ? (b0 - a0) + (b1 - a1) : 0;
        const int L0 = b0 - a0;
        int tot;
        const int pre = wave_excl_sum(T, lane, &tot);  // band `lane`'s entries are [pre, pre + T)
        swept = tot;
        for (int c0 = 0; c0 < tot; c0 += SWEEP_C) {
            wave_sync();  // the previous chunk's reads are done
            double tl[SWEEP_C / 64];
            float4 rl[SWEEP_C / 64];
            uint32_t kl[SWEEP_C / 64];
#pragma unroll
            for (int k = 0; k < SWEEP_C / 64; ++k) {
                const int t = c0 + 64 * k + lane;
                int jb = 0;  // the last swept band starting at or before t
                for (uint64_t m = swm; m; m &= m - 1) {
                    const int j = __ffsll((unsigned long long)m) - 1;
                    if (t >= __builtin_amdgcn_readlane(pre, j)) jb = j;
                }
                // the band's run data from lane jb, with every lane taking part
                // (a lane outside the exec mask gives no value to a shuffle)
                const int off = t - __shfl(pre, jb, 64);
                const int l0 = __shfl(L0, jb, 64), ja0 = __shfl(a0, jb, 64), ja1 = __shfl(a1, jb, 64);
                tl[k] = 0.0;
                rl[k] = make_float4(0.f, 0.f, 0.f, 0.f);
                kl[k] = 0u;
                if (t < tot) {
                    const int64_t pos = off < l0 ? (int64_t)ja0 + off : (int64_t)ja1 + (off - l0);
                    tl[k] = A.st[pos];
                    rl[k] = A.rec[pos];
                    kl[k] = A.keys[pos];
                }
            }
#pragma unroll
            for (int k = 0; k < SWEEP_C / 64; ++k) {
                S.t[64 * k + lane] = tl[k];
                S.rec[64 * k + lane] = rl[k];
                S.key[64 * k + lane] = kl[k];
            }
            wave_sync();
            const int cend = min(tot, c0 + SWEEP_C);
            for (uint64_t m = swm; m; m &= m - 1) {
                const int j = __ffsll((unsigned long long)m) - 1;
                const int pj = __builtin_amdgcn_readlane(pre, j), Tj = __builtin_amdgcn_readlane(T, j);
                const int ls = max(pj, c0) - c0, hs = min(pj + Tj, cend) - c0;
                if (ls >= hs || !(active && j >= J)) continue;
                const int ja0 = __builtin_amdgcn_readlane(a0, j), ja1 = __builtin_amdgcn_readlane(a1, j);
                const int jl0 = __builtin_amdgcn_readlane(L0, j);
                // a segment of a few candidates: each is tested as it is,
                // with no window to compute first
                if (hs - ls <= 4) {
                    for (int k = ls; k < hs; ++k) {
                        const float4 fc = S.rec[k];
                        if (__float_as_int(fc.w) == id) continue;
                        const int off = c0 + k - pj;
                        const int64_t pos = off < jl0 ? (int64_t)ja0 + off : (int64_t)ja1 + (off - jl0);
                        take(pos, S.t[k], fc, true, S);
                    }
                    continue;
                }
                const double w = (fq.z > 0.0f) ? window_fast(A, rsq, fq.x, fq.y, fq.z, j) : 4.0;
                // every tested candidate lies within w of the query, so the
                // two-term sine serves windows below 2^-5
                const bool fp = !(w < 0x1p-5);
                auto test = [&](int k) {
                    const double tc = S.t[k];
                    if (short_angle(tq, tc) > w) return;
                    const float4 fc = S.rec[k];
                    if (__float_as_int(fc.w) == id) return;
                    const int off = c0 + k - pj;
                    const int64_t pos = off < jl0 ? (int64_t)ja0 + off : (int64_t)ja1 + (off - jl0);
                    take(pos, tc, fc, fp, S);
                };
                // a half-width of 3 or more: the linear filter (the two pieces
                // below stay apart by more than a key step only for narrower
                // windows, 2 pi - 2w > 0.28 rad)
                if (!(w < 3.0) || hs - ls <= 8 || A.sweep_linear) {
                    for (int k = ls; k < hs; ++k) test(k);
                    continue;
                }
                // the window's position range in the chunk: the first
                // position whose key reaches the window's start, then on
                // while the key stays within its end (and, for a window
                // across 0 / 2 pi, its other piece)
                auto lower = [&](uint32_t kq) {
                    int lo = ls, hi = hs;
                    while (lo < hi) {
                        const int mid = (lo + hi) >> 1;
                        if (S.key[mid] < kq) lo = mid + 1;
                        else hi = mid;
                    }
                    return lo;
                };
                // (pieces in position order, so that the row order is that
                // of the linear filter)
                const double wlo = tq - w, whi = tq + w;
                if (whi >= RHG_TWO_PI_D) {
                    const uint32_t k2 = band_key(A, j, whi - RHG_TWO_PI_D);
                    for (int k = ls; k < hs && S.key[k] <= k2; ++k) test(k);
                }
                const uint32_t khi = band_key(A, j, fmin(whi, RHG_TWO_PI_D));
                for (int k = lower(band_key(A, j, fmax(wlo, 0.0))); k < hs && S.key[k] <= khi; ++k) test(k);
                if (wlo < 0.0)
                    for (int k = lower(band_key(A, j, wlo + RHG_TWO_PI_D)); k < hs; ++k) test(k);
            }
        }
    }

    if (EMIT && swm) {
        // the rest of every lane's buffered run, one lane's run per store
        SweepStage &S = SM.u.sw;
        wave_sync();
        for (uint64_t m = __ballot(nb > 0); m; m &= m - 1) {
            const int l = __ffsll((unsigned long long)m) - 1;
            const int ln = __builtin_amdgcn_readlane(nb, l);
            int32_t *const dst = (int32_t *)uni_lane64((int64_t)(out + fl), l);
            if (lane < ln) dst[lane] = S.row[lane][l];
        }
        wave_sync();  // the stage is reused by the per-query bands
    }

    // ---- per-query bands (the lanes' angles spread wider than the window):
    // each lane finds its own runs in band j; the runs of all lanes are then
    // concatenated (lane order) and worked through 64 candidates per step,
    // each candidate tested against the query of the lane that owns it.
    const uint64_t percell = __ballot(lane < B && mode == 2);
    for (uint64_t mk = percell; mk; mk &= mk - 1) {
        const int j = __ffsll((unsigned long long)mk) - 1;
        const int64_t s = A.band_start[j], e = A.band_start[j + 1];
        int ra0 = 0, rb0 = 0, ra1 = 0, rb1 = 0;  // positions are below 2^31
        double w = 0.0;
        const bool mine = active && j >= J;
        if (mine) {
            w = (fq.z > 0.0f) ? window_fast(A, rsq, fq.x, fq.y, fq.z, j) : 4.0;
            int64_t ra[2] = {0, 0}, rb[2] = {0, 0};
            if (w >= 3.0) { ra[0] = s; rb[0] = e; }
            else window_runs(A, j, tq - w, tq + w, s, e, ra, rb);
            ra0 = (int)ra[0]; rb0 = (int)rb[0]; ra1 = (int)ra[1]; rb1 = (int)rb[1];
        }
        const int len0 = rb0 - ra0, len = len0 + (rb1 - ra1);
        const int fpl = !(w + RHG_TWO_PI_D * ldexp(1.0, -A.cbits[j]) < 0x1p-5);
        int64_t total;
        const int64_t pre = wave_excl_sum64((int64_t)len, lane, &total);  // this lane's runs: [pre, pre + len)
        if (total == 0) continue;
        // A stream of at most 64 steps gets a map in LDS: one word per step
        // with a bit at each owner's first entry, and the owners' runs in
        // lane order.  The owner of an entry is then the owners starting
        // before its step plus the bits up to it, and one LDS read.
        const bool small = A.stream_stage && total <= 64 * STREAM_STEPS;
        if (small) {
            const int nz = __popcll(__ballot(len > 0) & lt_mask);
            wave_sync();  // the previous band's reads of the map are done
            SM.start[lane] = 0;
            wave_sync();
            if (len > 0) {
                atomicOr(&SM.start[pre >> 6], 1ull << (pre & 63));
                SM.run[nz] = make_int4((int)pre, len0 | (lane << 16), ra0, ra1);
            }
            wave_sync();
        }
        int before = 0;  // owners starting before the step being located
        // owner lane and position of stream entry t0 + lane, for the steps
        // t0 = 0, 64, 128, ... in order (every lane takes part)
        auto locate = [&](int64_t t0, int &l, int &c) {
            const int64_t t = t0 + lane;
            if (small) {
                const uint64_t bits = (uint64_t)uni64((int64_t)SM.start[t0 >> 6]);
                const uint64_t upto = lane == 63 ? ~0ull : (2ull << lane) - 1;
                const int4 r = SM.run[before + __popcll(bits & upto) - 1];
                before += __popcll(bits);
                l = r.y >> 16;
                const int l0 = r.y & 0xffff, k = (int)t - r.x;
                c = (k < l0) ? r.z + k : r.w + (k - l0);
                return;
            }
            l = 0;
#pragma unroll
            for (int step = 32; step > 0; step >>= 1) {
                const int64_t pv = __shfl(pre, l + step, 64);
                if (t >= pv) l += step;
            }
            const int k = (int)(t - __shfl(pre, l, 64));
            const int l0 = __shfl(len0, l, 64), la0 = __shfl(ra0, l, 64), la1 = __shfl(ra1, l, 64);
            c = (k < l0) ? la0 + k : la1 + (k - l0);
        };
        // one step of the stream: entry t0 + lane is candidate c of lane l's
        // query
        auto step = [&](int64_t t0, int l, int c, double tc, float4 fc) {
            const bool valid = t0 + lane < total;
            // the owner's query
            const double lt = __shfl(tq, l, 64), lw = __shfl(w, l, 64);
            const float le = __shfl(fq.x, l, 64), lmq = __shfl(fq.y, l, 64), ls = __shfl(fq.z, l, 64);
            const int64_t lp = base + l;
            const bool lfp = __shfl(fpl, l, 64) != 0;
            int acc = 0;
            const int cid = __float_as_int(fc.w);
            if (valid && c != lp && !(short_angle(lt, tc) > lw)) {
                ++tests;
                acc = decide<MODE, EXACT>(A, lp, lt, le, lmq, ls, c, tc, fc.x, fc.y, fc.z, lfp, -1);
            }
            const uint64_t bal = __ballot(acc);
            // this lane's part of the step, as the owner of [pre, pre + len)
            const int64_t lo = pre - t0, hi = pre + len - t0;
            const uint64_t lom = lo <= 0 ? ~0ull : (lo >= 64 ? 0ull : ~0ull << lo);
            const uint64_t him = hi >= 64 ? ~0ull : (hi <= 0 ? 0ull : ~(~0ull << hi));
            const int got = __popcll(bal & lom & him);
            if (EMIT) {
                // position inside the owner's row: its count before the step plus
                // the acceptances of its earlier entries in this step
                const int64_t lo_l = __shfl(pre, l, 64) - t0;
                const uint64_t seg = lo_l <= 0 ? ~0ull : ~0ull << lo_l;
                const int64_t at = __shfl(cnt, l, 64) + __popcll(bal & seg & lt_mask);
                int32_t *const lout = (int32_t *)__shfl((int64_t)out, l, 64);
                const int64_t llim = __shfl(lim, l, 64);
                if (STAGE && acc == 2) list_staged(A, lp, c, at < llim ? (int64_t)(lout - A.stage) + at : -1);
                if (acc && at < llim) lout[at] = cid | (STAGE && acc == 2 ? (int)STAGE_PENDING : 0);
            }
            if (STAGE) pend += __popcll(__ballot(acc == 2) & lom & him);
            cnt += got;
        };
        if (small) {
            // STREAM_CHUNK steps at a time: locate every entry and load its
            // candidate straight into the LDS stage (one memory round trip for
            // the chunk, no registers held), then test the steps from LDS
            StreamStage &G = SM.u.ss;
            const int32_t *const st32 = (const int32_t *)A.st;
            for (int64_t tc0 = 0; tc0 < total; tc0 += 64 * STREAM_CHUNK) {
                // every locate (LDS reads) before the first load: a read of
                // LDS after a load into LDS waits for that load
                int cs[STREAM_CHUNK];
#pragma unroll
                for (int k = 0; k < STREAM_CHUNK; ++k) {
                    cs[k] = 0;
                    const int64_t t0 = tc0 + 64 * k;
                    if (t0 < total) {
                        int l;
                        locate(t0, l, cs[k]);
                        G.own[k][lane] = make_int2(l, cs[k]);
                    }
                }
#pragma unroll
                for (int k = 0; k < STREAM_CHUNK; ++k) {
                    const int64_t t0 = tc0 + 64 * k, c = cs[k];
                    if (t0 + lane < total) {
                        __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)(A.rec + c),
                                                         (__attribute__((address_space(3))) void *)G.rec[k], 16, 0, 0);
                        __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)(st32 + 2 * c),
                                                         (__attribute__((address_space(3))) void *)G.tlo[k], 4, 0, 0);
                        __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)(st32 + 2 * c + 1),
                                                         (__attribute__((address_space(3))) void *)G.thi[k], 4, 0, 0);
                    }
                }
#pragma unroll
                for (int k = 0; k < STREAM_CHUNK; ++k) {
                    const int64_t t0 = tc0 + 64 * k;
                    if (t0 < total) {
                        const int2 lc = G.own[k][lane];
                        step(t0, lc.x, lc.y, __hiloint2double(G.thi[k][lane], G.tlo[k][lane]), G.rec[k][lane]);
                    }
                }
                wave_sync();  // the stage is rewritten by the next chunk
            }
            continue;
        }
        // a long stream: the loads of the next step are issued before the
        // current step is tested
        if (lane == 0) atomicAdd(&A.stats[ST_REG_STREAMS], 1ull);
        int ln, cn;
        locate(0, ln, cn);
        double tn = 0.0;
        float4 fn = make_float4(0.f, 0.f, 0.f, 0.f);
        if (lane < total) { tn = A.st[cn]; fn = A.rec[cn]; }
        for (int64_t t0 = 0; t0 < total; t0 += 64) {
            const int l = ln, c = cn;
            const double tc = tn;
            const float4 fc = fn;
            if (t0 + 64 < total) {
                locate(t0 + 64, ln, cn);
                if (t0 + 64 + lane < total) { tn = A.st[cn]; fn = A.rec[cn]; }
            }
            step(t0, l, c, tc, fc);
        }
    }
    if (COUNTING) {
        int tt;
        wave_excl_sum(tests, lane, &tt);
        if (lane == 0) A.wstat[base >> 6] = make_longlong2(tt, swept);
    }
    // a row that outgrew its slot: the emit pass searches this wavefront again
    const bool wovf = STAGE && __ballot(active && cnt > lim) != 0;
    if (wovf && lane == 0) A.sovf[base >> 6] = 1;
    if (!active) return;
    if (STAGE) {
        // the degree, with the slot's start / 4 + 1 above it (split off
        // before the row scan), and the slot's length word
        const int64_t sb = (int64_t)(out - A.stage) - 1;
        const uint64_t hs = sb < A.stage_cap ? (uint64_t)(sb >> 2) + 1 : 0xffffffffull;
        row_ptr[id + 1] = (int64_t)((hs << 32) | (uint64_t)(cnt - pend));
        if (sb < A.stage_cap) A.stage[sb] = wovf ? -1 : (int32_t)cnt;
    } else if (EMIT) {
        if (cnt != lim) atomicAdd(&A.stats[ST_EMIT_MISMATCH], 1ull);
    } else {
        row_ptr[id + 1] = cnt;
    }
}

// ------------------------------------------------------------ kernels

// The search: workgroups [0, heavy_blocks) are a pool striding over the
// heavy chunks in (query, band, chunk) order, hubs first; the rest take 256
// consecutive light positions each, one wavefront per 64.  The heavy pool
// has the lowest workgroup ids, so it starts first and the light
// wavefronts fill the chip around it.  The fast kernel (EXACT false) lists
// the pairs its FP32 screen leaves undecided; when that list overflowed in
// the count pass (dcount[1]) the EXACT kernels redo both passes, and each
// kind leaves as soon as it sees it is not the one to run.  The EXACT
// kernel strides over the light positions with a grid of any size.
template <int MODE, bool EXACT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8)))
search_kernel(SearchArgs A, int64_t *__restrict__ row_ptr, int32_t *__restrict__ col_idx, int gate)
{
    // emit pass into a buffer too small for the graph: write nothing (the
    // prologue has raised the overflow flag)
    if (MODE == M_EMIT && A.col_cap >= 0 && uni64(row_ptr[A.n]) > A.col_cap) return;
    if (gate && (__builtin_amdgcn_readfirstlane((int)A.dcount[1]) != 0) != EXACT) return;
    if ((int)blockIdx.x < A.heavy_blocks) {
        const int64_t nch = uni64(A.hplan[A.heavy_cap * A.B - 1]);
        for (int64_t c = blockIdx.x; c < nch; c += A.heavy_blocks) heavy_chunk<MODE, EXACT>(A, c, row_ptr, col_idx);
        return;
    }
    // emit pass after a staged count: the light rows are copied (and the
    // wavefronts whose rows outgrew their slots searched again) by the
    // kernels below
    if (A.light_skip) return;
    const int64_t lb = (A.n + 255) / 256, nb = (int64_t)gridDim.x - A.heavy_blocks;
    for (int64_t b = (int64_t)blockIdx.x - A.heavy_blocks; b < lb; b += nb) {
        light_wave<MODE, EXACT>(A, b * 256 + (threadIdx.x & ~63), row_ptr, col_idx);
        if (!EXACT) break;
    }
}

// Before a staged count: per wavefront of 64 sorted positions, the words of
// its light queries' slots (the search kernel sizes them the same way).
__global__ void __launch_bounds__(256) stage_wave_words(SearchArgs A, int64_t *__restrict__ wsum, int64_t waves)
{
    const int lane = threadIdx.x & 63;
    const int64_t hend = *A.heavy_end;
    for (int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); w < waves; w += (int64_t)gridDim.x * 4) {
        const int64_t p = w * 64 + lane;
        int quads = 0;
        if (p < A.n && p >= hend)
            quads = slot_quads(A, A.band_bits ? (int)(A.keys[p] >> (32 - A.band_bits)) : 0, A.sr[p]);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) quads += __shfl_xor(quads, o, 64);
        if (lane == 0) wsum[w] = 4 * (int64_t)quads;
    }
}

// After a staged count: each light row's degree carries its slot's start /
// 4 + 1 in the upper 32 bits; they move to sslot (0 for the heavy rows,
// whose degrees heavy_degrees wrote) before the row scan.
__global__ void __launch_bounds__(256) stage_split_kernel(int64_t *__restrict__ row_ptr, uint32_t *__restrict__ sslot,
                                                          int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const uint64_t v = (uint64_t)row_ptr[i + 1];
    sslot[i] = (uint32_t)(v >> 32);
    row_ptr[i + 1] = (int64_t)(v & 0xffffffffull);
}

// Emit pass after a staged count: the light rows copied from their slots,
// 64 consecutive ids to a wavefront, so that row_ptr and sslot are read in
// order and the wavefront's rows fill one stretch of col_idx.  A row is
// taken as flat (its slot holds exactly its row_ptr length) and joins a
// stream of entries that the wavefront copies 64 at a time, each lane
// finding its entry's row by a binary search over the rows' starts; the
// entries are loaded together with the slots' length words and stored only
// for the rows whose length word matches, so that a wavefront waits for
// memory about once per batch.  A row whose slot holds more (entries that
// the resolving kernel rejected) is compacted on its own; a length word of
// -1 leaves the row to stage_redo_kernel; one below the row_ptr length is
// an emit mismatch.  Few registers, so that many wavefronts keep their
// loads in flight.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8)))
stage_copy_kernel(SearchArgs A, const int64_t *__restrict__ row_ptr, int32_t *__restrict__ col)
{
    // a col_idx buffer too small for the graph: write nothing
    if (A.col_cap >= 0 && uni64(row_ptr[A.n]) > A.col_cap) return;
    const int lane = threadIdx.x & 63;
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    const int64_t wstride = (int64_t)gridDim.x * 4;
    for (int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); w * 64 < A.n; w += wstride) {
        const int64_t id = w * 64 + lane;
        int64_t dst = 0, rl = 0, sb = 0;
        bool has = false;
        if (id < A.n) {
            const uint32_t hs = A.sslot[id];
            dst = row_ptr[id];
            rl = row_ptr[id + 1] - dst;
            if (hs != 0u && hs != 0xffffffffu && rl > 0) {
                sb = (int64_t)(hs - 1u) * 4;
                has = sb < A.stage_cap;
            }
        }
        int len = -2;
        if (has) len = A.stage[sb];
        // entries loaded per row: its row_ptr length, kept inside the
        // staging area (a row whose slot is shorter is not stored); a row
        // longer than any slot (2^24 + 3 entries) cannot be flat, so the
        // wavefront's stream stays below 2^31 entries
        int tot;
        const bool fits = has && rl <= (1 << 24) + 3;
        const int pre = wave_excl_sum(fits ? (int)min<int64_t>(rl, A.stage_cap - sb - 1) : 0, lane, &tot);
        constexpr int COPY_BATCH = 5;
        for (int e0 = 0; e0 < tot; e0 += 64 * COPY_BATCH) {
            int32_t v[COPY_BATCH];
            int64_t at[COPY_BATCH];
            int rr[COPY_BATCH];
#pragma unroll
            for (int u = 0; u < COPY_BATCH; ++u) {
                const int e = e0 + 64 * u + lane;
                int r = 0;  // the last row starting at or before e
#pragma unroll
                for (int h = 32; h > 0; h >>= 1)
                    if (__shfl(pre, r + h, 64) <= e) r += h;
                const int k = e - __shfl(pre, r, 64);
                const int64_t so = __shfl(sb, r, 64);
                at[u] = __shfl(dst, r, 64) + k;
                rr[u] = r;
                v[u] = e < tot ? A.stage[so + 1 + k] : 0;
            }
            const int flat = fits && (int64_t)len == rl;
#pragma unroll
            for (int u = 0; u < COPY_BATCH; ++u) {
                const int ok = __shfl(flat, rr[u], 64);
                if (ok && e0 + 64 * u + lane < tot) {
                    if (v[u] < 0) atomicAdd(&A.stats[ST_EMIT_MISMATCH], 1ull);
                    col[at[u]] = v[u];
                }
            }
        }
        if (has && len >= 0 && (int64_t)len < rl) atomicAdd(&A.stats[ST_EMIT_MISMATCH], 1ull);
        for (uint64_t m = __ballot(has && (int64_t)len > rl); m; m &= m - 1) {
            const int l = __ffsll((unsigned long long)m) - 1;
            const int64_t lo = uni_lane64(sb, l) + 1, ld = uni_lane64(dst, l), le = ld + uni_lane64(rl, l);
            const int lu = __builtin_amdgcn_readlane(len, l);
            int64_t o = 0;
            for (int k0 = 0; k0 < lu; k0 += 64) {
                const int k = k0 + lane;
                const int32_t x = k < lu ? A.stage[lo + k] : STAGE_REJECT;
                const bool keep = x != STAGE_REJECT;
                const uint64_t bal = __ballot(keep);
                const int64_t at = ld + o + __popcll(bal & lt);
                if (keep && at < le) col[at] = x;
                o += __popcll(bal);
            }
            if (lane == 0 && ld + o != le) atomicAdd(&A.stats[ST_EMIT_MISMATCH], 1ull);
        }
    }
}

// Emit pass after a staged count: the wavefronts whose rows outgrew their
// slots, searched again.  Each wavefront reads 64 flags at a time.
template <bool EXACT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8)))
stage_redo_kernel(SearchArgs A, int64_t *__restrict__ row_ptr, int32_t *__restrict__ col, int gate)
{
    if (A.col_cap >= 0 && uni64(row_ptr[A.n]) > A.col_cap) return;
    if (gate && (__builtin_amdgcn_readfirstlane((int)A.dcount[1]) != 0) != EXACT) return;
    const int lane = threadIdx.x & 63;
    const int64_t waves = (A.n + 63) / 64;
    for (int64_t g0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 64; g0 < waves; g0 += (int64_t)gridDim.x * 256) {
        const int64_t w = g0 + lane;
        for (uint64_t m = __ballot(w < waves && A.sovf[w]); m; m &= m - 1)
            light_wave<M_EMIT, EXACT>(A, (g0 + __ffsll((unsigned long long)m) - 1) * 64, row_ptr, col);
    }
}

// After the fast count pass: decide the listed pairs exactly, count the
// edges among them (the light query's degree, or the heavy chunk's count)
// and enter them in the set the emit pass reads.  Flags an overflowed list.
__global__ void __launch_bounds__(256) resolve_kernel(SearchArgs A, int64_t *__restrict__ row_ptr)
{
    const unsigned long long cnt = A.dcount[0];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if ((int64_t)cnt > A.dcap) A.dcount[1] = 1;
        if (A.use_p32 && cnt) atomicAdd(&A.stats[ST_FP32_UNDECIDED], cnt);
    }
    if ((int64_t)cnt > A.dcap) return;
    const int64_t m = (int64_t)cnt, stride = (int64_t)gridDim.x * 256;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < m; i += stride) {
        const uint64_t key = A.dkeys[i];
        const int64_t q = (int64_t)((key >> 32) & 0x7fffffffull), c = (int64_t)(key & 0xffffffffull);
        const int32_t ch = A.dchunk[i];
        const int edge = edge_p64(A.sr[q], A.st[q], A.sr[c], A.st[c], A.C, A.C_lo, A.stats);
        if (A.staged && ch < 0) {  // the staged row's pending entry, decided
            const int64_t slot = A.dslot[i];
            if (slot >= 0) A.stage[slot] = edge ? (int32_t)A.ids[c] : STAGE_REJECT;
        }
        if (!edge) continue;
        for (uint64_t h = slot_hash(key) & (uint64_t)A.hmask;; h = (h + 1) & (uint64_t)A.hmask) {
            const unsigned long long prev = atomicCAS((unsigned long long *)&A.hset[h], 0ull, (unsigned long long)key);
            if (prev == 0ull || prev == key) break;
        }
        if (ch >= 0) atomicAdd((unsigned long long *)&A.hcnt[ch], 1ull);
        else atomicAdd((unsigned long long *)&row_ptr[__float_as_int(A.rec[q].w) + 1], 1ull);
    }
}

// Before the count pass: heavy_end = the first light position (the end of
// the heavy bands, capped); zero the plan's candidate total.
__global__ void search_prologue(SearchArgs A, int jh, int32_t *heavy_end, int64_t *row_ptr)
{
    if (threadIdx.x == 0) {
        int64_t h = jh > 0 ? (int64_t)A.band_start[jh] : 0;
        if (h > A.heavy_cap) h = A.heavy_cap;
        *heavy_end = (int32_t)h;
        row_ptr[0] = 0;
        A.hscal[0] = 0;
        A.dcount[0] = 0;
        A.dcount[1] = 0;
    }
}

__global__ void __launch_bounds__(256) fill_u8(uint8_t *p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = 0;
}

// Chunk -> item table: after the scan, item i owns chunks
// [hplan[i-1], hplan[i]).
__global__ void __launch_bounds__(256) heavy_chunk_items(SearchArgs A)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= A.heavy_cap * A.B) return;
    const int64_t b = i ? A.hplan[i - 1] : 0, e = A.hplan[i];
    for (int64_t c = b; c < e; ++c) A.hitem[c] = (int32_t)i;
}

// Before the emit pass: flag a col_idx buffer smaller than the graph.
__global__ void emit_prologue(const int64_t *row_ptr, int64_t n, int64_t cap, int32_t *overflow)
{
    if (threadIdx.x == 0 && overflow) *overflow = (cap >= 0 && row_ptr[n] > cap) ? 1 : 0;
}

// After the emit pass: bit 1 of the flag reports rows that the emit pass
// found longer or shorter than the count pass had counted them.
__global__ void emit_epilogue(const unsigned long long *stats, int32_t *overflow)
{
    if (threadIdx.x == 0 && stats[ST_EMIT_MISMATCH]) *overflow |= 2;
}

__global__ void __launch_bounds__(256) zero_i64(int64_t *p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = 0;
}

// After the count pass (and the scan of the chunk counts): heavy degrees.
__global__ void __launch_bounds__(256) heavy_degrees(SearchArgs A, int64_t *__restrict__ row_ptr)
{
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= *A.heavy_end) return;
    const int64_t f = q ? A.hplan[q * A.B - 1] : 0;   // first chunk of q
    const int64_t l = A.hplan[q * A.B + A.B - 1];     // one past its last chunk
    const int64_t hi = l ? A.hcnt[l - 1] : 0, lo = f ? A.hcnt[f - 1] : 0;
    row_ptr[__float_as_int(A.rec[q].w) + 1] = hi - lo;
}

// The search's launch arguments for an index (the emit pass sets col_cap).
static void make_search_args(rhg_index *idx, SearchArgs &A)
{
    const Layout &L = idx->L;
    const rhg_params &p = idx->p;
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
        A.rs_lo[j] = A.sh_lo[j] > 0.0f ? (float)(1.0 / sqrt((double)A.sh_lo[j])) * (1.0f + 0x1p-20f) : 0.0f;
        A.cbits[j] = L.cbits[j];
    }
    A.B = L.B;
    A.band_bits = L.band_bits;
    A.keys = idx->keys;
    A.ids = idx->ids;
    A.n = idx->n;
    A.heavy_cap = idx->heavy_cap;
    A.max_chunks = idx->max_chunks;
    A.heavy_blocks = idx->heavy_cap > 0 ? RHG_HEAVY_BLOCKS : 0;
    A.R = p.R;
    A.C = p.cosh_R;
    A.C_lo = p.cosh_R_lo;
    // The FP32 record stays finite and the screen's bound holds for R < 80,
    // the range every entry point accepts.
    A.use_p32 = (!L.fp64_only && p.R < 80.0) ? 1 : 0;
    A.stream_stage = L.no_stream_stage ? 0 : 1;
    A.sweep_max = L.sweep_max;
    A.sweep_linear = L.sweep_linear;
    A.band_start = idx->band_start;
    A.dir = idx->dir;
    A.sr = idx->sr;
    A.st = idx->st;
    A.rec = idx->rec;
    A.heavy_end = idx->heavy_end;
    A.hplan = idx->hplan;
    A.hcnt = idx->hcnt;
    A.hitem = idx->hitem;
    A.hscal = idx->hscal;
    A.stats = idx->stats;
    A.wstat = (longlong2 *)idx->wstat;
    A.dkeys = idx->dkeys;
    A.dchunk = idx->dchunk;
    A.dcount = idx->dcount;
    A.dcap = L.defer_cap;
    A.hset = idx->hset;
    A.hmask = idx->hset_slots - 1;
    for (int j = 0; j < L.B; ++j) {
        A.lmu_in[j] = L.lmu_in[j];
        A.lmu_out[j] = L.lmu_out[j];
    }
    A.stage_f = L.stage_f;
    A.stage_cap = L.stage_cap;
    A.stage = idx->stage;
    A.sslot = idx->sslot;
    A.sovf = idx->sovf;
    A.wsum = idx->wsum;
    A.dslot = idx->dslot;
    A.staged = L.staged;
    A.light_skip = 0;
}

hipError_t launch_search(rhg_index *idx, int64_t *row_ptr, int32_t *col_idx, int emit, hipStream_t s,
                         int64_t col_cap, int32_t *overflow)
{
    const Layout &L = idx->L;
    SearchArgs A;
    make_search_args(idx, A);
    A.col_cap = col_cap;
    const int64_t n = idx->n;
    const int64_t items = idx->heavy_cap * L.B;
    hipError_t e;
    PhaseScope plan_ps(RHG_PHASE_PLAN, s);  // ended before the search kernels
    if (!emit) {
        hipLaunchKernelGGL(search_prologue, dim3(1), dim3(64), 0, s, A, L.heavy_band, idx->heavy_end, row_ptr);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (n <= 0) return hipSuccess;
        if (L.staged && (e = launch_stage_slots(idx, 1.0f, s)) != hipSuccess) return e;
        if (items > 0) {
            const unsigned g = (unsigned)((items + 255) / 256);
            hipLaunchKernelGGL(heavy_plan_len, dim3(g), dim3(256), 0, s, A);
            hipLaunchKernelGGL(heavy_plan_chunks, dim3(g), dim3(256), 0, s, A);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            if ((e = inclusive_scan_i64(idx->hplan, items, idx->tmp, s)) != hipSuccess) return e;
            hipLaunchKernelGGL(heavy_chunk_items, dim3(g), dim3(256), 0, s, A);
            hipLaunchKernelGGL(zero_i64, dim3((unsigned)((idx->max_chunks + 255) / 256)), dim3(256), 0, s, idx->hcnt,
                               idx->max_chunks);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
    } else {
        if (overflow) {
            hipLaunchKernelGGL(emit_prologue, dim3(1), dim3(64), 0, s, row_ptr, n, col_cap, overflow);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
        if (n <= 0) return hipSuccess;
    }
    plan_ps.end();
    const dim3 g((unsigned)(A.heavy_blocks + (n + 255) / 256)), b(256);
    // the EXACT kernels, when they only stand by for an overflowed list,
    // run on a smaller grid (a smaller heavy pool; the light part strides)
    SearchArgs Ax = A;
    Ax.heavy_blocks = std::min(A.heavy_blocks, 64);
    const dim3 gx((unsigned)(Ax.heavy_blocks + std::min<int64_t>((n + 255) / 256, 64)));
    // with no FP32 screen (or on request) every undecided pair is decided
    // in place: the EXACT kernels alone
    const bool exact_only = !A.use_p32 || L.exact_inline;
    if (!emit && !exact_only && A.hmask >= 0)
        hipLaunchKernelGGL(zero_i64, dim3((unsigned)((A.hmask + 256) / 256)), dim3(256), 0, s, (int64_t *)A.hset,
                           A.hmask + 1);
    // staged: the count pass writes the light rows into their slots, the
    // emit pass copies them, emits the heavy chunks and searches again the
    // wavefronts whose rows outgrew their slots
    const bool staged = emit ? idx->staged_count != 0 : L.staged != 0;
    if (emit && staged) {
        A.light_skip = 1;
        Ax.light_skip = 1;
    }
    const dim3 gh((unsigned)std::max(A.heavy_blocks, 1)), ghx((unsigned)std::max(Ax.heavy_blocks, 1));
    const int64_t lwaves = (n + 63) / 64;
    const dim3 gr((unsigned)std::max<int64_t>(1, std::min<int64_t>((lwaves + 255) / 256, 4096)));
    {
        PhaseScope ps(emit ? RHG_PHASE_EMIT_PASS : RHG_PHASE_COUNT_PASS, s);
        if (emit && staged) {
            if (A.heavy_blocks > 0) {
                if (exact_only) hipLaunchKernelGGL((search_kernel<M_EMIT, true>), gh, b, 0, s, A, row_ptr, col_idx, 0);
                else hipLaunchKernelGGL((search_kernel<M_EMIT, false>), gh, b, 0, s, A, row_ptr, col_idx, 1);
            }
            if ((e = hipGetLastError()) != hipSuccess) return e;
            if ((e = launch_stage_copy(idx, row_ptr, col_idx, col_cap, s)) != hipSuccess) return e;
            if (exact_only) hipLaunchKernelGGL(stage_redo_kernel<true>, gr, b, 0, s, A, row_ptr, col_idx, 0);
            else hipLaunchKernelGGL(stage_redo_kernel<false>, gr, b, 0, s, A, row_ptr, col_idx, 1);
        } else if (exact_only) {
            if (emit) hipLaunchKernelGGL((search_kernel<M_EMIT, true>), g, b, 0, s, A, row_ptr, col_idx, 0);
            else if (staged) hipLaunchKernelGGL((search_kernel<M_STAGE, true>), g, b, 0, s, A, row_ptr, col_idx, 0);
            else hipLaunchKernelGGL((search_kernel<M_COUNT, true>), g, b, 0, s, A, row_ptr, col_idx, 0);
        } else if (emit) {
            hipLaunchKernelGGL((search_kernel<M_EMIT, false>), g, b, 0, s, A, row_ptr, col_idx, 1);
        } else if (staged) {
            hipLaunchKernelGGL((search_kernel<M_STAGE, false>), g, b, 0, s, A, row_ptr, col_idx, 1);
        } else {
            hipLaunchKernelGGL((search_kernel<M_COUNT, false>), g, b, 0, s, A, row_ptr, col_idx, 1);
        }
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (!exact_only) {
        PhaseScope ps(RHG_PHASE_PLAN, s);
        if (!emit) {
            hipLaunchKernelGGL(resolve_kernel, dim3(256), dim3(256), 0, s, A, row_ptr);
            if (staged) hipLaunchKernelGGL((search_kernel<M_STAGE, true>), gx, b, 0, s, Ax, row_ptr, col_idx, 1);
            else hipLaunchKernelGGL((search_kernel<M_COUNT, true>), gx, b, 0, s, Ax, row_ptr, col_idx, 1);
        } else if (staged) {
            if (A.heavy_blocks > 0)
                hipLaunchKernelGGL((search_kernel<M_EMIT, true>), ghx, b, 0, s, Ax, row_ptr, col_idx, 1);
            hipLaunchKernelGGL(stage_redo_kernel<true>, dim3(std::min(gr.x, 64u)), b, 0, s, Ax, row_ptr, col_idx, 1);
        } else {
            hipLaunchKernelGGL((search_kernel<M_EMIT, true>), gx, b, 0, s, Ax, row_ptr, col_idx, 1);
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (!emit) idx->staged_count = staged ? 1 : 0;
    if (emit && overflow) {
        hipLaunchKernelGGL(emit_epilogue, dim3(1), dim3(64), 0, s, (const unsigned long long *)idx->stats, overflow);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (!emit && items > 0) {
        PhaseScope ps(RHG_PHASE_PLAN, s);
        if ((e = inclusive_scan_i64(idx->hcnt, idx->max_chunks, idx->tmp, s)) != hipSuccess) return e;
        hipLaunchKernelGGL(heavy_degrees, dim3((unsigned)((idx->heavy_cap + 255) / 256)), dim3(256), 0, s, A,
                           row_ptr);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (!emit && staged) e = launch_stage_split(idx, row_ptr, s);
    return e;
}

// The staging slots' starts before a staged count (per wavefront its
// slots' words, then their inclusive prefix) and the overflow flags
// cleared; the slots' sizes scaled by `scale`.  heavy_end must be set.
hipError_t launch_stage_slots(rhg_index *idx, float scale, hipStream_t s)
{
    SearchArgs A;
    make_search_args(idx, A);
    A.stage_f *= scale;
    const int64_t waves = (idx->n + 63) / 64;
    if (waves <= 0) return hipSuccess;
    hipLaunchKernelGGL(stage_wave_words, dim3((unsigned)std::min<int64_t>((waves + 3) / 4, 8192)), dim3(256), 0, s,
                       A, idx->wsum, waves);
    hipLaunchKernelGGL(fill_u8, dim3((unsigned)((waves + 255) / 256)), dim3(256), 0, s, idx->sovf, waves);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return inclusive_scan_i64(idx->wsum, waves, idx->tmp, s);
}

// After a staged count (the heavy rows' degrees written): the slot starts
// split off the degrees.
hipError_t launch_stage_split(rhg_index *idx, int64_t *row_ptr, hipStream_t s)
{
    if (idx->n <= 0) return hipSuccess;
    PhaseScope ps(RHG_PHASE_PLAN, s);
    hipLaunchKernelGGL(stage_split_kernel, dim3((unsigned)((idx->n + 255) / 256)), dim3(256), 0, s, row_ptr,
                       idx->sslot, idx->n);
    return hipGetLastError();
}

// Emit pass after a staged count: the light rows copied from their slots.
hipError_t launch_stage_copy(rhg_index *idx, const int64_t *row_ptr, int32_t *col_idx, int64_t col_cap,
                             hipStream_t s)
{
    SearchArgs A;
    make_search_args(idx, A);
    A.col_cap = col_cap;
    const int64_t waves = (idx->n + 63) / 64;
    if (waves <= 0) return hipSuccess;
    hipLaunchKernelGGL(stage_copy_kernel, dim3((unsigned)std::min<int64_t>((waves + 3) / 4, 16384)), dim3(256), 0, s,
                       A, row_ptr, col_idx);
    return hipGetLastError();
}


// ------------------------------------------------------------ listed rows
//
// The rows of a list of vertices (their sorted positions qpos[0..k)) on the
// whole index: a wavefront per query, every band's window (or the whole
// band inside the circle) tested 64 candidates at a time with the exact
// decision in place.  The count pass writes each row's length to cnt[i];
// the emit pass writes row i to ocol[optr[i] ..) in (band, position) order.
template <int MODE>
__global__ void __launch_bounds__(256) query_rows_kernel(SearchArgs A, const int32_t *__restrict__ qpos, int64_t k,
                                                         int64_t *__restrict__ cnt, const int64_t *__restrict__ optr,
                                                         int32_t *__restrict__ ocol)
{
    constexpr bool EMIT = MODE == M_EMIT;
    const int lane = threadIdx.x & 63;
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    const int64_t waves = (int64_t)gridDim.x * 4;
    for (int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); i < k; i += waves) {
        const int64_t q = qpos[i];
        const double rq = A.sr[q], tq = A.st[q];
        const float4 fq = A.rec[q];
        int64_t c_out = 0, base = 0, lim = 0;
        if (EMIT) {
            base = optr[i];
            lim = optr[i + 1] - base;
        }
        for (int j = 0; j < A.B; ++j) {
            const int64_t s = A.band_start[j], e = A.band_start[j + 1];
            if (s == e) continue;
            int64_t ra[2], rb[2];
            int nr = 1;
            bool inside = false, fp = true;
            if (band_inside(A, rq, j)) {
                ra[0] = s; rb[0] = e; inside = true;
            } else {
                const double w = window_w(A, fq.x, fq.y, fq.z, j);
                if (w >= 3.0) { ra[0] = s; rb[0] = e; }
                else nr = window_runs(A, j, tq - w, tq + w, s, e, ra, rb);
                fp = !(w + RHG_TWO_PI_D * ldexp(1.0, -A.cbits[j]) < 0x1p-5);
            }
            for (int r = 0; r < nr; ++r) {
                for (int64_t c0 = ra[r]; c0 < rb[r]; c0 += 64) {
                    const int64_t c = c0 + lane;
                    int acc = 0;
                    float4 fc = make_float4(0.f, 0.f, 0.f, 0.f);
                    if (c < rb[r] && c != q) {
                        fc = A.rec[c];
                        acc = inside ? 1
                                     : decide<MODE, true>(A, q, tq, fq.x, fq.y, fq.z, c, A.st[c], fc.x, fc.y, fc.z,
                                                          fp, -1);
                    }
                    const uint64_t bal = __ballot(acc);
                    if (EMIT && acc) {
                        const int64_t o = c_out + __popcll(bal & lt);
                        if (o < lim) ocol[base + o] = __float_as_int(fc.w);
                    }
                    c_out += __popcll(bal);
                }
            }
        }
        if (lane == 0) {
            if (!EMIT) cnt[i] = c_out;
            else if (c_out != lim) atomicAdd(&A.stats[ST_EMIT_MISMATCH], 1ull);
        }
    }
}

hipError_t launch_query_rows(rhg_index *idx, const int32_t *qpos, int64_t k, int64_t *cnt, const int64_t *optr,
                             int32_t *ocol, int emit, hipStream_t s)
{
    if (k <= 0) return hipSuccess;
    SearchArgs A;
    make_search_args(idx, A);
    const unsigned g = (unsigned)std::min<int64_t>((k + 3) / 4, 16384);
    if (emit) hipLaunchKernelGGL(query_rows_kernel<M_EMIT>, dim3(g), dim3(256), 0, s, A, qpos, k, cnt, optr, ocol);
    else hipLaunchKernelGGL(query_rows_kernel<M_COUNT>, dim3(g), dim3(256), 0, s, A, qpos, k, cnt, optr, ocol);
    return hipGetLastError();
}

// ------------------------------------------------------------ small graphs
//
// A batch's small graphs (n <= RHG_SMALL_GRAPH) are generated by one
// persistent launch: each workgroup takes the next graph from a device
// counter and runs its whole pipeline -- sample, sort, index, count, scan,
// emit -- alone, with workgroup barriers between the steps, so a small
// graph costs no kernel launches of its own.  The composite keys
// (sort key, id) of up to RHG_SMALL_GRAPH points are sorted in LDS by a
// bitonic network (unique keys, so the order is deterministic); the band
// windows are found by binary search on the sorted keys; each wavefront
// takes one query at a time and its lanes test the candidates 64 at a
// time, with the exact stages decided in place.  Rows hold the inside bands,
// then each band's window in position order.

struct SmallGraph {
    SearchArgs A;                 // bands, constants and the sorted arrays below
    int64_t n;
    uint32_t k0, k1;              // Philox key
    double alpha, cam1, cam1_lo;  // cosh(alpha R) - 1 as double-double
    double *r, *theta;
    int64_t *row_ptr;
    int32_t *col;
    int64_t col_cap;
    int32_t *overflow;
    uint32_t *keys;
    double inv, sc;               // 1 / sqrt(2 cosh R), sqrt(2 / cosh R)
};

constexpr int SMALL_THREADS = 1024;

__device__ __forceinline__ int small_band_of(const SearchArgs &A, double r)
{
    int lo = 0, hi = A.B - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (A.E[mid] <= r) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// One query (sorted position q) by one wavefront: count or emit its row.
template <int MODE>
__device__ void small_query(const SmallGraph &S, int64_t q, const uint64_t *skey, const int32_t *bstart,
                            int *mismatch)
{
    constexpr bool EMIT = MODE == M_EMIT;
    const SearchArgs &A = S.A;
    const int lane = threadIdx.x & 63;
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    const double rq = A.sr[q], tq = A.st[q];
    const float4 fq = A.rec[q];
    const int32_t id = __float_as_int(fq.w);
    int J = 0;
    while (J < A.B && band_inside(A, rq, J)) ++J;
    int64_t cnt = 0, base = 0, lim = 0;
    if (EMIT) {
        base = S.row_ptr[id];
        lim = S.row_ptr[id + 1] - base;
    }
    // inside bands, without tests
    {
        const int64_t s0 = bstart[0], e0 = bstart[J];
        if (EMIT) {
            for (int64_t c0 = s0; c0 < e0; c0 += 64) {
                const int64_t c = c0 + lane;
                const bool valid = c < e0 && c != q;
                const uint64_t bal = __ballot(valid);
                if (valid) {
                    const int64_t o = cnt + __popcll(bal & lt);
                    if (o < lim) S.col[base + o] = (int32_t)(skey[c] & 0xffffffffull);
                }
                cnt += __popcll(bal);
            }
        } else {
            cnt = (e0 - s0) - ((q >= s0 && q < e0) ? 1 : 0);
        }
    }
    // first position in [s, e) whose sort key is at least k (or above k)
    auto lower = [&](int64_t s, int64_t e, uint32_t k, bool above) {
        while (s < e) {
            const int64_t mid = (s + e) >> 1;
            const uint32_t km = (uint32_t)(skey[mid] >> 32);
            if (above ? km <= k : km < k) s = mid + 1;
            else e = mid;
        }
        return s;
    };
    for (int j = J; j < A.B; ++j) {
        const int64_t s = bstart[j], e = bstart[j + 1];
        if (s == e) continue;
        const double w = window_w(A, fq.x, fq.y, fq.z, j);
        const bool fp = !(w < 0x1p-5);
        int64_t ra[3], rb[3];
        int nr = 0;
        if (!(w < 3.0)) {
            ra[0] = s; rb[0] = e; nr = 1;
        } else {
            const double lo = tq - w, hi = tq + w;
            if (hi >= RHG_TWO_PI_D) {
                ra[nr] = s; rb[nr] = lower(s, e, band_key(A, j, hi - RHG_TWO_PI_D), true); ++nr;
            }
            ra[nr] = lower(s, e, band_key(A, j, fmax(lo, 0.0)), false);
            rb[nr] = lower(s, e, band_key(A, j, fmin(hi, RHG_TWO_PI_D)), true);
            ++nr;
            if (lo < 0.0) {
                ra[nr] = lower(s, e, band_key(A, j, lo + RHG_TWO_PI_D), false); rb[nr] = e; ++nr;
            }
        }
        for (int k = 0; k < nr; ++k) {
            for (int64_t c0 = ra[k]; c0 < rb[k]; c0 += 64) {
                const int64_t c = c0 + lane;
                int acc = 0;
                if (c < rb[k] && c != q) {
                    const double tc = A.st[c];
                    if (!(short_angle(tq, tc) > w)) {
                        const float4 fc = A.rec[c];
                        acc = decide<MODE, true>(A, q, tq, fq.x, fq.y, fq.z, c, tc, fc.x, fc.y, fc.z, fp, -1);
                    }
                }
                const uint64_t bal = __ballot(acc);
                if (EMIT && acc) {
                    const int64_t o = cnt + __popcll(bal & lt);
                    if (o < lim) S.col[base + o] = (int32_t)(skey[c] & 0xffffffffull);
                }
                cnt += __popcll(bal);
            }
        }
    }
    if (lane == 0) {
        if (!EMIT) S.row_ptr[id + 1] = cnt;
        else if (cnt != lim) *mismatch = 1;
    }
}

// One query by one lane (the outer points: few candidates per band), with
// the same window runs and row order as small_query.
template <int MODE>
__device__ void small_query_lane(const SmallGraph &S, int64_t q, const uint64_t *skey, const int32_t *bstart,
                                 int *mismatch)
{
    constexpr bool EMIT = MODE == M_EMIT;
    const SearchArgs &A = S.A;
    const double rq = A.sr[q], tq = A.st[q];
    const float4 fq = A.rec[q];
    const int32_t id = __float_as_int(fq.w);
    int J = 0;
    while (J < A.B && band_inside(A, rq, J)) ++J;
    int64_t cnt = 0, base = 0, lim = 0;
    if (EMIT) {
        base = S.row_ptr[id];
        lim = S.row_ptr[id + 1] - base;
    }
    {
        const int64_t s0 = bstart[0], e0 = bstart[J];
        if (EMIT) {
            for (int64_t c = s0; c < e0; ++c) {
                if (c == q) continue;
                if (cnt < lim) S.col[base + cnt] = (int32_t)(skey[c] & 0xffffffffull);
                ++cnt;
            }
        } else {
            cnt = (e0 - s0) - ((q >= s0 && q < e0) ? 1 : 0);
        }
    }
    auto lower = [&](int64_t s, int64_t e, uint32_t k, bool above) {
        while (s < e) {
            const int64_t mid = (s + e) >> 1;
            const uint32_t km = (uint32_t)(skey[mid] >> 32);
            if (above ? km <= k : km < k) s = mid + 1;
            else e = mid;
        }
        return s;
    };
    for (int j = J; j < A.B; ++j) {
        const int64_t s = bstart[j], e = bstart[j + 1];
        if (s == e) continue;
        const double w = window_w(A, fq.x, fq.y, fq.z, j);
        const bool fp = !(w < 0x1p-5);
        int64_t ra[3], rb[3];
        int nr = 0;
        if (!(w < 3.0)) {
            ra[0] = s; rb[0] = e; nr = 1;
        } else {
            const double lo = tq - w, hi = tq + w;
            if (hi >= RHG_TWO_PI_D) {
                ra[nr] = s; rb[nr] = lower(s, e, band_key(A, j, hi - RHG_TWO_PI_D), true); ++nr;
            }
            ra[nr] = lower(s, e, band_key(A, j, fmax(lo, 0.0)), false);
            rb[nr] = lower(s, e, band_key(A, j, fmin(hi, RHG_TWO_PI_D)), true);
            ++nr;
            if (lo < 0.0) {
                ra[nr] = lower(s, e, band_key(A, j, lo + RHG_TWO_PI_D), false); rb[nr] = e; ++nr;
            }
        }
        for (int k = 0; k < nr; ++k)
            for (int64_t c = ra[k]; c < rb[k]; ++c) {
                if (c == q) continue;
                const double tc = A.st[c];
                if (short_angle(tq, tc) > w) continue;
                const float4 fc = A.rec[c];
                if (decide<MODE, true>(A, q, tq, fq.x, fq.y, fq.z, c, tc, fc.x, fc.y, fc.z, fp, -1)) {
                    if (EMIT && cnt < lim) S.col[base + cnt] = (int32_t)(skey[c] & 0xffffffffull);
                    ++cnt;
                }
            }
    }
    if (!EMIT) S.row_ptr[id + 1] = cnt;
    else if (cnt != lim) *mismatch = 1;
}

// Sorted positions below this many (the innermost points, whose windows
// hold the most candidates) are searched a wavefront per query, the rest a
// lane per query.
constexpr int64_t SMALL_WAVE_QUERIES = 512;

__global__ void __launch_bounds__(SMALL_THREADS) small_batch_kernel(const SmallGraph *G, int count,
                                                                    unsigned int *head)
{
    __shared__ uint64_t skey[RHG_SMALL_GRAPH];
    __shared__ dd tab[LOGT_N];
    __shared__ int32_t bstart[RHG_MAX_BANDS + 1];
    __shared__ int64_t part[SMALL_THREADS / 64];
    __shared__ int gnext, mismatch;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nwave = SMALL_THREADS / 64;
    fill_log_table(tab, tid, SMALL_THREADS);
    for (;;) {
        __syncthreads();
        if (tid == 0) {
            gnext = (int)atomicAdd(head, 1u);
            mismatch = 0;
        }
        __syncthreads();
        const int g = gnext;
        if (g >= count) return;
        const SmallGraph &S = G[g];
        const SearchArgs &A = S.A;
        const int64_t n = S.n;
        int64_t P = 2;
        while (P < n) P <<= 1;
        // sample; composite keys (sort key, id)
        for (int64_t i = tid; i < P; i += SMALL_THREADS) {
            uint64_t k = ~0ull;
            if (i < n) {
                double ri, ti;
                sample_point(i, S.k0, S.k1, S.alpha, A.R, S.cam1, S.cam1_lo, tab, &ri, &ti);
                S.r[i] = ri;
                S.theta[i] = ti;
                const uint32_t b = (uint32_t)small_band_of(A, ri);
                const uint32_t ak = angle_key_s(ti);
                const uint32_t key = A.band_bits ? ((b << (32 - A.band_bits)) | (ak >> A.band_bits)) : ak;
                k = ((uint64_t)key << 32) | (uint64_t)i;
            }
            skey[i] = k;
        }
        __syncthreads();
        // bitonic sort of the P keys, ascending
        for (int64_t kk = 2; kk <= P; kk <<= 1)
            for (int64_t jj = kk >> 1; jj > 0; jj >>= 1) {
                for (int64_t i = tid; i < P; i += SMALL_THREADS) {
                    const int64_t l = i ^ jj;
                    if (l > i) {
                        const uint64_t a = skey[i], b = skey[l];
                        if ((a > b) == ((i & kk) == 0)) {
                            skey[i] = b;
                            skey[l] = a;
                        }
                    }
                }
                __syncthreads();
            }
        // sorted records; band starts
        for (int64_t p = tid; p < n; p += SMALL_THREADS) {
            const uint32_t id = (uint32_t)(skey[p] & 0xffffffffull);
            const double ri = S.r[id], ti = S.theta[id];
            S.keys[p] = (uint32_t)(skey[p] >> 32);
            ((double *)A.sr)[p] = ri;
            ((double *)A.st)[p] = ti;
            ((float4 *)A.rec)[p] = make_float4((float)(exp(ri) * S.inv), (float)(exp(-ri) * S.inv),
                                               (float)(sinh(ri) * S.sc), __int_as_float((int)id));
        }
        if (tid <= A.B) {
            int64_t pos = n;
            if (tid < A.B) {
                const uint64_t k = (uint64_t)(A.band_bits ? ((uint32_t)tid << (32 - A.band_bits)) : 0u) << 32;
                int64_t s = 0, e = n;
                while (s < e) {
                    const int64_t mid = (s + e) >> 1;
                    if (skey[mid] < k) s = mid + 1; else e = mid;
                }
                pos = tid == 0 ? 0 : s;
            }
            bstart[tid] = (int32_t)pos;
        }
        if (tid == 0) S.row_ptr[0] = 0;
        __syncthreads();
        // count pass: the innermost queries one per wavefront, the rest one
        // per lane
        const int64_t hq = n < SMALL_WAVE_QUERIES ? n : SMALL_WAVE_QUERIES;
        for (int64_t q = wave; q < hq; q += nwave) small_query<M_COUNT>(S, q, skey, bstart, &mismatch);
        for (int64_t q = hq + tid; q < n; q += SMALL_THREADS) small_query_lane<M_COUNT>(S, q, skey, bstart, &mismatch);
        __syncthreads();
        // row offsets: inclusive scan of row_ptr[1 .. n] in steps of 1024
        int64_t carry = 0;
        for (int64_t b0 = 0; b0 < n; b0 += SMALL_THREADS) {
            const int64_t i = b0 + tid;
            int64_t v = i < n ? S.row_ptr[1 + i] : 0;
            int64_t tot;
            int64_t x = v - 0;
            const int64_t ex = wave_excl_sum64(x, lane, &tot);
            if (lane == 0) part[wave] = tot;
            __syncthreads();
            int64_t before = 0, all = 0;
            for (int w2 = 0; w2 < nwave; ++w2) {
                if (w2 < wave) before += part[w2];
                all += part[w2];
            }
            if (i < n) S.row_ptr[1 + i] = carry + before + ex + v;
            carry += all;
            __syncthreads();
        }
        const int64_t nnz = carry;
        if (nnz > S.col_cap) {
            if (tid == 0) *S.overflow = 1;
            continue;
        }
        // emit pass
        for (int64_t q = wave; q < hq; q += nwave) small_query<M_EMIT>(S, q, skey, bstart, &mismatch);
        for (int64_t q = hq + tid; q < n; q += SMALL_THREADS) small_query_lane<M_EMIT>(S, q, skey, bstart, &mismatch);
        __syncthreads();
        if (tid == 0) *S.overflow = mismatch ? 2 : 0;
    }
}

__global__ void small_batch_reset(unsigned int *head)
{
    if (threadIdx.x == 0) *head = 0u;
}

size_t small_graph_record_bytes() { return sizeof(SmallGraph); }

// Fills the device record of a small graph (host memory `out`, copied to the
// device by the caller).  Returns false when the workspace is too small.
bool make_small_graph(const rhg_params &p, const Layout &L, double *r, double *theta, void *ws, size_t ws_bytes,
                      int64_t *row_ptr, int32_t *col, int64_t col_cap, int32_t *overflow,
                      unsigned long long *stats, void *out)
{
    SmallGraph &G = *(SmallGraph *)out;
    memset(&G, 0, sizeof(G));
    SearchArgs &A = G.A;
    const int64_t n = p.n;
    const size_t N = (size_t)(n > 0 ? n : 1);
    char *b = (char *)align_up((size_t)ws, 256);
    const size_t need = align_up(4 * N, 256) + 2 * align_up(8 * N, 256) + align_up(16 * N, 256) + 256;
    if (!ws || ws_bytes < need) return false;
    G.keys = (uint32_t *)b;
    b += align_up(4 * N, 256);
    A.sr = (const double *)b;
    b += align_up(8 * N, 256);
    A.st = (const double *)b;
    b += align_up(8 * N, 256);
    A.rec = (const float4 *)b;
    G.inv = 1.0 / sqrt(2.0 * p.cosh_R);
    G.sc = sqrt(2.0 / p.cosh_R);
    for (int j = 0; j <= L.B; ++j) A.E[j] = L.E[j];
    for (int j = 0; j < L.B; ++j) {
        A.ep_lo[j] = (float)(exp(L.E[j]) * G.inv);
        A.em_lo[j] = (float)(exp(-L.E[j]) * G.inv);
        A.sh_lo[j] = (float)(sinh(L.E[j]) * G.sc);
        A.rs_lo[j] = A.sh_lo[j] > 0.0f ? (float)(1.0 / sqrt((double)A.sh_lo[j])) * (1.0f + 0x1p-20f) : 0.0f;
        A.cbits[j] = L.cbits[j];
    }
    A.B = L.B;
    A.band_bits = L.band_bits;
    A.n = n;
    A.R = p.R;
    A.C = p.cosh_R;
    A.C_lo = p.cosh_R_lo;
    A.use_p32 = (!L.fp64_only && p.R < 80.0) ? 1 : 0;
    A.keys = G.keys;
    A.stats = stats;
    G.n = n;
    G.k0 = (uint32_t)p.seed;
    G.k1 = (uint32_t)(p.seed >> 32);
    G.alpha = p.alpha;
    G.cam1 = p.cosh_aR_m1;
    G.cam1_lo = p.cosh_aR_m1_lo;
    G.r = r;
    G.theta = theta;
    G.row_ptr = row_ptr;
    G.col = col;
    G.col_cap = col_cap;
    G.overflow = overflow;
    return true;
}

hipError_t launch_small_batch(const void *table, int count, unsigned int *head, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(small_batch_reset, dim3(1), dim3(64), 0, s, head);
    const int grid = std::min(count, 256);
    hipLaunchKernelGGL(small_batch_kernel, dim3(grid), dim3(SMALL_THREADS), 0, s, (const SmallGraph *)table, count,
                       head);
    return hipGetLastError();
}

}  // namespace rhg
