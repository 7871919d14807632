// rhg_temp.hip -- the neighbour search of the temperature model: the
// distance-dependent connection probability that Sec. 2.1 sets aside, taken
// in Krioukov et al.'s Fermi-Dirac form with curvature 1,
//     p(d) = 1 / (1 + e^{(d - R) / (2T)}),  0 < T < 1.
// Pair {i, j} draws one coin u = a 2^-53, a = k + 1 in [1, 2^53], k the top
// 53 bits of the word (x1:x0) of the Philox4x32-10 block with key
// (seed_lo, seed_hi) and counter (min(i,j), max(i,j), 2, 0), and is an edge
// iff u < p(d).  With b = 2^53 - a (so that (1 - u)/u = b/a exactly):
//     u < p(d)  <=>  d < D = R + 2T ln(b/a)  <=>  cosh d < cosh D,
// never when b = 0 or D <= 0.
//
// Truncation.  The smallest coin is 2^-53, so a pair can be an edge only if
// p(d) > 2^-53, i.e. d < rho = R + 2T ln(2^53 - 1): the search is the
// threshold search of radius rho on the same index (bands, cells, sorted
// records), and the rule cuts nothing the model could join.
//
// Exact decision per candidate inside the windows:
//   P32  P = cosh d / cosh R from the FP32 records, as in the threshold
//        search (relative error <= 21 u, u = 2^-24, plus 2^-34 absolute);
//        P > K (1 + 2^-16), K = cosh(rho) / cosh(R): beyond rho, no coin.
//   coin, then in FP32 the threshold c = cosh D / cosh R
//        = (e^x + e^{-2R - x}) / (1 + e^{-2R}),  x = 2T ln(b/a),
//        from log2f / exp2f of the coin's integers (relative error of c
//        below 2^-15 for T < 1; see the design notes), so P and c more than
//        2^-12 max(P, c) + 2^-32 apart decide the pair;
//   P64  binary64 (cosh d and cosh D, margin 2^-30), and
//   DD   double-double for the rest.
//
// Work split.  As in the threshold search: the innermost (heavy) queries
// are split into (query, band, chunk) work items of a workgroup each; every
// other query is one lane of a wavefront of 64 consecutive sorted
// positions, which walks its own window in every band.  Rows come out in
// (band, position) order; the emit pass repeats the count pass's work in
// the same order, or, staged (large graphs), the count pass also writes
// each light row into its slot of the index's staging area (the threshold
// search's slots) and the emit pass searches only the heavy chunks again,
// copies the light rows and searches again the wavefronts whose rows
// outgrew a slot.
#include <string.h>

#include <algorithm>

#include "rhg_geom.h"
#include "rhg_internal.h"
#include "rhg_philox.h"

namespace rhg {

struct TempArgs {
    double E[RHG_MAX_BANDS + 1];      // band edges
    float ep_lo[RHG_MAX_BANDS];       // e'(E[j]), m'(E[j]), s'(E[j]) of the records
    float em_lo[RHG_MAX_BANDS];
    float sh_lo[RHG_MAX_BANDS];
    int64_t dir_base[RHG_MAX_BANDS + 1];
    int cbits[RHG_MAX_BANDS];
    int B;
    int64_t n;
    int64_t heavy_cap, max_chunks;
    int heavy_blocks;
    double R, twoT;                   // R and 2T
    float K;                          // cosh(rho) / cosh(R), rounded up
    float Ktr;                        // K (1 + 2^-16): the truncation test
    float twoTf;                      // 2T
    float RL2E;                       // R log2(e)
    float R2L2E;                      // 2 R log2(e)
    float f1;                         // 1 / (1 + e^{-2R})
    int use_p32;
    uint32_t k0, k1;                  // coin key
    const int32_t *band_start;
    const int32_t *dir;
    const double *sr, *st;
    const float4 *rec;
    const int32_t *heavy_end;
    int64_t *hplan, *hcnt;
    int32_t *hitem;
    int64_t *hscal;
    unsigned long long *stats;
    // pairs the FP32 stage leaves undecided (as in the threshold search):
    // listed by the count pass, decided by the resolving kernel, which adds
    // the edges to the degrees and to the set the emit pass reads
    uint64_t *dkeys;
    int32_t *dchunk;
    unsigned long long *dcount;       // [0] pairs listed, [1] the list overflowed
    int64_t dcap;
    uint64_t *hset;
    int64_t hmask;
    int64_t col_cap;                  // emit pass: capacity of col_idx (< 0: unchecked)
    int tally;                        // count pass: this launch adds to the candidate and coin tallies
    longlong2 *tal;                   // per-wavefront table of (candidates, coins)
    int64_t tal_slots;
    // staged count: each light query's row goes to its slot (sized as in
    // the threshold search, wavefront w's slots from wsum[w - 1]), its
    // length first (-1: the wavefront outgrew a slot), then its entries;
    // an undecided entry carries STAGE_PENDING until the resolving kernel
    // writes the id or STAGE_REJECT; wavefronts with a row longer than its
    // slot are flagged in sovf
    float lmu_in[RHG_MAX_BANDS], lmu_out[RHG_MAX_BANDS];
    float stage_f;
    int band_bits;
    const uint32_t *keys;
    int32_t *stage;
    int64_t stage_cap;
    const int64_t *wsum;
    uint8_t *sovf;
    int64_t *dslot;
    int staged;                       // count pass: stage the light rows
    int light_skip;                   // emit pass after a staged count: heavy chunks only
};

// T_STAGE: counted as T_COUNT, the light rows also written to their slots.
enum { T_COUNT = 0, T_EMIT = 1, T_STAGE = 2 };

// The pair's coin: a = k + 1 in [1, 2^53].
__device__ __forceinline__ uint64_t temp_coin(uint32_t ida, uint32_t idb, uint32_t k0, uint32_t k1)
{
    uint32_t c0 = min(ida, idb), c1 = max(ida, idb), c2 = 2u, c3 = 0u;
    philox4x32_10(c0, c1, c2, c3, k0, k1);
    return ((((uint64_t)c1 << 32) | c0) >> 11) + 1;
}

// binary64, then double-double: u = a 2^-53 < p(d) for the points (rq, tq)
// and (rc, tc).  Rare (pairs the FP32 stage leaves undecided).
__device__ __noinline__ int temp_exact(double rq, double tq, double rc, double tc, uint64_t a, double R,
                                       double twoT, unsigned long long *stats, int count_pass)
{
    if (count_pass) atomicAdd(&stats[ST_FP32_UNDECIDED], 1ull);
    const uint64_t b = (1ull << 53) - a;
    if (b == 0) return 0;
    const double ad = (double)a, bd = (double)b;  // exact
    const double D = R + twoT * log(bd / ad);
    if (D < -0x1p-30) return 0;
    if (D > 0x1p-30) {
        const double L = cosh_dist64(rq, tq, rc, tc);
        const double C = cosh(D);
        if (L < C * (1.0 - 0x1p-30)) return 1;
        if (L > C * (1.0 + 0x1p-30)) return 0;
    }
    atomicAdd(&stats[ST_DD], 1ull);
    // ln(b/a) = +-log1p(|b - a| / min(a, b)); b - a is exact
    const dd lr = bd >= ad ? dd_log1p(dd_div(dd_make(bd - ad), dd_make(ad)))
                           : dd_neg(dd_log1p(dd_div(dd_make(ad - bd), dd_make(bd))));
    const dd Dd = dd_add_d(dd_mul_d(lr, twoT), R);
    if (fabs(Dd.hi) <= 1e-26) atomicAdd(&stats[ST_TIES], 1ull);
    if (Dd.hi <= 0.0) return 0;
    const dd C = dd_cosh(Dd);
    const dd diff = dd_sub(cosh_dist_dd(rq, tq, rc, tc), C);
    if (fabs(diff.hi) <= 1e-26 * C.hi) atomicAdd(&stats[ST_TIES], 1ull);
    return diff.hi < 0.0;
}

// The pair (query q, candidate c, both sorted positions): the FP32 stage,
// then the exact test.  EXACT decides it here (temp_exact is a call that
// needs a stack and the caller's registers, so the fast kernels keep it
// out): the count pass instead lists the pair for the resolving kernel and
// counts it there if it is an edge, and the emit pass finds the resolved
// edges in the set.  1 edge, 0 not, 2 (a staged light row's pair) listed
// by the caller with its staging entry.  The count pass tallies the coins it
// draws in `coins`; `chunk` is the heavy chunk of the pair (-1: light).
template <int MODE, bool EXACT>
__device__ __forceinline__ int temp_decide(const TempArgs &A, int64_t q, double tq, float4 fq, int64_t c,
                                           double tc, float4 fc, int &coins, int64_t chunk)
{
    const uint32_t idq = (uint32_t)__float_as_int(fq.w), idc = (uint32_t)__float_as_int(fc.w);
    int v = 2;
    uint64_t a = 0;
    if (!A.use_p32) {
        if (MODE != T_EMIT) ++coins;
        a = temp_coin(idq, idc, A.k0, A.k1);
    } else {
        // P = cosh d / cosh R: e'_q m'_c + m'_q e'_c + s'_q s'_c sin^2(dtheta/2),
        // sin by its degree-11 Taylor polynomial (any angle up to pi)
        const float x = (float)(0.5 * short_angle(tq, tc));
        const float x2 = x * x;
        float p = -1.0f / 39916800.0f;
        p = fmaf(p, x2, 1.0f / 362880.0f);
        p = fmaf(p, x2, -1.0f / 5040.0f);
        p = fmaf(p, x2, 1.0f / 120.0f);
        p = fmaf(p, x2, -1.0f / 6.0f);
        p = fmaf(p, x2, 1.0f);
        const float s = x * p;
        float P = fmaf(fq.x, fc.y, fq.y * fc.x);
        P = fmaf(fq.z * fc.z, s * s, P);
        if (P > A.Ktr) return 0;  // d > rho: p(d) <= 2^-53 <= u
        if (MODE != T_EMIT) ++coins;
        a = temp_coin(idq, idc, A.k0, A.k1);
        const uint64_t b = (1ull << 53) - a;
        if (b == 0) return 0;
        // y = 2T log2(b/a) = x log2(e), the ratio formed first so that
        // coins near 1/2 keep their small logarithm accurate (a and b are
        // exact in binary64, so each float is rounded once; v_rcp_f32 is
        // within 1 ulp); D > 0  <=>  Dl = R log2(e) + y > 0
        const float af = (float)(double)a, bf = (float)(double)b;
        const float y = log2f(bf * __builtin_amdgcn_rcpf(af)) * A.twoTf;
        const float Dl = A.RL2E + y;
        if (Dl < -0x1p-10f) {
            v = 0;
        } else if (Dl > 0x1p-10f) {
            const float cr = (exp2f(y) + exp2f(-A.R2L2E - y)) * A.f1;  // cosh D / cosh R
            // the stage's error is below (36 + 3 |y|) 2^-24 relative (plus
            // 2^-34 absolute) where e^{-2D} <= 2^-16, below 2^-15 elsewhere
            const float rel = Dl >= 8.0f ? fmaf(fabsf(y), 0x1p-21f, 0x1p-17f) : 0x1p-12f;
            const float tol = rel * fmaxf(P, cr) + 0x1p-32f;
            v = P < cr - tol ? 1 : (P > cr + tol ? 0 : 2);
        }
        if (v != 2) return v;
    }
    if (EXACT) return temp_exact(A.sr[q], tq, A.sr[c], tc, a, A.R, A.twoT, A.stats, MODE != T_EMIT && A.use_p32);
    // a staged light row lists the pair itself, with its staging entry
    if (MODE == T_STAGE && chunk < 0) return 2;
    const uint64_t key = pair_key(q, c);
    if (MODE != T_EMIT) {
        const unsigned long long k = atomicAdd(&A.dcount[0], 1ull);
        if ((int64_t)k < A.dcap) {
            A.dkeys[k] = key;
            A.dchunk[k] = (int32_t)chunk;
        }
        return 0;
    }
    for (uint64_t h = slot_hash(key) & (uint64_t)A.hmask;; h = (h + 1) & (uint64_t)A.hmask) {
        const uint64_t z = A.hset[h];
        if (z == key) return 1;
        if (z == 0) return 0;
    }
}

// ------------------------------------------------------------ windows

// Conservative half-width of band j's window of radius rho for a query with
// record (eq, mq, sq); >= 3 means the whole band.  A point at radius r and
// angle difference dtheta is within rho iff sin^2(dtheta/2) <= X(r) =
// (cosh rho - cosh(r_q - r)) / (2 sinh r_q sinh r) = (K - N) / (s'_q s'(r)),
// N = cosh(r_q - r) / cosh R, and X decreases in r (rho >= r_q), so the
// band's inner edge gives a window for the whole band.  N carries at most
// 4 u relative error and K is rounded up, so with K - N >= K/64 (else the
// whole band) the computed X is within about 330 u of the exact one; the
// factor 1 + 2^-12 and the 2^-40 absolute pad keep the window conservative,
// as in the threshold search.
__device__ __forceinline__ double temp_window(const TempArgs &A, float eq, float mq, float sq, int j)
{
    const float shl = A.sh_lo[j];
    if (A.E[j] < 0.25 || shl == 0.0f || sq == 0.0f) return 4.0;
    const float num = A.K - fmaf(eq, A.em_lo[j], mq * A.ep_lo[j]);
    if (!(num >= 0x1p-6f * A.K)) return 4.0;  // also catches NaN
    const float X = num / (sq * shl);
    if (!(X < 0.25f)) {
        if (!(X < 0.999f)) return 4.0;
        return 2.0 * asin(sqrt((double)X * (1.0 + 0x1p-12))) * (1.0 + 0x1p-12) + 0x1p-40;
    }
    const float Xp = fmaxf(X, 0.0f);
    return (double)(2.0f * sqrtf(Xp) * fmaf(Xp, 0.2f, 1.0f)) * (1.0 + 0x1p-12) + 0x1p-40;
}

// Position runs [a0, b0), [a1, b1) of band j that hold query q's window.
struct TRuns {
    int64_t a0, b0, a1, b1;
};

__device__ __forceinline__ TRuns temp_runs(const TempArgs &A, double tq, float4 fq, int j)
{
    TRuns t;
    t.a0 = t.b0 = t.a1 = t.b1 = 0;
    const int64_t s = A.band_start[j], e = A.band_start[j + 1];
    if (s == e) return t;
    const double w = temp_window(A, fq.x, fq.y, fq.z, j);
    int64_t ra[2], rb[2];
    int nr;
    if (w >= 3.0) {
        ra[0] = s; rb[0] = e; nr = 1;
    } else {
        nr = cell_runs(A.dir + A.dir_base[j], A.cbits[j], tq - w, tq + w, s, e, ra, rb);
    }
    t.a0 = ra[0]; t.b0 = rb[0];
    if (nr == 2) { t.a1 = ra[1]; t.b1 = rb[1]; }
    return t;
}

__device__ __forceinline__ int64_t tuni64(int64_t v)
{
    const int lo = __builtin_amdgcn_readfirstlane((int)(uint32_t)(uint64_t)v);
    const int hi = __builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// ------------------------------------------------------------ heavy plan

// Before the count pass: heavy_end = the first light position (the end of
// the heavy bands, capped); row_ptr[0] = 0; the candidate total cleared.
__global__ void temp_prologue(TempArgs A, int jh, int32_t *heavy_end, int64_t *row_ptr)
{
    if (threadIdx.x == 0) {
        int64_t h = jh > 0 ? (int64_t)A.band_start[jh] : 0;
        if (h > A.heavy_cap) h = A.heavy_cap;
        *heavy_end = (int32_t)h;
        row_ptr[0] = 0;
        A.hscal[0] = 0;
        A.stats[ST_TEMP_CAND] = 0;
        A.stats[ST_TEMP_COINS] = 0;
        A.dcount[0] = 0;
        A.dcount[1] = 0;
    }
}

// Count pass: a wavefront's tallies of screened candidates and coins, added
// to slot `slot` of the per-wavefront table (one device-wide atomic counter
// for every wavefront would serialise them), summed by temp_tally_sum.
__device__ __forceinline__ void temp_tally(const TempArgs &A, long long cand, long long coins, int64_t slot)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        cand += __shfl_xor(cand, o, 64);
        coins += __shfl_xor(coins, o, 64);
    }
    if ((threadIdx.x & 63) == 0 && (cand | coins)) {
        atomicAdd((unsigned long long *)&A.tal[slot].x, (unsigned long long)cand);
        atomicAdd((unsigned long long *)&A.tal[slot].y, (unsigned long long)coins);
    }
}

// After the count pass: the table's sums into the index's diagnostics.
__global__ void __launch_bounds__(256) temp_tally_sum(TempArgs A, int64_t slots)
{
    __shared__ long long part[2][4];
    long long c = 0, k = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < slots; i += (int64_t)gridDim.x * 256) {
        c += A.tal[i].x;
        k += A.tal[i].y;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        c += __shfl_xor(c, o, 64);
        k += __shfl_xor(k, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        part[0][threadIdx.x >> 6] = c;
        part[1][threadIdx.x >> 6] = k;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        c = part[0][0] + part[0][1] + part[0][2] + part[0][3];
        k = part[1][0] + part[1][1] + part[1][2] + part[1][3];
        if (c) atomicAdd(&A.stats[ST_TEMP_CAND], (unsigned long long)c);
        if (k) atomicAdd(&A.stats[ST_TEMP_COINS], (unsigned long long)k);
    }
}

// Candidates of every heavy item (query, band); 0 past the heavy queries.
__global__ void __launch_bounds__(256) temp_plan_len(TempArgs A)
{
    __shared__ long long part[4];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    long long len = 0;
    if (i < A.heavy_cap * A.B) {
        const int64_t q = i / A.B;
        const int j = (int)(i % A.B);
        if (q < *A.heavy_end) {
            const TRuns t = temp_runs(A, A.st[q], A.rec[q], j);
            len = (t.b0 - t.a0) + (t.b1 - t.a1);
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

// Chunks per item, with the chunk size CH chosen so the table cannot
// overflow (each item adds at most one partial chunk).
__global__ void __launch_bounds__(256) temp_plan_chunks(TempArgs A)
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

// Chunk -> item table: after the scan, item i owns chunks [hplan[i-1], hplan[i]).
__global__ void __launch_bounds__(256) temp_chunk_items(TempArgs A)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= A.heavy_cap * A.B) return;
    const int64_t b = i ? A.hplan[i - 1] : 0, e = A.hplan[i];
    for (int64_t c = b; c < e; ++c) A.hitem[c] = (int32_t)i;
}

__global__ void __launch_bounds__(256) temp_zero(int64_t *p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = 0;
}

// After the count pass and the scan of the chunk counts: heavy degrees.
__global__ void __launch_bounds__(256) temp_heavy_degrees(TempArgs A, int64_t *__restrict__ row_ptr)
{
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= *A.heavy_end) return;
    const int64_t f = q ? A.hplan[q * A.B - 1] : 0;   // first chunk of q
    const int64_t l = A.hplan[q * A.B + A.B - 1];     // one past its last chunk
    const int64_t hi = l ? A.hcnt[l - 1] : 0, lo = f ? A.hcnt[f - 1] : 0;
    row_ptr[__float_as_int(A.rec[q].w) + 1] = hi - lo;
}

// ------------------------------------------------------------ heavy chunks

// One chunk of a heavy item: a workgroup decides its candidates 256 at a
// time; the emit pass places them by the prefix of the count pass's chunk
// counts (row order: band, chunk, candidate).
template <int MODE, bool EXACT>
__device__ void temp_chunk(const TempArgs &A, int64_t c, const int64_t *row_ptr, int32_t *col)
{
    constexpr bool EMIT = MODE == T_EMIT;
    __shared__ int wave_cnt[2][4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t item = tuni64(A.hitem[c]);
    const int64_t first = item ? tuni64(A.hplan[item - 1]) : 0;
    const int64_t q = item / A.B;
    const int j = (int)(item % A.B);
    const int64_t ch = tuni64(A.hscal[1]);
    const double tq = A.st[q];
    const float4 fq = A.rec[q];
    const TRuns t = temp_runs(A, tq, fq, j);
    const int64_t a0 = tuni64(t.a0), b0 = tuni64(t.b0), a1 = tuni64(t.a1), b1 = tuni64(t.b1);
    const int64_t len0 = b0 - a0, len = len0 + (b1 - a1);
    const int64_t v0 = (c - first) * ch, v1 = min(len, v0 + ch);
    const int32_t id = __float_as_int(fq.w);
    int64_t out = 0, row_end = 0;
    if (EMIT) {
        const int64_t qfirst = q ? tuni64(A.hplan[q * A.B - 1]) : 0;
        const int64_t base_c = c ? tuni64(A.hcnt[c - 1]) : 0;
        const int64_t base_q = qfirst ? tuni64(A.hcnt[qfirst - 1]) : 0;
        out = row_ptr[id] + (base_c - base_q);
        row_end = row_ptr[id + 1];
        if (A.col_cap >= 0 && row_end > A.col_cap) row_end = A.col_cap;
    }
    int64_t total = 0;
    int cand = 0, coins = 0;
    for (int64_t vb = v0; vb < v1; vb += 256) {
        const int64_t v = vb + threadIdx.x;
        int acc = 0;
        int32_t cid = 0;
        if (v < v1) {
            const int64_t pos = (v < len0) ? a0 + v : a1 + (v - len0);
            const float4 fc = A.rec[pos];
            cid = __float_as_int(fc.w);
            if (pos != q) {
                ++cand;
                acc = temp_decide<MODE, EXACT>(A, q, tq, fq, pos, A.st[pos], fc, coins, c);
            }
        }
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
    __syncthreads();
    if (!EMIT && A.tally) temp_tally(A, cand, coins, c % A.tal_slots);
    if (!EMIT && threadIdx.x == 0) A.hcnt[c] = total;
    if (EMIT && threadIdx.x == 0 && total != A.hcnt[c] - (c ? A.hcnt[c - 1] : 0))
        atomicAdd(&A.stats[ST_EMIT_MISMATCH], 1ull);
}

// ------------------------------------------------------------ light queries

// One lane per query: every band's window, candidate by candidate.  The
// count pass writes the degree to row_ptr[id + 1] (staged: with the slot's
// start / 4 + 1 above it, and the row into the slot); the emit pass writes
// the row and checks its length.  Every lane of a wavefront of 64
// consecutive positions calls it together.
template <int MODE, bool EXACT>
__device__ void temp_light(const TempArgs &A, int64_t q, int64_t *row_ptr, int32_t *col)
{
    constexpr bool EMIT = MODE == T_EMIT;
    constexpr bool STAGE = MODE == T_STAGE;
    const bool active = q < A.n && q >= *A.heavy_end;
    double tq = 0.0;
    float4 fq = make_float4(0.f, 0.f, 0.f, 0.f);
    if (active) {
        tq = A.st[q];
        fq = A.rec[q];
    }
    const int32_t id = __float_as_int(fq.w);
    int64_t out = 0, row_end = 0;
    if (EMIT && active) {
        out = row_ptr[id];
        row_end = row_ptr[id + 1];
    }
    const int64_t row_start = out;
    const int64_t cap_end = (EMIT && A.col_cap >= 0) ? A.col_cap : INT64_MAX;
    // STAGE: the slot after the wavefront's earlier lanes' slots; word 0
    // holds the row's length, entry k goes to word 1 + k while k < lim
    int64_t sb = 0, lim = 0, pend = 0;
    // (a wavefront past the last point has no slots, and no prefix entry)
    if (STAGE && __ballot(active) != 0) {
        int quads = 0;
        if (active)
            quads = stage_slot_quads(A.E, A.lmu_in, A.lmu_out, A.stage_f,
                                     A.band_bits ? (int)(A.keys[q] >> (32 - A.band_bits)) : 0, A.sr[q]);
        int wt;
        const int64_t wv = q >> 6;
        sb = (wv ? A.wsum[wv - 1] : 0) + 4 * (int64_t)wave_excl_sum(quads, (int)(threadIdx.x & 63), &wt);
        lim = active ? max<int64_t>(0, min<int64_t>(4 * (int64_t)quads - 1, A.stage_cap - sb - 1)) : 0;
    }
    int64_t cnt = 0;
    int cand = 0, coins = 0;
    for (int j = 0; j < A.B; ++j) {
        TRuns t;
        t.a0 = t.b0 = t.a1 = t.b1 = 0;
        if (active) t = temp_runs(A, tq, fq, j);
        for (int r = 0; r < 2; ++r) {
            const int64_t a = r ? t.a1 : t.a0, b = r ? t.b1 : t.b0;
            // each candidate's record is loaded one step ahead
            float4 fn = make_float4(0.f, 0.f, 0.f, 0.f);
            double tn = 0.0;
            if (a < b) {
                fn = A.rec[a];
                tn = A.st[a];
            }
            for (int64_t c = a; c < b; ++c) {
                const float4 fc = fn;
                const double tc = tn;
                if (c + 1 < b) {
                    fn = A.rec[c + 1];
                    tn = A.st[c + 1];
                }
                if (c == q) continue;
                ++cand;
                const int v = temp_decide<MODE, EXACT>(A, q, tq, fq, c, tc, fc, coins, -1);
                if (!v) continue;
                if (STAGE) {
                    if (v == 2) {
                        const unsigned long long k = atomicAdd(&A.dcount[0], 1ull);
                        if ((int64_t)k < A.dcap) {
                            A.dkeys[k] = pair_key(q, c);
                            A.dchunk[k] = -1;
                            A.dslot[k] = cnt < lim ? sb + 1 + cnt : -1;
                        }
                        ++pend;
                    }
                    if (cnt < lim) A.stage[sb + 1 + cnt] = __float_as_int(fc.w) | (v == 2 ? (int)STAGE_PENDING : 0);
                }
                if (EMIT) {
                    const int64_t o = row_start + cnt;
                    if (o < row_end && o < cap_end) col[o] = __float_as_int(fc.w);
                }
                ++cnt;
            }
        }
    }
    if (!EMIT && A.tally) temp_tally(A, cand, coins, (q >> 6) % A.tal_slots);
    // a row that outgrew its slot: the emit pass searches this wavefront again
    const bool wovf = STAGE && __ballot(active && cnt > lim) != 0;
    if (wovf && (threadIdx.x & 63) == 0) A.sovf[q >> 6] = 1;
    if (!active) return;
    if (STAGE) {
        const uint64_t hs = sb < A.stage_cap ? (uint64_t)(sb >> 2) + 1 : 0xffffffffull;
        row_ptr[id + 1] = (int64_t)((hs << 32) | (uint64_t)(cnt - pend));
        if (sb < A.stage_cap) A.stage[sb] = wovf ? -1 : (int32_t)cnt;
    } else if (!EMIT) {
        row_ptr[id + 1] = cnt;
    } else if (cnt != row_end - row_start) {
        atomicAdd(&A.stats[ST_EMIT_MISMATCH], 1ull);
    }
}

// Heavy chunks on the first heavy_blocks workgroups, light queries (256 a
// workgroup) striding over the rest.  With `gate` the kernel runs only if
// the count pass's undecided-pair list overflowed (EXACT) or did not
// (fast).  The fast kernels are held to 96 registers (five wavefronts per
// SIMD: the staged count then takes 524 instead of 554 ms at n = 1e8,
// T = 0.1, with 6 registers spilled); the EXACT kernels, which call the
// exact test, keep their own budget.
template <int MODE, bool EXACT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(EXACT ? 1 : 5)))
temp_kernel(TempArgs A, int64_t *__restrict__ row_ptr, int32_t *__restrict__ col_idx, int gate)
{
    // emit pass into a buffer too small for the graph: write nothing
    if (MODE == T_EMIT && A.col_cap >= 0 && tuni64(row_ptr[A.n]) > A.col_cap) return;
    if (gate && (__builtin_amdgcn_readfirstlane((int)A.dcount[1]) != 0) != EXACT) return;
    if ((int)blockIdx.x < A.heavy_blocks) {
        const int64_t nch = tuni64(A.hplan[A.heavy_cap * A.B - 1]);
        for (int64_t c = blockIdx.x; c < nch; c += A.heavy_blocks) temp_chunk<MODE, EXACT>(A, c, row_ptr, col_idx);
        return;
    }
    // emit pass after a staged count: the light rows are copied (and the
    // wavefronts whose rows outgrew their slots searched again) by the
    // kernels below
    if (A.light_skip) return;
    const int64_t lb = (A.n + 255) / 256, nb = (int64_t)gridDim.x - A.heavy_blocks;
    for (int64_t b = (int64_t)blockIdx.x - A.heavy_blocks; b < lb; b += nb)
        temp_light<MODE, EXACT>(A, b * 256 + threadIdx.x, row_ptr, col_idx);
}

// Emit pass after a staged count: the wavefronts whose rows outgrew their
// slots, searched again.  Each wavefront reads 64 flags at a time.
template <bool EXACT>
__global__ void __launch_bounds__(256) temp_redo_kernel(TempArgs A, int64_t *__restrict__ row_ptr,
                                                        int32_t *__restrict__ col, int gate)
{
    if (A.col_cap >= 0 && tuni64(row_ptr[A.n]) > A.col_cap) return;
    if (gate && (__builtin_amdgcn_readfirstlane((int)A.dcount[1]) != 0) != EXACT) return;
    const int lane = threadIdx.x & 63;
    const int64_t waves = (A.n + 63) / 64;
    for (int64_t g0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 64; g0 < waves; g0 += (int64_t)gridDim.x * 256) {
        const int64_t w = g0 + lane;
        for (uint64_t m = __ballot(w < waves && A.sovf[w]); m; m &= m - 1)
            temp_light<T_EMIT, EXACT>(A, (g0 + __ffsll((unsigned long long)m) - 1) * 64 + lane, row_ptr, col);
    }
}

// After the fast count pass: decide the listed pairs exactly, count the
// edges among them (the light query's degree, or the heavy chunk's count)
// and enter them in the set the emit pass reads.  Flags an overflowed list.
__global__ void __launch_bounds__(256) temp_resolve(TempArgs A, int64_t *__restrict__ row_ptr)
{
    const unsigned long long cnt = A.dcount[0];
    if (blockIdx.x == 0 && threadIdx.x == 0 && (int64_t)cnt > A.dcap) A.dcount[1] = 1;
    if ((int64_t)cnt > A.dcap) return;
    const int64_t m = (int64_t)cnt, stride = (int64_t)gridDim.x * 256;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < m; i += stride) {
        const uint64_t key = A.dkeys[i];
        const int64_t q = (int64_t)((key >> 32) & 0x7fffffffull), c = (int64_t)(key & 0xffffffffull);
        const float4 fq = A.rec[q], fc = A.rec[c];
        const uint64_t a = temp_coin((uint32_t)__float_as_int(fq.w), (uint32_t)__float_as_int(fc.w), A.k0, A.k1);
        const int edge = temp_exact(A.sr[q], A.st[q], A.sr[c], A.st[c], a, A.R, A.twoT, A.stats, 1);
        const int32_t ch = A.dchunk[i];
        if (A.staged && ch < 0) {  // the staged row's pending entry, decided
            const int64_t slot = A.dslot[i];
            if (slot >= 0) A.stage[slot] = edge ? __float_as_int(fc.w) : STAGE_REJECT;
        }
        if (!edge) continue;
        for (uint64_t h = slot_hash(key) & (uint64_t)A.hmask;; h = (h + 1) & (uint64_t)A.hmask) {
            const unsigned long long prev = atomicCAS((unsigned long long *)&A.hset[h], 0ull, (unsigned long long)key);
            if (prev == 0ull || prev == key) break;
        }
        if (ch >= 0) atomicAdd((unsigned long long *)&A.hcnt[ch], 1ull);
        else atomicAdd((unsigned long long *)&row_ptr[__float_as_int(fq.w) + 1], 1ull);
    }
}

hipError_t launch_temp_search(rhg_index *idx, double T, int64_t *row_ptr, int32_t *col_idx, int emit,
                              hipStream_t s, int64_t col_cap)
{
    const Layout &L = idx->L;
    const rhg_params &p = idx->p;
    TempArgs A;
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
    A.max_chunks = idx->max_chunks;
    A.heavy_blocks = idx->heavy_cap > 0 ? RHG_HEAVY_BLOCKS : 0;
    A.R = p.R;
    A.twoT = 2.0 * T;
    // rho = R + 2T ln(2^53 - 1); K = cosh(rho) / cosh(R) rounded up, with
    // 2^-20 relative to spare for the binary64 evaluation
    const double rho = p.R + 2.0 * T * log(9007199254740991.0);
    const double K = cosh(rho) / cosh(p.R) * (1.0 + 0x1p-20);
    A.K = nextafterf((float)K, INFINITY);
    A.Ktr = nextafterf((float)(K * (1.0 + 0x1p-16)), INFINITY);
    A.twoTf = (float)(2.0 * T);
    A.RL2E = (float)(p.R * 1.4426950408889634);
    A.R2L2E = (float)(2.0 * p.R * 1.4426950408889634);
    A.f1 = (float)(1.0 / (1.0 + exp(-2.0 * p.R)));
    A.use_p32 = (!L.fp64_only && p.R < 80.0) ? 1 : 0;
    A.k0 = (uint32_t)p.seed;
    A.k1 = (uint32_t)(p.seed >> 32);
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
    A.dkeys = idx->dkeys;
    A.dchunk = idx->dchunk;
    A.dcount = idx->dcount;
    A.dcap = L.defer_cap;
    A.hset = idx->hset;
    A.hmask = idx->hset_slots - 1;
    A.col_cap = col_cap;
    A.tally = 1;
    A.tal = (longlong2 *)idx->wstat;
    A.tal_slots = std::max<int64_t>((idx->n + 63) / 64, 1);
    for (int j = 0; j < L.B; ++j) {
        A.lmu_in[j] = L.lmu_in[j];
        A.lmu_out[j] = L.lmu_out[j];
    }
    // the slots are the threshold search's scaled by pi T' / sin(pi T'),
    // T' = min(2T, 0.45): the temperature model's degree exceeds the
    // threshold model's by about pi T / sin(pi T) where the pairs' count
    // grows as e^{d/2}, and by more near the hubs
    const double Tp = std::min(2.0 * T, 0.45);
    const float tscale = (float)(M_PI * Tp / sin(M_PI * Tp));
    A.stage_f = L.stage_f * tscale;
    A.band_bits = L.band_bits;
    A.keys = idx->keys;
    A.stage = idx->stage;
    A.stage_cap = L.stage_cap;
    A.wsum = idx->wsum;
    A.sovf = idx->sovf;
    A.dslot = idx->dslot;
    // staged: the count pass writes the light rows into their slots, the
    // emit pass searches the heavy chunks again, copies the light rows and
    // searches again the wavefronts whose rows outgrew their slots
    const bool staged = emit ? idx->staged_count != 0 : L.staged != 0;
    A.staged = staged ? 1 : 0;
    A.light_skip = (emit && staged) ? 1 : 0;
    const int64_t n = idx->n;
    const int64_t items = idx->heavy_cap * L.B;
    hipError_t e;
    if (!emit) {
        PhaseScope ps(RHG_PHASE_PLAN, s);
        hipLaunchKernelGGL(temp_prologue, dim3(1), dim3(64), 0, s, A, L.heavy_band, idx->heavy_end, row_ptr);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (n <= 0) return hipSuccess;
        if (staged && (e = launch_stage_slots(idx, tscale, s)) != hipSuccess) return e;
        if (items > 0) {
            const unsigned g = (unsigned)((items + 255) / 256);
            hipLaunchKernelGGL(temp_plan_len, dim3(g), dim3(256), 0, s, A);
            hipLaunchKernelGGL(temp_plan_chunks, dim3(g), dim3(256), 0, s, A);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            if ((e = inclusive_scan_i64(idx->hplan, items, idx->tmp, s)) != hipSuccess) return e;
            hipLaunchKernelGGL(temp_chunk_items, dim3(g), dim3(256), 0, s, A);
            hipLaunchKernelGGL(temp_zero, dim3((unsigned)((idx->max_chunks + 255) / 256)), dim3(256), 0, s,
                               idx->hcnt, idx->max_chunks);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
    } else if (n <= 0) {
        return hipSuccess;
    }
    const dim3 g((unsigned)(A.heavy_blocks + (n + 255) / 256)), b(256);
    // the EXACT kernels, when they only stand by for an overflowed list, run
    // on a smaller grid (a smaller heavy pool; the light part strides)
    TempArgs Ax = A;
    Ax.heavy_blocks = std::min(A.heavy_blocks, 64);
    Ax.tally = 0;
    const dim3 gx((unsigned)(Ax.heavy_blocks + std::min<int64_t>((n + 255) / 256, 64)));
    // with no FP32 stage (or on request) every pair is decided in place
    const bool exact_only = !A.use_p32 || L.exact_inline;
    if (!emit && !exact_only)
        hipLaunchKernelGGL(temp_zero, dim3((unsigned)((A.hmask + 256) / 256)), dim3(256), 0, s, (int64_t *)A.hset,
                           A.hmask + 1);
    if (!emit)
        hipLaunchKernelGGL(temp_zero, dim3((unsigned)((2 * A.tal_slots + 255) / 256)), dim3(256), 0, s,
                           (int64_t *)A.tal, 2 * A.tal_slots);
    const dim3 gh((unsigned)std::max(A.heavy_blocks, 1)), ghx((unsigned)std::max(Ax.heavy_blocks, 1));
    const dim3 gr((unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 63) / 64 / 256 + 1, 4096)));
    {
        PhaseScope ps(emit ? RHG_PHASE_EMIT_PASS : RHG_PHASE_COUNT_PASS, s);
        if (emit && staged) {
            if (A.heavy_blocks > 0) {
                if (exact_only) hipLaunchKernelGGL((temp_kernel<T_EMIT, true>), gh, b, 0, s, A, row_ptr, col_idx, 0);
                else hipLaunchKernelGGL((temp_kernel<T_EMIT, false>), gh, b, 0, s, A, row_ptr, col_idx, 1);
            }
            if ((e = hipGetLastError()) != hipSuccess) return e;
            if ((e = launch_stage_copy(idx, row_ptr, col_idx, col_cap, s)) != hipSuccess) return e;
            if (exact_only) hipLaunchKernelGGL(temp_redo_kernel<true>, gr, b, 0, s, A, row_ptr, col_idx, 0);
            else hipLaunchKernelGGL(temp_redo_kernel<false>, gr, b, 0, s, A, row_ptr, col_idx, 1);
        } else if (exact_only) {
            if (emit) hipLaunchKernelGGL((temp_kernel<T_EMIT, true>), g, b, 0, s, A, row_ptr, col_idx, 0);
            else if (staged) hipLaunchKernelGGL((temp_kernel<T_STAGE, true>), g, b, 0, s, A, row_ptr, col_idx, 0);
            else hipLaunchKernelGGL((temp_kernel<T_COUNT, true>), g, b, 0, s, A, row_ptr, col_idx, 0);
        } else if (emit) {
            hipLaunchKernelGGL((temp_kernel<T_EMIT, false>), g, b, 0, s, A, row_ptr, col_idx, 1);
        } else if (staged) {
            hipLaunchKernelGGL((temp_kernel<T_STAGE, false>), g, b, 0, s, A, row_ptr, col_idx, 1);
        } else {
            hipLaunchKernelGGL((temp_kernel<T_COUNT, false>), g, b, 0, s, A, row_ptr, col_idx, 1);
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (!exact_only) {
        PhaseScope ps(RHG_PHASE_PLAN, s);
        if (!emit) {
            hipLaunchKernelGGL(temp_resolve, dim3(256), dim3(256), 0, s, A, row_ptr);
            if (staged) hipLaunchKernelGGL((temp_kernel<T_STAGE, true>), gx, b, 0, s, Ax, row_ptr, col_idx, 1);
            else hipLaunchKernelGGL((temp_kernel<T_COUNT, true>), gx, b, 0, s, Ax, row_ptr, col_idx, 1);
        } else if (staged) {
            if (A.heavy_blocks > 0)
                hipLaunchKernelGGL((temp_kernel<T_EMIT, true>), ghx, b, 0, s, Ax, row_ptr, col_idx, 1);
            hipLaunchKernelGGL(temp_redo_kernel<true>, dim3(std::min(gr.x, 64u)), b, 0, s, Ax, row_ptr, col_idx, 1);
        } else {
            hipLaunchKernelGGL((temp_kernel<T_EMIT, true>), gx, b, 0, s, Ax, row_ptr, col_idx, 1);
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (!emit) idx->staged_count = staged ? 1 : 0;
    if (!emit) {
        hipLaunchKernelGGL(temp_tally_sum, dim3(256), dim3(256), 0, s, A, A.tal_slots);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (!emit && items > 0) {
        PhaseScope ps(RHG_PHASE_PLAN, s);
        if ((e = inclusive_scan_i64(idx->hcnt, idx->max_chunks, idx->tmp, s)) != hipSuccess) return e;
        hipLaunchKernelGGL(temp_heavy_degrees, dim3((unsigned)((idx->heavy_cap + 255) / 256)), dim3(256), 0, s, A,
                           row_ptr);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (!emit && staged) e = launch_stage_split(idx, row_ptr, s);
    return e;
}

}  // namespace rhg
