/*
 * rhg_oracle.c -- plain, slow CPU oracle for random hyperbolic graph (RHG)
 * generation (von Looz, Meyerhenke, Prutkin, Staudt: "Fast generation of
 * complex networks with underlying hyperbolic geometry").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant with
 * the GPU library.
 *
 * What it computes, step by step, in the paper's order:
 *   1. alpha from the power-law exponent: gamma = 2*alpha + 1 with the
 *      curvature fixed to 1 (Sec. 2.1).
 *   2. R from the expected average degree of Krioukov et al.'s Eq. (22) as
 *      restated in Appendix B.1 ("getTargetRadius"), solved by bisection on
 *      its decreasing branch (Appendix B.1; Algorithm 1, first step).
 *   3. n points: angle uniform on [0, 2*pi) (Algorithm 1, angular draw) and
 *      radius with density alpha*sinh(alpha r)/(cosh(alpha R)-1) (Eq. (1)),
 *      drawn by inverting the cell-probability CDF of Appendix C.
 *   4. Edges: every pair {i, j}, i != j, whose hyperbolic distance is at most
 *      R (Sec. 2.1; Proposition 2 says Algorithm 1 produces exactly this set).
 *      Brute force over all pairs: no spatial index, no pruning.
 *
 * Precision.  Step 4 is decided exactly on the given binary64 coordinates:
 * the distance test is evaluated in binary64 from a well-conditioned form,
 * and any pair whose value lies within a relative 1e-9 of the threshold is
 * re-evaluated in binary128 (libquadmath).  Pairs that even binary128 cannot
 * separate from the threshold (relative 1e-30) are counted as ties.
 * Steps 2 and 3 are evaluated in binary128 and rounded once to binary64, so
 * R is the unique double defined in orc_solve_R and each radius is the
 * correctly rounded inverse CDF (a near-midpoint counter reports the
 * astronomically rare cases binary128 cannot settle).
 *
 * Random numbers (the paper does not fix a generator): Philox4x32-10,
 * implemented from its published definition (Salmon, Moraes, Dror, Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3", SC'11).  Vertex i uses
 * counter (i_lo, i_hi, 0, 0) and key (seed_lo, seed_hi).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <quadmath.h>
#include <omp.h>

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al., SC'11): 10 rounds of the 4x32 S-box    */
/* with Weyl-sequence key schedule.                                      */
/* ------------------------------------------------------------------ */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += PHILOX_W0; k1 += PHILOX_W1; }
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* The two 53-bit uniforms of vertex i: u_theta from words (x1:x0),
 * u_r from words (x3:x2), each the top 53 bits scaled by 2^-53. */
void orc_uniforms(uint64_t seed, int64_t i, double *u_theta, double *u_r)
{
    uint32_t ctr[4] = { (uint32_t)(uint64_t)i, (uint32_t)((uint64_t)i >> 32), 0u, 0u };
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    uint32_t x[4];
    orc_philox4x32_10(ctr, key, x);
    uint64_t a = ((uint64_t)x[1] << 32) | x[0];
    uint64_t b = ((uint64_t)x[3] << 32) | x[2];
    *u_theta = (double)(a >> 11) * 0x1p-53;
    *u_r     = (double)(b >> 11) * 0x1p-53;
}

/* ------------------------------------------------------------------ */
/* Step 1 and 2: alpha and R.                                           */
/* ------------------------------------------------------------------ */

/* alpha = (gamma - 1) / 2, evaluated as two binary64 operations. */
double orc_alpha(double gamma) { return (gamma - 1.0) * 0.5; }

/* Expected average degree, Eq. (22) of Krioukov et al. as printed in
 * Appendix B.1, with zeta = 1 and xi = alpha / (alpha - 1/2):
 *   kbar = (2/pi) xi^2 n ( e^{-R/2}
 *          + e^{-alpha R} ( alpha (R/2) ( (pi/4)(1/alpha)^2
 *                                         - (pi-1)(1/alpha) + (pi-2) ) - 1 ) )
 * The printed middle term reads "(pi-1) xi/alpha"; with that literal reading
 * no positive R reaches any practical target degree, so the zeta/alpha
 * reading (zeta = 1) is used.  literal != 0 selects the printed xi/alpha
 * term, kept only so a test can show it has no root. */
static __float128 kbar_q(double n, double alpha, double R, int literal)
{
    const __float128 pi = M_PIq;
    __float128 a = alpha, r = R, nn = n;
    __float128 xi = a / (a - 0.5Q);
    __float128 mid = literal ? xi / a : 1.0Q / a;
    __float128 inner = (pi / 4.0Q) * (1.0Q / a) * (1.0Q / a) - (pi - 1.0Q) * mid + (pi - 2.0Q);
    __float128 t = expq(-r / 2.0Q) + expq(-a * r) * (a * (r / 2.0Q) * inner - 1.0Q);
    return (2.0Q / pi) * xi * xi * nn * t;
}

double orc_kbar_eq22(double n, double alpha, double R, int literal)
{
    return (double)kbar_q(n, alpha, R, literal);
}

/* Eq. (22) minus a target, formed in binary128 before rounding, so that its
 * sign is the binary128 comparison used by orc_solve_R. */
double orc_kbar_minus(double n, double alpha, double R, double target)
{
    return (double)(kbar_q(n, alpha, R, 0) - (__float128)target);
}

/* R is defined as the smallest binary64 value on the decreasing branch of
 * Eq. (22) whose expected degree is at most the target.  The bracket is
 * [R_peak, 2 ln n + 40]; R_peak is located by golden-section search for the
 * maximum of Eq. (22).  The result does not depend on the bracket, only on
 * Eq. (22) decreasing across it.  Returns 0 on success, 1 when gamma <= 2 or
 * the target is not reachable (it exceeds the peak of Eq. (22)). */
int orc_solve_R(double n, double kbar, double gamma, double *alpha_out, double *R_out)
{
    if (!(gamma > 2.0) || !(kbar > 0.0) || !(n >= 2.0)) return 1;
    double alpha = orc_alpha(gamma);
    double hi = 2.0 * log(n) + 40.0;
    /* golden-section search for the maximum of Eq. (22) on (0, hi] */
    double a = 1e-6, b = hi;
    const double g = 0.6180339887498949;
    for (int it = 0; it < 200; ++it) {
        double c = b - g * (b - a), d = a + g * (b - a);
        if (kbar_q(n, alpha, c, 0) > kbar_q(n, alpha, d, 0)) b = d; else a = c;
    }
    double lo = 0.5 * (a + b);
    __float128 target = kbar;
    if (!(kbar_q(n, alpha, lo, 0) > target)) return 1;
    if (!(kbar_q(n, alpha, hi, 0) <= target)) return 1;
    /* bisection over binary64 values down to adjacent doubles */
    for (;;) {
        double mid = lo + 0.5 * (hi - lo);
        if (mid <= lo || mid >= hi) break;
        if (kbar_q(n, alpha, mid, 0) <= target) hi = mid; else lo = mid;
    }
    *alpha_out = alpha;
    *R_out = hi;
    return 0;
}

/* cosh(R) rounded once from binary128. */
double orc_cosh(double x) { return (double)coshq((__float128)x); }

/* ------------------------------------------------------------------ */
/* Step 3: points.                                                      */
/* ------------------------------------------------------------------ */
static const double TWO_PI_D = 6.283185307179586;   /* 2*pi rounded to binary64 */

/* Correctly rounded radius for the uniform u: the r with
 * F(r) = (cosh(alpha r) - 1)/(cosh(alpha R) - 1) = u (Appendix C, cell
 * probability with the whole disk's angle range), i.e.
 * r = acosh(1 + u (cosh(alpha R) - 1)) / alpha, evaluated in binary128 as
 * log1p(x + sqrt(x (x + 2))) / alpha with x = u (cosh(alpha R) - 1).
 * *hard is set when the binary128 value is too close to a rounding midpoint
 * for the rounding to be certain. */
static double radius_q(double u, double alpha, double R, int *hard)
{
    __float128 c = coshq((__float128)alpha * (__float128)R) - 1.0Q;
    __float128 x = (__float128)u * c;
    __float128 rq = log1pq(x + sqrtq(x * (x + 2.0Q))) / (__float128)alpha;
    double rd = (double)rq;
    *hard = 0;
    if (rd != 0.0) {
        double up = nextafter(rd, INFINITY), dn = nextafter(rd, 0.0);
        __float128 mid_up = ((__float128)rd + (__float128)up) * 0.5Q;
        __float128 mid_dn = ((__float128)rd + (__float128)dn) * 0.5Q;
        __float128 tol = fabsq(rq) * 0x1p-100Q;
        if (fabsq(rq - mid_up) < tol || fabsq(rq - mid_dn) < tol) *hard = 1;
    }
    return rd;
}

/* The radius for one uniform u (exposed for tests of the rounding). */
double orc_radius(double u, double alpha, double R, int *hard)
{
    return radius_q(u, alpha, R, hard);
}

/* Sample points [i0, i0 + count) of graph (seed, alpha, R).  theta is the
 * single binary64 product TWO_PI_D * u_theta, which lies in [0, 2*pi).
 * Returns the number of near-midpoint radii. */
int64_t orc_sample(uint64_t seed, double alpha, double R, int64_t i0, int64_t count,
                   double *r, double *theta, int nthreads)
{
    int64_t hard_total = 0;
    if (nthreads > 0) omp_set_num_threads(nthreads);
    #pragma omp parallel for schedule(static) reduction(+:hard_total)
    for (int64_t k = 0; k < count; ++k) {
        double ut, ur;
        orc_uniforms(seed, i0 + k, &ut, &ur);
        int hard;
        theta[k] = TWO_PI_D * ut;
        r[k] = radius_q(ur, alpha, R, &hard);
        hard_total += hard;
    }
    return hard_total;
}

/* ------------------------------------------------------------------ */
/* Step 4: the edge relation.                                           */
/* ------------------------------------------------------------------ */
/* 2*pi - TWO_PI_D, to well beyond binary128 precision. */
static const __float128 TWO_PI_RES_Q = 2.44929359829470635445213186455000211641949889e-16Q;
static const double TWO_PI_RES_D = 2.4492935982947064e-16;

typedef struct { int64_t quad; int64_t ties; } orc_stats;

/* The distance law in the native representation (Krioukov et al.):
 *   cosh d = cosh r_i cosh r_j - sinh r_i sinh r_j cos(dtheta),
 * rewritten with 1 - cos x = 2 sin^2(x/2) as the sum of non-negative terms
 *   cosh d = cosh(r_i - r_j) + 2 sinh r_i sinh r_j sin^2(dtheta/2),
 * where dtheta is the angle between the points taken in [0, pi].
 * Edge iff cosh d <= cosh R. */
static int edge_quad(double ri, double ti, double rj, double tj, double R, orc_stats *st)
{
    __float128 dq;
    double tmax = ti > tj ? ti : tj, tmin = ti > tj ? tj : ti;
    dq = (__float128)tmax - (__float128)tmin;              /* exact */
    if (dq > M_PIq)                                          /* the short way round */
        dq = ((__float128)(TWO_PI_D - tmax) + (__float128)tmin) + TWO_PI_RES_Q;
    __float128 s = sinq(dq * 0.5Q);
    __float128 L = coshq((__float128)ri - (__float128)rj)
                 + 2.0Q * sinhq((__float128)ri) * sinhq((__float128)rj) * s * s;
    __float128 C = coshq((__float128)R);
    if (fabsq(L - C) <= C * 1e-30Q) st->ties++;
    return L <= C;
}

/* shi, shj: sinh(ri), sinh(rj) as the libm returns them (the callers that
 * test one point against many pass them in from a table of the same values,
 * which leaves every operation and its result unchanged). */
static int edge64s(double ri, double ti, double shi, double rj, double tj, double shj, double R, double coshR,
                   orc_stats *st)
{
    double tmax = ti > tj ? ti : tj, tmin = ti > tj ? tj : ti;
    double d = tmax - tmin;
    /* the short way round; TWO_PI_D - tmax is exact (tmax > pi) */
    if (d > M_PI) d = ((TWO_PI_D - tmax) + tmin) + TWO_PI_RES_D;
    double s = sin(0.5 * d);
    double L = cosh(ri - rj) + 2.0 * shi * shj * s * s;
    if (L < coshR * (1.0 - 1e-9)) return 1;
    if (L > coshR * (1.0 + 1e-9)) return 0;
    st->quad++;
    return edge_quad(ri, ti, rj, tj, R, st);
}

static int edge64(double ri, double ti, double rj, double tj, double R, double coshR, orc_stats *st)
{
    return edge64s(ri, ti, sinh(ri), rj, tj, sinh(rj), R, coshR, st);
}

/* Single pair decision (i != j assumed by the caller). */
int orc_is_edge(double ri, double ti, double rj, double tj, double R, int64_t stats[2])
{
    orc_stats st = {0, 0};
    int e = edge64(ri, ti, rj, tj, R, orc_cosh(R), &st);
    if (stats) { stats[0] += st.quad; stats[1] += st.ties; }
    return e;
}

/* The distance law as printed, evaluated literally in binary64:
 *   cosh r_i cosh r_j - sinh r_i sinh r_j cos(theta_i - theta_j) <= cosh R.
 * Diagnostic only, never used for a decision: near the rim both products
 * are about e^{r_i + r_j} / 4 while their difference is about cosh R, so the
 * cancellation leaves an error of the order of cosh R itself at large R.
 * A test shows how often it disagrees with the exact relation. */
int orc_is_edge_literal(double ri, double ti, double rj, double tj, double R)
{
    const double lhs = cosh(ri) * cosh(rj) - sinh(ri) * sinh(rj) * cos(ti - tj);
    return lhs <= orc_cosh(R);
}

/* Binary128-only decision, for tests of the binary64 screen. */
int orc_is_edge_quad(double ri, double ti, double rj, double tj, double R)
{
    orc_stats st = {0, 0};
    return edge_quad(ri, ti, rj, tj, R, &st);
}

/* deg[i] = |{ j != i : edge(i, j) }| for every i, by testing all pairs. */
void orc_degrees(int64_t n, const double *r, const double *theta, double R,
                 int32_t *deg, int nthreads, int64_t stats[2])
{
    double coshR = orc_cosh(R);
    int64_t q = 0, t = 0;
    if (nthreads > 0) omp_set_num_threads(nthreads);
    #pragma omp parallel for schedule(dynamic, 64) reduction(+:q,t)
    for (int64_t i = 0; i < n; ++i) {
        orc_stats st = {0, 0};
        int32_t c = 0;
        for (int64_t j = 0; j < n; ++j)
            if (j != i) c += edge64(r[i], theta[i], r[j], theta[j], R, coshR, &st);
        deg[i] = c;
        q += st.quad; t += st.ties;
    }
    if (stats) { stats[0] += q; stats[1] += t; }
}

/* Full CSR with ascending rows; row_ptr must hold the exclusive prefix sum
 * of the degrees from orc_degrees (n + 1 entries). */
void orc_csr_fill(int64_t n, const double *r, const double *theta, double R,
                  const int64_t *row_ptr, int32_t *col, int nthreads)
{
    double coshR = orc_cosh(R);
    if (nthreads > 0) omp_set_num_threads(nthreads);
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        orc_stats st = {0, 0};
        int64_t k = row_ptr[i];
        for (int64_t j = 0; j < n; ++j)
            if (j != i && edge64(r[i], theta[i], r[j], theta[j], R, coshR, &st))
                col[k++] = (int32_t)j;
    }
}

/* Neighbours of the vertices in rows[0..nrows), ascending, each row tested
 * against all n points.  out_ptr gets nrows + 1 offsets into out (capacity
 * cap); returns -1 if cap is too small, else the total neighbour count.
 * Rows are taken ORC_ROW_BLOCK at a time; the threads split the vertices
 * into contiguous static ranges and keep their hits in thread order, so each
 * row comes out ascending when the threads' lists are joined in order. */
#define ORC_ROW_BLOCK 32
typedef struct { int64_t *v; int64_t len, cap; } orc_list;

static void list_push(orc_list *l, int64_t x)
{
    if (l->len == l->cap) {
        l->cap = l->cap ? 2 * l->cap : 1024;
        l->v = (int64_t *)realloc(l->v, (size_t)l->cap * sizeof(int64_t));
    }
    l->v[l->len++] = x;
}

int64_t orc_rows(int64_t n, const double *r, const double *theta, double R,
                 const int64_t *rows, int64_t nrows, int64_t *out_ptr, int32_t *out,
                 int64_t cap, int nthreads, int64_t stats[2])
{
    double coshR = orc_cosh(R);
    int64_t q = 0, t = 0, total = 0, overflow = 0;
    if (nthreads > 0) omp_set_num_threads(nthreads);
    const int T = omp_get_max_threads();
    double *sh = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    orc_list *hits = (orc_list *)calloc((size_t)T, sizeof(orc_list));
    #pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j) sh[j] = sinh(r[j]);
    out_ptr[0] = 0;
    for (int64_t a0 = 0; a0 < nrows; a0 += ORC_ROW_BLOCK) {
        const int64_t nb = nrows - a0 < ORC_ROW_BLOCK ? nrows - a0 : ORC_ROW_BLOCK;
        /* hits are (row in block) * 2^40 + j, in ascending j per thread */
        #pragma omp parallel num_threads(T) reduction(+:q,t)
        {
            orc_list *l = &hits[omp_get_thread_num()];
            l->len = 0;
            orc_stats st = {0, 0};
            #pragma omp for schedule(static)
            for (int64_t j = 0; j < n; ++j)
                for (int64_t b = 0; b < nb; ++b) {
                    const int64_t i = rows[a0 + b];
                    if (j != i && edge64s(r[i], theta[i], sh[i], r[j], theta[j], sh[j], R, coshR, &st))
                        list_push(l, (b << 40) | j);
                }
            q += st.quad; t += st.ties;
        }
        for (int64_t b = 0; b < nb; ++b) {
            for (int th = 0; th < T; ++th)
                for (int64_t k = 0; k < hits[th].len; ++k) {
                    if ((hits[th].v[k] >> 40) != b) continue;
                    if (total < cap) out[total] = (int32_t)(hits[th].v[k] & ((1LL << 40) - 1));
                    else overflow = 1;
                    ++total;
                }
            out_ptr[a0 + b + 1] = total;
        }
    }
    for (int th = 0; th < T; ++th) free(hits[th].v);
    free(hits);
    free(sh);
    if (stats) { stats[0] += q; stats[1] += t; }
    return overflow ? -1 : total;
}

/* Whole-graph summary without storing the graph: every pair i < j is tested
 * once; deg[] gets the degrees and fp[0], fp[1] the wrapping sum and the xor,
 * over the edges, of mix64(i * 2^32 + j) -- an order-independent fingerprint
 * of the edge set.  mix64 is the finaliser of Steele, Lea and Flood's
 * SplitMix64 ("Fast splittable pseudorandom number generators", OOPSLA 2014). */
static uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

uint64_t orc_mix64(uint64_t z) { return mix64(z); }

void orc_pair_scan(int64_t n, const double *r, const double *theta, double R, int32_t *deg,
                   uint64_t fp[2], int nthreads, int64_t stats[2], double *loop_s)
{
    double coshR = orc_cosh(R);
    if (nthreads > 0) omp_set_num_threads(nthreads);
    const int T = omp_get_max_threads();
    double *sh = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    int32_t *part = (int32_t *)calloc((size_t)T * (size_t)(n > 0 ? n : 1), sizeof(int32_t));
    uint64_t fsum = 0, fxor = 0;
    int64_t q = 0, t = 0;
    #pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j) sh[j] = sinh(r[j]);
    const double t0 = omp_get_wtime();
    #pragma omp parallel num_threads(T) reduction(+:q,t,fsum) reduction(^:fxor)
    {
        int32_t *d = part + (size_t)omp_get_thread_num() * (size_t)n;
        orc_stats st = {0, 0};
        #pragma omp for schedule(dynamic, 16)
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = i + 1; j < n; ++j)
                if (edge64s(r[i], theta[i], sh[i], r[j], theta[j], sh[j], R, coshR, &st)) {
                    d[i]++;
                    d[j]++;
                    const uint64_t h = mix64(((uint64_t)i << 32) | (uint64_t)j);
                    fsum += h;
                    fxor ^= h;
                }
        q += st.quad; t += st.ties;
    }
    if (loop_s) *loop_s = omp_get_wtime() - t0;  /* the pair loop alone */
    for (int64_t i = 0; i < n; ++i) {
        int32_t c = 0;
        for (int th = 0; th < T; ++th) c += part[(size_t)th * (size_t)n + i];
        deg[i] = c;
    }
    free(part);
    free(sh);
    fp[0] = fsum;
    fp[1] = fxor;
    if (stats) { stats[0] += q; stats[1] += t; }
}

int orc_max_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------------------------------ */
/* Long-range augmentation (RHG-LR: Sec. 4.2, the generator table of   */
/* Sec. 4.3, Appendix I): a small share of extra edges between          */
/* uniformly chosen vertex pairs.                                       */
/* ------------------------------------------------------------------ */

/* Candidate pair j of the augmentation: Philox4x32-10 with the vertex
 * key (seed_lo, seed_hi) and counter (j_lo, j_hi, 1, 0) -- the third word 1
 * keeps these draws apart from the points' (third word 0).  Each 64-bit
 * word w = (x1:x0), (x3:x2) picks a vertex floor(w * n / 2^64); the pair is
 * returned as (min, max).  The paper fixes no generator or pair law beyond
 * "uniformly at random". */
void orc_lr_candidates(uint64_t seed, int64_t j0, int64_t count, int64_t n, int64_t *a, int64_t *b)
{
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int64_t c = 0; c < count; ++c) {
        const uint64_t j = (uint64_t)(j0 + c);
        const uint32_t ctr[4] = {(uint32_t)j, (uint32_t)(j >> 32), 1u, 0u};
        uint32_t x[4];
        orc_philox4x32_10(ctr, key, x);
        const uint64_t w0 = ((uint64_t)x[1] << 32) | x[0], w1 = ((uint64_t)x[3] << 32) | x[2];
        const uint64_t u = (uint64_t)(((unsigned __int128)w0 * (uint64_t)n) >> 64);
        const uint64_t v = (uint64_t)(((unsigned __int128)w1 * (uint64_t)n) >> 64);
        a[c] = (int64_t)(u < v ? u : v);
        b[c] = (int64_t)(u < v ? v : u);
    }
}

/* ------------------------------------------------------------------ */
/* Temperature model.  Sec. 2.1 sets aside Krioukov et al.'s more       */
/* general model, in which a pair is joined with a probability that     */
/* depends on its distance.  Reading taken here: the Fermi-Dirac        */
/* probability of that model with curvature 1,                          */
/*     p(d) = 1 / (1 + e^{(d - R) / (2T)}),  0 < T < 1,                 */
/* which tends to the threshold rule d <= R as T -> 0.  Pair {i, j}     */
/* draws one coin u = a 2^-53 with a = k + 1 in [1, 2^53], k the top    */
/* 53 bits of the word (x1:x0) of the Philox4x32-10 block with key      */
/* (seed_lo, seed_hi) and counter (min(i,j), max(i,j), 2, 0) -- the     */
/* third word 2 keeps coins apart from the points' draws (0) and the    */
/* long-range candidates (1).  The pair is an edge iff u < p(d).        */
/* ------------------------------------------------------------------ */

/* a = k + 1 of pair {i, j} (i != j, both below 2^32). */
uint64_t orc_temp_coin(uint64_t seed, int64_t i, int64_t j)
{
    const uint64_t lo = (uint64_t)(i < j ? i : j), hi = (uint64_t)(i < j ? j : i);
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    const uint32_t ctr[4] = {(uint32_t)lo, (uint32_t)hi, 2u, 0u};
    uint32_t x[4];
    orc_philox4x32_10(ctr, key, x);
    return ((((uint64_t)x[1] << 32) | x[0]) >> 11) + 1;
}

/* With b = 2^53 - a, so that (1 - u)/u = b/a exactly:
 *   u < p(d)  <=>  e^{(d - R)/(2T)} < b/a  <=>  d < D = R + 2T ln(b/a),
 * never when b = 0 (u = 1) or D <= 0 (d >= 0), and otherwise
 *   <=>  cosh d < cosh D,
 * with cosh d in the non-negative form of edge_quad / edge64s. */
static int temp_quad(double ri, double ti, double rj, double tj, double R, double T, uint64_t a, orc_stats *st)
{
    const uint64_t b = (1ull << 53) - a;
    if (b == 0) return 0;
    const __float128 D = (__float128)R + 2.0Q * (__float128)T * logq((__float128)b / (__float128)a);
    if (fabsq(D) <= 1e-30Q) st->ties++;
    if (D <= 0) return 0;
    double tmax = ti > tj ? ti : tj, tmin = ti > tj ? tj : ti;
    __float128 dq = (__float128)tmax - (__float128)tmin;
    if (dq > M_PIq) dq = ((__float128)(TWO_PI_D - tmax) + (__float128)tmin) + TWO_PI_RES_Q;
    const __float128 s = sinq(dq * 0.5Q);
    const __float128 L = coshq((__float128)ri - (__float128)rj)
                       + 2.0Q * sinhq((__float128)ri) * sinhq((__float128)rj) * s * s;
    const __float128 C = coshq(D);
    if (fabsq(L - C) <= C * 1e-30Q) st->ties++;
    return L < C;
}

/* binary64 with a relative margin of 1e-9 (on D near 0 an absolute one),
 * binary128 inside it.  shi, shj as in edge64s. */
static int temp64s(double ri, double ti, double shi, double rj, double tj, double shj, double R, double T,
                   uint64_t a, orc_stats *st)
{
    const uint64_t b = (1ull << 53) - a;
    if (b == 0) return 0;
    const double D = R + 2.0 * T * log((double)b / (double)a);
    if (D < -1e-9) return 0;
    if (D > 1e-9) {
        double tmax = ti > tj ? ti : tj, tmin = ti > tj ? tj : ti;
        double d = tmax - tmin;
        if (d > M_PI) d = ((TWO_PI_D - tmax) + tmin) + TWO_PI_RES_D;
        const double s = sin(0.5 * d);
        const double L = cosh(ri - rj) + 2.0 * shi * shj * s * s;
        const double C = cosh(D);
        if (L < C * (1.0 - 1e-9)) return 1;
        if (L > C * (1.0 + 1e-9)) return 0;
    }
    st->quad++;
    return temp_quad(ri, ti, rj, tj, R, T, a, st);
}

/* Single pair decision for a given coin a (i != j assumed by the caller). */
int orc_temp_is_edge(double ri, double ti, double rj, double tj, double R, double T, uint64_t a, int64_t stats[2])
{
    orc_stats st = {0, 0};
    const int e = temp64s(ri, ti, sinh(ri), rj, tj, sinh(rj), R, T, a, &st);
    if (stats) { stats[0] += st.quad; stats[1] += st.ties; }
    return e;
}

/* binary128 only, for tests of the binary64 stage. */
int orc_temp_is_edge_quad(double ri, double ti, double rj, double tj, double R, double T, uint64_t a)
{
    orc_stats st = {0, 0};
    return temp_quad(ri, ti, rj, tj, R, T, a, &st);
}

/* Every pair i < j, each tested once with its own coin: the edges as
 * (i, j) in out_i, out_j (capacity cap, in no particular order).  Returns
 * the edge count (the lists hold the first cap of them). */
int64_t orc_temp_edges(int64_t n, const double *r, const double *theta, double R, double T, uint64_t seed,
                       int64_t *out_i, int64_t *out_j, int64_t cap, int nthreads, int64_t stats[2])
{
    if (nthreads > 0) omp_set_num_threads(nthreads);
    double *sh = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    int64_t total = 0, q = 0, t = 0;
    #pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j) sh[j] = sinh(r[j]);
    #pragma omp parallel for schedule(dynamic, 16) reduction(+:q,t)
    for (int64_t i = 0; i < n; ++i) {
        orc_stats st = {0, 0};
        for (int64_t j = i + 1; j < n; ++j) {
            const uint64_t a = orc_temp_coin(seed, i, j);
            if (temp64s(r[i], theta[i], sh[i], r[j], theta[j], sh[j], R, T, a, &st)) {
                int64_t k;
                #pragma omp atomic capture
                k = total++;
                if (k < cap) { out_i[k] = i; out_j[k] = j; }
            }
        }
        q += st.quad; t += st.ties;
    }
    free(sh);
    if (stats) { stats[0] += q; stats[1] += t; }
    return total;
}

/* Neighbours of the vertices rows[0..nrows), ascending, each row tested
 * against all n points with the pair's coin; as orc_rows otherwise. */
int64_t orc_temp_rows(int64_t n, const double *r, const double *theta, double R, double T, uint64_t seed,
                      const int64_t *rows, int64_t nrows, int64_t *out_ptr, int32_t *out, int64_t cap,
                      int nthreads, int64_t stats[2])
{
    int64_t q = 0, t = 0, total = 0, overflow = 0;
    if (nthreads > 0) omp_set_num_threads(nthreads);
    const int NT = omp_get_max_threads();
    double *sh = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    orc_list *hits = (orc_list *)calloc((size_t)NT, sizeof(orc_list));
    #pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j) sh[j] = sinh(r[j]);
    out_ptr[0] = 0;
    for (int64_t a0 = 0; a0 < nrows; a0 += ORC_ROW_BLOCK) {
        const int64_t nb = nrows - a0 < ORC_ROW_BLOCK ? nrows - a0 : ORC_ROW_BLOCK;
        #pragma omp parallel num_threads(NT) reduction(+:q,t)
        {
            orc_list *l = &hits[omp_get_thread_num()];
            l->len = 0;
            orc_stats st = {0, 0};
            #pragma omp for schedule(static)
            for (int64_t j = 0; j < n; ++j)
                for (int64_t b = 0; b < nb; ++b) {
                    const int64_t i = rows[a0 + b];
                    if (j == i) continue;
                    const uint64_t a = orc_temp_coin(seed, i, j);
                    if (temp64s(r[i], theta[i], sh[i], r[j], theta[j], sh[j], R, T, a, &st))
                        list_push(l, (b << 40) | j);
                }
            q += st.quad; t += st.ties;
        }
        for (int64_t b = 0; b < nb; ++b) {
            for (int th = 0; th < NT; ++th)
                for (int64_t k = 0; k < hits[th].len; ++k) {
                    if ((hits[th].v[k] >> 40) != b) continue;
                    if (total < cap) out[total] = (int32_t)(hits[th].v[k] & ((1LL << 40) - 1));
                    else overflow = 1;
                    ++total;
                }
            out_ptr[a0 + b + 1] = total;
        }
    }
    for (int th = 0; th < NT; ++th) free(hits[th].v);
    free(hits);
    free(sh);
    if (stats) { stats[0] += q; stats[1] += t; }
    return overflow ? -1 : total;
}
