// rhg_plan.hip -- host planning: alpha, R (Eq. (22)), the derived constants
// the kernels use, and the radial band layout of the index.
#include <math.h>
#include <string.h>

#include <algorithm>

#include "rhg_internal.h"

namespace rhg {

static const dd PI_DD = {3.141592653589793, 1.2246467991473532e-16};

// Expected average degree, Eq. (22) of Krioukov et al. as restated in
// Appendix B.1, curvature zeta = 1, xi = alpha / (alpha - 1/2):
//   kbar = (2/pi) xi^2 n ( e^{-R/2} + e^{-alpha R} ( alpha (R/2) inner - 1 ) ),
//   inner = (pi/4) (1/alpha)^2 - (pi - 1) (1/alpha) + (pi - 2).
// The printed "(pi-1) xi/alpha" is read as (pi-1) zeta/alpha: with xi/alpha
// heavy-tailed targets have no root at all.  Evaluated in double-double.
static dd kbar_eq22(double n, double alpha, double R)
{
    dd a = dd_make(alpha);
    dd inv_a = dd_div(dd_make(1.0), a);
    dd xi = dd_div(a, dd_add_d(a, -0.5));
    dd inner = dd_mul(dd_mul(dd_mul_pow2(PI_DD, 0.25), inv_a), inv_a);
    inner = dd_sub(inner, dd_mul(dd_add_d(PI_DD, -1.0), inv_a));
    inner = dd_add(inner, dd_add_d(PI_DD, -2.0));
    dd aR = two_prod(alpha, R);
    dd t1 = dd_exp(dd_make(-0.5 * R));  // R/2 is exact
    dd t2 = dd_exp(dd_neg(aR));
    dd bracket = dd_add_d(dd_mul(dd_mul_d(aR, 0.5), inner), -1.0);
    dd t = dd_add(t1, dd_mul(t2, bracket));
    dd pref = dd_mul(dd_div(dd_make(2.0), PI_DD), dd_mul(xi, xi));
    return dd_mul(dd_mul_d(pref, n), t);
}

static bool above(double n, double alpha, double R, double target)
{
    return dd_cmp(kbar_eq22(n, alpha, R), dd_make(target)) > 0;
}

// Eq. (22) in plain binary64: only used to find the peak and to place a
// narrow bracket around the crossing; every decision that fixes R is taken
// by the double-double evaluation above.
static double kbar_eq22_d(double n, double alpha, double R)
{
    const double pi = 3.141592653589793;
    const double ia = 1.0 / alpha, xi = alpha / (alpha - 0.5);
    const double inner = 0.25 * pi * ia * ia - (pi - 1.0) * ia + (pi - 2.0);
    return (2.0 / pi) * xi * xi * n * (exp(-0.5 * R) + exp(-alpha * R) * (alpha * 0.5 * R * inner - 1.0));
}

// R = smallest binary64 on the decreasing branch of Eq. (22) whose value is
// <= target.  The branch starts at the maximum of Eq. (22) (golden-section
// search) and the search ends at 2 ln n + 40.  A binary64 bisection places
// the crossing to a few ulps; the bracket is then widened until the
// double-double predicate holds at its ends and bisected down to adjacent
// doubles, so the result depends only on where Eq. (22) crosses the target.
static rhg_status solve_radius(double n, double alpha, double target, double *R_out)
{
    const double top = 2.0 * log(n) + 40.0;
    double a = 1e-6, b = top;
    const double g = 0.6180339887498949;
    for (int it = 0; it < 100 && b - a > 1e-12 * b; ++it) {
        const double c = b - g * (b - a), d = a + g * (b - a);
        if (kbar_eq22_d(n, alpha, c) > kbar_eq22_d(n, alpha, d)) b = d; else a = c;
    }
    const double peak = 0.5 * (a + b);
    if (!above(n, alpha, peak, target))
        return fail(RHG_ENOROOT, "average degree exceeds the maximum of Eq. (22) for this n and gamma");
    if (above(n, alpha, top, target)) return fail(RHG_ENOROOT, "Eq. (22) bracket does not contain the target");
    double lo = peak, hi = top;
    for (int it = 0; it < 200; ++it) {  // binary64 estimate of the crossing
        const double mid = lo + 0.5 * (hi - lo);
        if (mid <= lo || mid >= hi) break;
        if (kbar_eq22_d(n, alpha, mid) > target) lo = mid; else hi = mid;
    }
    // widen [lo, hi] geometrically until the exact predicate brackets it
    double step = 4.0 * (nextafter(hi, INFINITY) - hi);
    double L = std::max(peak, lo - step), H = std::min(top, hi + step);
    while (L > peak && !above(n, alpha, L, target)) {
        step *= 8.0;
        L = std::max(peak, lo - step);
    }
    step = 4.0 * (nextafter(hi, INFINITY) - hi);
    while (H < top && above(n, alpha, H, target)) {
        step *= 8.0;
        H = std::min(top, hi + step);
    }
    lo = L;
    hi = H;
    for (;;) {
        const double mid = lo + 0.5 * (hi - lo);
        if (mid <= lo || mid >= hi) break;
        if (above(n, alpha, mid, target)) lo = mid; else hi = mid;
    }
    *R_out = hi;
    return RHG_OK;
}

static void derive(rhg_params *p)
{
    dd cR = dd_cosh(dd_make(p->R));
    p->cosh_R = cR.hi;
    p->cosh_R_lo = cR.lo;
    dd aR = two_prod(p->alpha, p->R);
    dd c = dd_add_d(dd_cosh(aR), -1.0);
    p->cosh_aR_m1 = c.hi;
    p->cosh_aR_m1_lo = c.lo;
}

rhg_status plan(int64_t n, double kbar, double gamma, uint64_t seed, rhg_params *out)
{
    if (!out) return fail(RHG_EINVAL, "rhg_plan: out is NULL");
    if (n < 0 || n > 2147483647LL) return fail(RHG_EINVAL, "rhg_plan: n must be in [0, 2^31 - 1]");
    if (!(gamma > 2.0) || !isfinite(gamma))
        return fail(RHG_EINVAL, "rhg_plan: gamma must be a finite number > 2 (alpha > 1/2)");
    if (!(kbar > 0.0) || !isfinite(kbar)) return fail(RHG_EINVAL, "rhg_plan: avg_degree must be > 0");
    if (n >= 2 && !(kbar < (double)(n - 1)))
        return fail(RHG_EINVAL, "rhg_plan: avg_degree must be < n - 1");
    rhg_params p;
    memset(&p, 0, sizeof(p));
    p.n = n;
    p.avg_degree = kbar;
    p.gamma = gamma;
    p.seed = seed;
    p.alpha = (gamma - 1.0) * 0.5;
    if (n >= 2) {
        rhg_status s = solve_radius((double)n, p.alpha, kbar, &p.R);
        if (s != RHG_OK) return s;
        if (!(p.R < 80.0))
            return fail(RHG_EINVAL, "rhg_plan: the requested degree needs R >= 80, beyond the search's range");
    } else {
        p.R = 1.0;  // no pairs: any radius gives the empty graph
    }
    derive(&p);
    *out = p;
    return RHG_OK;
}

rhg_status plan_radius(int64_t n, double alpha, double R, uint64_t seed, rhg_params *out)
{
    if (!out) return fail(RHG_EINVAL, "rhg_plan_radius: out is NULL");
    if (n < 0 || n > 2147483647LL) return fail(RHG_EINVAL, "rhg_plan_radius: n must be in [0, 2^31 - 1]");
    if (!(alpha > 0.5) || !isfinite(alpha)) return fail(RHG_EINVAL, "rhg_plan_radius: alpha must be > 1/2");
    if (!(R > 0.0) || !(R < 80.0)) return fail(RHG_EINVAL, "rhg_plan_radius: R must be in (0, 80)");
    if (!(alpha * R < 600.0)) return fail(RHG_EINVAL, "rhg_plan_radius: alpha * R must be < 600");
    rhg_params p;
    memset(&p, 0, sizeof(p));
    p.n = n;
    p.avg_degree = NAN;
    p.gamma = NAN;
    p.seed = seed;
    p.alpha = alpha;
    p.R = R;
    derive(&p);
    *out = p;
    return RHG_OK;
}

// Radial band layout.  The outer bands have (at most) the tuning's width
// and end at R; everything below `inner_radius` forms one band, chosen by
// default so that it holds about one point in expectation (the CDF of
// Eq. (1) at that radius is 1/n).  Each band's angular cells hold about
// `cell_target` points in expectation, so the cells are the equal-mass
// leaves of the paper's polar quadtree restricted to that band (Lemma 1).
void make_layout(const rhg_params &p, const rhg_tuning *t, Layout *L)
{
    memset(L, 0, sizeof(*L));
    const double R = p.R, a = p.alpha;
    const double n = (double)std::max<int64_t>(p.n, 1);
    double w = (t && t->band_width > 0.0) ? t->band_width : 2.0;
    double rin;
    if (t && t->inner_radius > 0.0) rin = std::min(t->inner_radius, R);
    else rin = std::max(0.0, R - log(std::max(n, 2.0)) / a);
    int K = (int)ceil((R - rin) / w);
    if (K < 1) K = 1;
    int maxK = RHG_MAX_BANDS - (rin > 0.0 ? 1 : 0);
    if (K > maxK) K = maxK;
    int B = 0;
    L->E[B] = 0.0;
    if (rin > 0.0) L->E[++B] = rin;
    for (int i = 1; i <= K; ++i) L->E[B + i] = (i == K) ? R : rin + (R - rin) * (double)i / (double)K;
    B += K;
    L->B = B;
    int bb = 0;
    while ((1 << bb) < B) ++bb;
    L->band_bits = bb;
    double target = (t && t->cell_target > 0) ? (double)t->cell_target : 1.0;
    double denom = p.cosh_aR_m1;
    int64_t base = 0;
    for (int j = 0; j < B; ++j) {
        double F0 = (cosh(a * L->E[j]) - 1.0) / denom;
        double F1 = (cosh(a * L->E[j + 1]) - 1.0) / denom;
        double expect = n * std::max(0.0, std::min(1.0, F1) - F0);
        int cb = 0;
        while (cb < 32 - bb && (double)(1ull << cb) * target < expect) ++cb;
        L->cbits[j] = cb;
        L->dir_base[j] = base;
        base += (int64_t)(1ull << cb) + 1;
    }
    L->dir_base[B] = base;
    L->dir_total = base;
    // Heavy queries: the innermost bands, holding about `heavy_points` points
    // in expectation (those with the largest degrees, about 5e3 and more at
    // n = 1e8).  The cap leaves room for the statistical excess.
    const double hp = (t && t->heavy_points > 0) ? (double)t->heavy_points : 16384.0;
    int jh = 0;
    while (jh < B && n * ((cosh(a * L->E[jh + 1]) - 1.0) / denom) <= hp) ++jh;
    if (jh >= B) jh = B - 1;
    L->heavy_band = jh;
    const double cap = 1.25 * hp + 1024.0;
    L->heavy_cap = jh > 0 ? (int64_t)std::min(cap, n) : 0;
    // An upper estimate of the entries of the graph (2m): per band
    // sub-interval, its expected points times the expected degree at its
    // inner edge, where the degree is largest.  It sizes the workspace of
    // the canonical row sort.
    double entries = 0.0;
    for (int j = 0; j < B; ++j) {
        for (int sub = 0; sub < RHG_KAP_SUB; ++sub) {
            const double ra = L->E[j] + (L->E[j + 1] - L->E[j]) * sub / RHG_KAP_SUB;
            const double rb = L->E[j] + (L->E[j + 1] - L->E[j]) * (sub + 1) / RHG_KAP_SUB;
            const double pts = n * std::max(0.0, (cosh(a * rb) - cosh(a * ra)) / denom);
            if (pts <= 0.0) continue;
            entries += pts * expected_degree(n, a, R, ra);
        }
    }
    L->entries_est = p.n >= 2 ? entries : 0.0;
    L->fp64_only = (t && t->fp64_only) ? 1 : 0;
    L->no_stream_stage = (t && t->no_stream_stage) ? 1 : 0;
    // A wavefront's union window of up to sweep_max candidates is staged and
    // swept even where its lanes' windows do not overlap: one contiguous
    // read for all lanes instead of a directory lookup and a run per lane.
    L->sweep_max = (t && t->sweep_max > 0) ? t->sweep_max : (t && t->sweep_max < 0) ? 0 : 128;
    L->sweep_linear = (t && t->sweep_linear) ? 1 : 0;
    // Pairs the FP32 screen leaves undecided are listed for an exact pass
    // after the search (about 1.5e-4 of the edges at n = 1e8); a longer list
    // sends both passes to the kernels that decide them in place.
    L->exact_inline = (t && t->exact_inline) ? 1 : 0;
    L->defer_cap = (t && t->defer_cap > 0) ? (int64_t)t->defer_cap : 65536 + (int64_t)(n / 1024.0);
    int64_t hs = 1;
    while (hs < 2 * L->defer_cap) hs <<= 1;
    L->hset_slots = hs;
    // Staged count: a light query's slot holds its row's length, then room
    // for stage_pct % of mu + 5 sqrt(mu) + 8 entries (at most 2^24), mu the
    // expected degree at the query's radius (log-linear between its band's
    // edges, raised by the largest ratio of the true curve to that line at
    // 15 inner points), in a multiple of 4 words.  A row that outgrows its
    // slot is searched again by the emit pass.  The workspace holds the
    // slots' expected total over the light bands' radii plus ten standard
    // deviations and 64 of the largest slots, plus 5 % for the temperature
    // model's larger slots; a slot's start / 4 + 1 must fit in 32 bits.
    const int st = t ? t->stage : 0;
    L->staged = (st > 0 || (st == 0 && p.n >= (int64_t)1 << 19)) && p.n >= 1 ? 1 : 0;
    L->stage_cap = 0;
    if (L->staged) {
        const double pct = (t && t->stage_pct > 0) ? t->stage_pct / 100.0 : 1.0;
        L->stage_f = (float)pct;
        double mean = 0.0, var = 0.0, maxw = 0.0;
        for (int j = 0; j < B; ++j) {
            const double e0 = L->E[j], e1 = L->E[j + 1];
            const double m0 = std::max(expected_degree(n, a, R, e0), 1e-6);
            const double m1 = std::max(expected_degree(n, a, R, e1), 1e-6);
            double corr = 1.0;
            for (int k = 1; k < 16; ++k) {
                const double f = k / 16.0;
                const double line = exp((1.0 - f) * log(m0) + f * log(m1));
                corr = std::max(corr, expected_degree(n, a, R, e0 + (e1 - e0) * f) / line);
            }
            corr *= 1.001;
            L->lmu_in[j] = (float)log2(m0 * corr);
            L->lmu_out[j] = (float)log2(m1 * corr);
            if (j < jh) continue;  // heavy bands: no slots
            for (int sub = 0; sub < 64; ++sub) {
                const double ra = e0 + (e1 - e0) * sub / 64.0, rb = e0 + (e1 - e0) * (sub + 1) / 64.0;
                const double pts = n * std::max(0.0, (cosh(a * rb) - cosh(a * ra)) / denom);
                // the largest slot of the sub-interval (the degree falls with r),
                // with room for the device's single-precision rounding
                const double f = (ra - e0) / (e1 - e0);
                const double mu = exp2((1.0 - f) * L->lmu_in[j] + f * L->lmu_out[j]) * 1.01;
                const double wd = std::min(pct * (mu + 5.0 * sqrt(mu) + 8.0), 16777216.0) + 8.0;
                mean += pts * wd;
                var += pts * wd * wd;
                maxw = std::max(maxw, wd);
            }
        }
        const double cap = 1.05 * (mean + 10.0 * sqrt(var) + 64.0 * maxw + 1024.0);
        L->stage_cap = (int64_t)std::min(cap, 4.0 * 4294967294.0);
    }
}

}  // namespace rhg
