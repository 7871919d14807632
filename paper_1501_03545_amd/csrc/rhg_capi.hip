// rhg_capi.hip -- the extern "C" boundary: argument checks, workspace
// carving, launch sequencing and error reporting.  No exception crosses it.
#include <stdio.h>
#include <string.h>

#include <math.h>

#include <algorithm>
#include <limits>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "rhg_internal.h"

namespace rhg {

static thread_local std::string g_last_error;

rhg_status fail(rhg_status s, const std::string &msg)
{
    g_last_error = msg;
    return s;
}

rhg_status check_hip(hipError_t e, const char *what)
{
    return fail(RHG_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

rhg_status plan(int64_t n, double kbar, double gamma, uint64_t seed, rhg_params *out);
rhg_status plan_radius(int64_t n, double alpha, double R, uint64_t seed, rhg_params *out);

__global__ void zero_u64_kernel(unsigned long long *p, int count)
{
    const int i = threadIdx.x;
    if (i < count) p[i] = 0ull;
}

// ---- optional phase timing: HIP events recorded on the caller's stream
// around each kernel group, kept in a ring and averaged on request.
static const char *kPhaseNames[RHG_PHASE_COUNT] = {"sample", "keys+sort", "index", "gather", "plan",
                                                   "count", "scan", "emit", "rows"};
struct ProfRec {
    int phase;
    hipEvent_t a, b;
};
static const int kProfRing = 512;
static ProfRec g_prof[kProfRing];
static int g_prof_on = 0, g_prof_next = 0, g_prof_used = 0, g_prof_ready = 0;

void *phase_begin(int phase, hipStream_t s)
{
    if (!g_prof_on || !g_prof_ready) return nullptr;
    ProfRec *rec = &g_prof[g_prof_next];
    g_prof_next = (g_prof_next + 1) % kProfRing;
    if (g_prof_used < kProfRing) ++g_prof_used;
    rec->phase = phase;
    (void)hipEventRecord(rec->a, s);
    return rec;
}

void phase_end(void *rec, hipStream_t s)
{
    if (rec) (void)hipEventRecord(((ProfRec *)rec)->b, s);
}

struct WsPlan {
    size_t keys, v0, band_start, dir, sr, st, rec, rt, heavy_end, hplan, hcnt, hitem, hscal, stats, wstat, dkeys, dchunk,
        dcount, hset, dslot, stage, sslot, sovf, wsum, raux, tmp, total, tmp_bytes;
    int64_t max_chunks, rows_lcap, rows_mapcap, rows_nnz_cap;
};

static WsPlan ws_plan(int64_t n, const Layout &L)
{
    WsPlan w;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes, 256);
        return o;
    };
    const size_t N = (size_t)(n > 0 ? n : 1);
    w.keys = take(N * 4);
    w.v0 = take(N * 4);
    w.band_start = take((size_t)(L.B + 1) * 4);
    w.dir = take((size_t)L.dir_total * 4);
    w.sr = take(N * 8);
    w.st = take(N * 8);
    w.rec = take(N * 16);
    w.rt = take(N * 16);
    w.heavy_end = take(16);
    const int64_t items = L.heavy_cap * L.B;
    // Each heavy query's windows cover at most the n points once, so the
    // chunk count stays below items + heavy_cap * n / RHG_HEAVY_CHUNK + 1;
    // past RHG_HEAVY_EXTRA_CHUNKS the planner widens the chunks instead.
    const int64_t extra = std::min<int64_t>(RHG_HEAVY_EXTRA_CHUNKS, L.heavy_cap * (n / RHG_HEAVY_CHUNK + 1) + 1);
    w.max_chunks = items > 0 ? items + extra : 1;
    w.hplan = take((size_t)(items > 0 ? items : 1) * 8);
    w.hcnt = take((size_t)w.max_chunks * 8);
    w.hitem = take((size_t)w.max_chunks * 4);
    w.hscal = take(64);
    w.stats = take(ST_COUNT * 8);
    w.wstat = take((N + 63) / 64 * 16);
    w.dkeys = take((size_t)L.defer_cap * 8);
    w.dchunk = take((size_t)L.defer_cap * 4);
    w.dcount = take(16);
    w.hset = take((size_t)L.hset_slots * 8);
    w.dslot = take(L.staged ? (size_t)L.defer_cap * 8 : 8);
    w.stage = take(L.staged ? (size_t)L.stage_cap * 4 : 4);
    w.sslot = take(L.staged ? N * 4 : 4);
    w.sovf = take(L.staged ? (N + 63) / 64 : 1);
    w.wsum = take(L.staged ? (size_t)((N + 63) / 64) * 8 : 8);
    // canonical rows: room for the long rows and tiles of a graph of up to
    // twice the estimated entries (plus 2^23)
    w.rows_nnz_cap = (int64_t)std::min(9.0e18, 2.0 * L.entries_est + 8388608.0);
    w.rows_lcap = std::min<int64_t>((int64_t)N, rows_long_bound(w.rows_nnz_cap));
    w.rows_mapcap = rows_tile_bound(w.rows_nnz_cap, w.rows_lcap);
    w.raux = take(rows_aux_bytes(w.rows_lcap, w.rows_mapcap));
    size_t t1 = radix_sort_tmp_bytes(n), t2 = scan_tmp_bytes(n + 1);
    size_t t3 = scan_tmp_bytes(w.max_chunks), t4 = scan_tmp_bytes(items > 0 ? items : 1);
    w.tmp_bytes = std::max(std::max(t1, t2), std::max(t3, t4));
    w.tmp = take(w.tmp_bytes);
    w.total = off + 256;  // slack for aligning the base pointer
    return w;
}

}  // namespace rhg

using namespace rhg;

extern "C" {

const char *rhg_last_error(void) { return g_last_error.c_str(); }

const char *rhg_version(void) { return "rhg-mi355x 0.1 (gfx950)"; }

rhg_status rhg_set_profiling(int on)
{
    g_last_error.clear();
    if (on && !g_prof_ready) {
        for (int i = 0; i < kProfRing; ++i) {
            RHG_HIP(hipEventCreate(&g_prof[i].a));
            RHG_HIP(hipEventCreate(&g_prof[i].b));
        }
        g_prof_ready = 1;
    }
    g_prof_on = on ? 1 : 0;
    g_prof_next = 0;
    g_prof_used = 0;
    return RHG_OK;
}

rhg_status rhg_phase_times(double *avg_ms, int64_t *count, int cap)
{
    g_last_error.clear();
    if (!avg_ms || !count || cap < RHG_PHASE_COUNT) return fail(RHG_EINVAL, "rhg_phase_times: bad buffers");
    for (int k = 0; k < RHG_PHASE_COUNT; ++k) { avg_ms[k] = 0.0; count[k] = 0; }
    for (int i = 0; i < g_prof_used; ++i) {
        RHG_HIP(hipEventSynchronize(g_prof[i].b));
        float ms = 0.f;
        RHG_HIP(hipEventElapsedTime(&ms, g_prof[i].a, g_prof[i].b));
        avg_ms[g_prof[i].phase] += ms;
        count[g_prof[i].phase] += 1;
    }
    for (int k = 0; k < RHG_PHASE_COUNT; ++k)
        if (count[k]) avg_ms[k] /= (double)count[k];
    return RHG_OK;
}

const char *rhg_phase_name(int phase)
{
    return (phase >= 0 && phase < RHG_PHASE_COUNT) ? kPhaseNames[phase] : "";
}

rhg_status rhg_plan(int64_t n, double avg_degree, double gamma, uint64_t seed, rhg_params *out)
{
    g_last_error.clear();
    return plan(n, avg_degree, gamma, seed, out);
}

rhg_status rhg_plan_radius(int64_t n, double alpha, double R, uint64_t seed, rhg_params *out)
{
    g_last_error.clear();
    return plan_radius(n, alpha, R, seed, out);
}

static rhg_status check_params(const rhg_params *p, const char *who)
{
    if (!p) return fail(RHG_EINVAL, std::string(who) + ": params is NULL");
    if (p->n < 0 || p->n > 2147483647LL) return fail(RHG_EINVAL, std::string(who) + ": n out of range");
    if (!(p->alpha > 0.5) || !(p->R > 0.0) || !(p->cosh_R >= 1.0) || !(p->cosh_aR_m1 > 0.0))
        return fail(RHG_EINVAL, std::string(who) + ": params were not filled by rhg_plan");
    // the search's FP32 records (e^r / sqrt(2 cosh R) and its kin) and the
    // screen's error bound need R < 80
    if (!(p->R < 80.0)) return fail(RHG_EINVAL, std::string(who) + ": R must be below 80");
    return RHG_OK;
}

rhg_status rhg_sample_points(const rhg_params *p, double *r, double *theta, void *stream)
{
    g_last_error.clear();
    rhg_status st = check_params(p, "rhg_sample_points");
    if (st != RHG_OK) return st;
    if (p->n > 0 && (!r || !theta)) return fail(RHG_EINVAL, "rhg_sample_points: NULL output");
    PhaseScope ps(RHG_PHASE_SAMPLE, (hipStream_t)stream);
    RHG_HIP(launch_sample(*p, r, theta, (hipStream_t)stream));
    return RHG_OK;
}

rhg_status rhg_layout_bands(const rhg_params *p, const rhg_tuning *t, double *edges, int cap, int *bands)
{
    g_last_error.clear();
    rhg_status st = check_params(p, "rhg_layout_bands");
    if (st != RHG_OK) return st;
    if (!edges || !bands || cap < 0) return fail(RHG_EINVAL, "rhg_layout_bands: NULL output");
    Layout L;
    make_layout(*p, t, &L);
    *bands = L.B;
    for (int j = 0; j <= L.B && j < cap; ++j) edges[j] = L.E[j];
    return RHG_OK;
}

size_t rhg_index_workspace_bytes(const rhg_params *p, const rhg_tuning *t)
{
    if (!p) return 0;
    Layout L;
    make_layout(*p, t, &L);
    return ws_plan(p->n, L).total;
}

rhg_status rhg_build_index(const rhg_params *p, const double *r, const double *theta, const rhg_tuning *t,
                           void *workspace, size_t workspace_bytes, int validate, rhg_index **out,
                           void *stream)
{
    g_last_error.clear();
    rhg_status st = check_params(p, "rhg_build_index");
    if (st != RHG_OK) return st;
    if (!out) return fail(RHG_EINVAL, "rhg_build_index: out is NULL");
    *out = nullptr;
    if (p->n > 0 && (!r || !theta)) return fail(RHG_EINVAL, "rhg_build_index: NULL points");
    if (t && (t->band_width < 0.0 || t->inner_radius < 0.0 || t->cell_target < 0 || t->heavy_points < 0 ||
              !(t->band_width < 1e6)))
        return fail(RHG_EINVAL, "rhg_build_index: negative tuning value");
    rhg_index *idx = new (std::nothrow) rhg_index;
    if (!idx) return fail(RHG_ENOMEM, "rhg_build_index: host allocation failed");
    memset(idx, 0, sizeof(*idx));
    idx->p = *p;
    idx->n = p->n;
    make_layout(*p, t, &idx->L);
    const WsPlan w = ws_plan(p->n, idx->L);
    if (!workspace || workspace_bytes < w.total) {
        delete idx;
        return fail(RHG_ECAPACITY, "rhg_build_index: workspace smaller than rhg_index_workspace_bytes");
    }
    char *base = (char *)align_up((size_t)workspace, 256);
    idx->keys = (uint32_t *)(base + w.keys);
    uint32_t *v0 = (uint32_t *)(base + w.v0);
    idx->ids = v0;
    idx->band_start = (int32_t *)(base + w.band_start);
    idx->dir = (int32_t *)(base + w.dir);
    idx->sr = (double *)(base + w.sr);
    idx->st = (double *)(base + w.st);
    idx->rec = (float4 *)(base + w.rec);
    idx->rt = (double2 *)(base + w.rt);
    idx->heavy_end = (int32_t *)(base + w.heavy_end);
    idx->hplan = (int64_t *)(base + w.hplan);
    idx->hcnt = (int64_t *)(base + w.hcnt);
    idx->hitem = (int32_t *)(base + w.hitem);
    idx->hscal = (int64_t *)(base + w.hscal);
    idx->heavy_cap = idx->L.heavy_cap;
    idx->max_chunks = w.max_chunks;
    idx->stats = (unsigned long long *)(base + w.stats);
    idx->wstat = base + w.wstat;
    idx->dkeys = (uint64_t *)(base + w.dkeys);
    idx->dchunk = (int32_t *)(base + w.dchunk);
    idx->dcount = (unsigned long long *)(base + w.dcount);
    idx->hset = (uint64_t *)(base + w.hset);
    idx->dslot = (int64_t *)(base + w.dslot);
    idx->stage = (int32_t *)(base + w.stage);
    idx->sslot = (uint32_t *)(base + w.sslot);
    idx->sovf = (uint8_t *)(base + w.sovf);
    idx->wsum = (int64_t *)(base + w.wsum);
    idx->hset_slots = idx->L.hset_slots;
    idx->rows_aux = base + w.raux;
    idx->rows_lcap = w.rows_lcap;
    idx->rows_mapcap = w.rows_mapcap;
    idx->rows_nnz_cap = w.rows_nnz_cap;
    idx->tmp = base + w.tmp;
    idx->tmp_bytes = w.tmp_bytes;
    // the sort's second key/value buffers live in the FP32 record array,
    // which the gather step fills only after the sort has finished
    uint32_t *k1 = (uint32_t *)idx->rec;
    uint32_t *v1 = k1 + (p->n > 0 ? p->n : 1);
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(64), 0, s, idx->stats, (int)ST_COUNT);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = launch_build_index(idx, r, theta, k1, v0, v1, validate, s);
    if (e != hipSuccess) {
        delete idx;
        return check_hip(e, "rhg_build_index");
    }
    if (validate) {
        unsigned long long bad = 0;
        e = hipMemcpyAsync(&bad, idx->stats + ST_BAD_INPUT, 8, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            delete idx;
            return check_hip(e, "rhg_build_index (validate)");
        }
        if (bad) {
            delete idx;
            return fail(RHG_EINVAL, "rhg_build_index: " + std::to_string(bad) +
                                        " points outside 0 <= r <= R, 0 <= theta < 2 pi");
        }
    }
    *out = idx;
    return RHG_OK;
}

rhg_status rhg_count_edges(rhg_index *idx, int64_t *row_ptr, void *stream)
{
    g_last_error.clear();
    if (!idx || !row_ptr) return fail(RHG_EINVAL, "rhg_count_edges: NULL argument");
    hipStream_t s = (hipStream_t)stream;
    RHG_HIP(launch_search(idx, row_ptr, nullptr, 0, s));
    idx->counted = 1;
    idx->count_model = 1;
    if (idx->n > 0) {
        PhaseScope ps(RHG_PHASE_SCAN, s);
        RHG_HIP(inclusive_scan_i64(row_ptr + 1, idx->n, idx->tmp, s));
    }
    return RHG_OK;
}

rhg_status rhg_emit_edges(rhg_index *idx, const int64_t *row_ptr, int32_t *col_idx, int64_t col_capacity,
                          int canonical_rows, void *stream)
{
    g_last_error.clear();
    if (!idx || !row_ptr) return fail(RHG_EINVAL, "rhg_emit_edges: NULL argument");
    if (col_capacity < 0) return fail(RHG_EINVAL, "rhg_emit_edges: negative capacity");
    if (idx->count_model != 1) return fail(RHG_EINVAL, "rhg_emit_edges: the index's last count pass was not rhg_count_edges");
    hipStream_t s = (hipStream_t)stream;
    int64_t nnz = 0;
    RHG_HIP(hipMemcpyAsync(&nnz, row_ptr + idx->n, 8, hipMemcpyDeviceToHost, s));
    RHG_HIP(hipStreamSynchronize(s));
    if (nnz > col_capacity)
        return fail(RHG_ECAPACITY, "rhg_emit_edges: col_idx holds " + std::to_string(col_capacity) +
                                       " entries, the graph needs " + std::to_string(nnz));
    if (nnz > 0 && !col_idx) return fail(RHG_EINVAL, "rhg_emit_edges: col_idx is NULL");
    if (canonical_rows && nnz > idx->rows_nnz_cap)
        return fail(RHG_ECAPACITY, "rhg_emit_edges: canonical rows of " + std::to_string(nnz) +
                                       " entries (over twice the expected count) need rhg_sort_rows");
    if (nnz > 0) RHG_HIP(launch_search(idx, (int64_t *)row_ptr, col_idx, 1, s));
    if (nnz > 0 && canonical_rows) {
        PhaseScope ps(RHG_PHASE_ROWS, s);
        RHG_HIP(launch_sort_rows(row_ptr, col_idx, idx->n, std::min<int64_t>(nnz, idx->n - 1), idx->rows_aux,
                                 idx->rows_lcap, idx->rows_mapcap, s));
    }
    return RHG_OK;
}

static int64_t sort_lcap(int64_t n, int64_t nnz) { return std::min<int64_t>(std::max<int64_t>(n, 1), rows_long_bound(nnz)); }

size_t rhg_sort_rows_workspace_bytes(int64_t n, int64_t nnz)
{
    if (n < 0 || nnz < 0) return 0;
    const int64_t lcap = sort_lcap(n, nnz);
    return rows_aux_bytes(lcap, rows_tile_bound(nnz, lcap)) + 256;
}

rhg_status rhg_sort_rows(int64_t n, const int64_t *row_ptr, int32_t *col_idx, int64_t nnz, void *workspace,
                         size_t workspace_bytes, void *stream)
{
    g_last_error.clear();
    if (n < 0 || n > (int64_t)INT32_MAX || nnz < 0) return fail(RHG_EINVAL, "rhg_sort_rows: bad n or nnz");
    if (n == 0 || nnz == 0) return RHG_OK;
    if (!row_ptr || !col_idx || !workspace) return fail(RHG_EINVAL, "rhg_sort_rows: NULL argument");
    if (workspace_bytes < rhg_sort_rows_workspace_bytes(n, nnz))
        return fail(RHG_ECAPACITY, "rhg_sort_rows: workspace smaller than rhg_sort_rows_workspace_bytes");
    void *aux = (void *)align_up((size_t)workspace, 256);
    const int64_t lcap = sort_lcap(n, nnz);
    hipStream_t s = (hipStream_t)stream;
    PhaseScope ps(RHG_PHASE_ROWS, s);
    RHG_HIP(launch_sort_rows(row_ptr, col_idx, n, nnz, aux, lcap, rows_tile_bound(nnz, lcap), s));
    return RHG_OK;
}

size_t rhg_graph_stats_workspace_bytes(int64_t n, int64_t nnz, int triangles)
{
    if (n < 0 || nnz < 0) return 0;
    return stats_workspace_bytes(n, nnz, triangles ? 1 : 0);
}

rhg_status rhg_graph_stats(int64_t n, const int64_t *row_ptr, const int32_t *col_idx, int64_t nnz, double kmin,
                           int triangles, void *workspace, size_t workspace_bytes, rhg_graph_summary *out,
                           void *stream)
{
    g_last_error.clear();
    if (n < 0 || n > (int64_t)INT32_MAX || nnz < 0) return fail(RHG_EINVAL, "rhg_graph_stats: bad n or nnz");
    if (!(kmin >= 1.0)) return fail(RHG_EINVAL, "rhg_graph_stats: kmin must be at least 1");
    if (!out || !row_ptr || !workspace || (nnz > 0 && !col_idx)) return fail(RHG_EINVAL, "rhg_graph_stats: NULL argument");
    if (workspace_bytes < stats_workspace_bytes(n, nnz, triangles ? 1 : 0))
        return fail(RHG_ECAPACITY, "rhg_graph_stats: workspace smaller than rhg_graph_stats_workspace_bytes");
    double d[8] = {0};
    int64_t iv[48] = {0};
    RHG_HIP(launch_graph_stats(n, row_ptr, col_idx, nnz, kmin, triangles ? 1 : 0, workspace, d, iv,
                               (hipStream_t)stream));
    memset(out, 0, sizeof(*out));
    const double nan = std::numeric_limits<double>::quiet_NaN();
    out->n = n;
    out->nnz = nnz;
    out->max_degree = iv[0];
    for (int b = 0; b < 33; ++b) out->hist[b] = iv[8 + b];
    out->kmin = kmin;
    out->tail_count = iv[1];
    out->gamma_mle = iv[1] > 0 ? 1.0 + (double)iv[1] / d[0] : nan;
    out->assortativity = nan;
    if (nnz > 0) {
        const double M = (double)nnz, ex = d[1] / M, exx = d[2] / M, exy = d[3] / M;
        const double var = exx - ex * ex;
        if (var > 0.0) out->assortativity = (exy - ex * ex) / var;
    }
    out->triads = iv[2];
    out->ascending_rows = iv[3] ? 0 : 1;
    out->triangles = iv[4];
    out->transitivity = nan;
    out->avg_local_clustering = nan;
    if (iv[4] >= 0) {
        if (iv[2] > 0) out->transitivity = 3.0 * (double)iv[4] / (double)iv[2];
        if (iv[5] > 0) out->avg_local_clustering = d[4] / (double)iv[5];
    }
    if (triangles && iv[4] < 0 && n > 0)
        return fail(RHG_EINVAL, "rhg_graph_stats: triangles need ascending rows (rhg_sort_rows)");
    return RHG_OK;
}

size_t rhg_long_range_workspace_bytes(int64_t n, int64_t k)
{
    if (n < 0 || k < 0 || k > (INT32_MAX - 4096) / 2) return 0;
    return lr_workspace_bytes(n, k);
}

rhg_status rhg_long_range(int64_t n, const int64_t *row_ptr, const int32_t *col_idx, int64_t nnz, int64_t k,
                          uint64_t seed, void *workspace, size_t workspace_bytes, int64_t *row_ptr_out,
                          int32_t *col_out, int64_t col_out_capacity, int64_t *added, void *stream)
{
    g_last_error.clear();
    if (n < 0 || n > (int64_t)INT32_MAX || nnz < 0) return fail(RHG_EINVAL, "rhg_long_range: bad n or nnz");
    if (k < 0 || k > (INT32_MAX - 4096) / 2) return fail(RHG_EINVAL, "rhg_long_range: k out of range");
    if (!row_ptr || !row_ptr_out || !added || !workspace || (nnz > 0 && !col_idx) ||
        (nnz + 2 * k > 0 && !col_out))
        return fail(RHG_EINVAL, "rhg_long_range: NULL argument");
    if (col_out_capacity < nnz + 2 * k)
        return fail(RHG_ECAPACITY, "rhg_long_range: col_out holds " + std::to_string(col_out_capacity) +
                                       " entries, nnz + 2k = " + std::to_string(nnz + 2 * k));
    if (workspace_bytes < lr_workspace_bytes(n, k))
        return fail(RHG_ECAPACITY, "rhg_long_range: workspace smaller than rhg_long_range_workspace_bytes");
    RHG_HIP(launch_long_range(n, row_ptr, col_idx, nnz, k, seed, workspace, row_ptr_out, col_out, added,
                              (hipStream_t)stream));
    return RHG_OK;
}

rhg_status rhg_index_stats(rhg_index *idx, rhg_stats *out, void *stream)
{
    g_last_error.clear();
    if (!idx || !out) return fail(RHG_EINVAL, "rhg_index_stats: NULL argument");
    unsigned long long h[ST_COUNT];
    hipStream_t s = (hipStream_t)stream;
    RHG_HIP(hipMemcpyAsync(h, idx->stats, sizeof(h), hipMemcpyDeviceToHost, s));
    RHG_HIP(hipStreamSynchronize(s));
    out->fp32_undecided = (int64_t)h[ST_FP32_UNDECIDED];
    out->dd_fallbacks = (int64_t)h[ST_DD];
    out->ties = (int64_t)h[ST_TIES];
    out->register_streams = (int64_t)h[ST_REG_STREAMS];
    out->temp_candidates = (int64_t)h[ST_TEMP_CAND];
    out->temp_coins = (int64_t)h[ST_TEMP_COINS];
    // the last count pass's per-wavefront tallies (zero before any count pass)
    out->swept = out->tests = 0;
    if (idx->counted && idx->n > 0) {
        const size_t nw = (size_t)(idx->n + 63) / 64;
        std::vector<long long> w(2 * nw);
        RHG_HIP(hipMemcpyAsync(w.data(), idx->wstat, nw * 16, hipMemcpyDeviceToHost, s));
        RHG_HIP(hipStreamSynchronize(s));
        for (size_t i = 0; i < nw; ++i) {
            out->tests += w[2 * i];
            out->swept += w[2 * i + 1];
        }
    }
    // the staged count's overflow flags, one byte per wavefront
    out->staged_waves = out->stage_overflows = 0;
    if (idx->staged_count && idx->n > 0) {
        const size_t nw = (size_t)(idx->n + 63) / 64;
        std::vector<uint8_t> f(nw);
        int32_t hend = 0;
        RHG_HIP(hipMemcpyAsync(f.data(), idx->sovf, nw, hipMemcpyDeviceToHost, s));
        RHG_HIP(hipMemcpyAsync(&hend, idx->heavy_end, sizeof(hend), hipMemcpyDeviceToHost, s));
        RHG_HIP(hipStreamSynchronize(s));
        for (size_t i = 0; i < nw; ++i) out->stage_overflows += f[i] != 0;
        out->staged_waves = (int64_t)nw - (int64_t)std::max(hend, 0) / 64;
    }
    if (h[ST_EMIT_MISMATCH]) return fail(RHG_EINTERNAL, "emit pass disagreed with the count pass");
    return RHG_OK;
}

void rhg_index_free(rhg_index *idx) { delete idx; }

rhg_status rhg_generate_async(const rhg_params *p, const rhg_tuning *t, double *r, double *theta, void *workspace,
                              size_t workspace_bytes, int64_t *row_ptr, int32_t *col_idx, int64_t col_capacity,
                              int32_t *overflow, void *stream)
{
    g_last_error.clear();
    rhg_status st = check_params(p, "rhg_generate_async");
    if (st != RHG_OK) return st;
    if (!row_ptr || !overflow || col_capacity < 0 || (col_capacity > 0 && !col_idx))
        return fail(RHG_EINVAL, "rhg_generate_async: NULL buffer or negative capacity");
    hipStream_t s = (hipStream_t)stream;
    if ((st = rhg_sample_points(p, r, theta, stream)) != RHG_OK) return st;
    rhg_index *idx = nullptr;
    if ((st = rhg_build_index(p, r, theta, t, workspace, workspace_bytes, 0, &idx, stream)) != RHG_OK) return st;
    if ((st = rhg_count_edges(idx, row_ptr, stream)) != RHG_OK) { rhg_index_free(idx); return st; }
    {
        const hipError_t e = launch_search(idx, row_ptr, col_idx, 1, s, col_capacity, overflow);
        if (e != hipSuccess) { rhg_index_free(idx); return check_hip(e, "rhg_generate_async (emit)"); }
    }
    rhg_index_free(idx);  // the launches hold their arguments by value
    return RHG_OK;
}

// The index workspace of rhg_generate_async_noalloc: one array per GPU
// (each device holds its own copy at its own address), held until the
// process ends.  Host code takes its address from hipGetSymbolAddress, once
// per device, and passes that pointer on; the array's name is no device
// address in host code.
static __device__ __align__(256) unsigned char g_noalloc_scratch[RHG_NOALLOC_SCRATCH_BYTES];
static std::mutex g_noalloc_mu;
static void *g_noalloc_ptr[256];

rhg_status rhg_generate_async_noalloc(const rhg_params *p, const rhg_tuning *t, double *r, double *theta,
                                      int64_t *row_ptr, int32_t *col_idx, int64_t col_capacity, int32_t *overflow,
                                      void *stream)
{
    g_last_error.clear();
    rhg_status st = check_params(p, "rhg_generate_async_noalloc");
    if (st != RHG_OK) return st;
    // no staging area in the library's array: the emit pass searches again
    rhg_tuning tt;
    memset(&tt, 0, sizeof(tt));
    if (t) tt = *t;
    tt.stage = -1;
    t = &tt;
    const size_t need = rhg_index_workspace_bytes(p, t);
    if (need > RHG_NOALLOC_SCRATCH_BYTES)
        return fail(RHG_ECAPACITY, "rhg_generate_async_noalloc: the index needs " + std::to_string(need) +
                                       " bytes of workspace, the library's array holds " +
                                       std::to_string((unsigned long long)RHG_NOALLOC_SCRATCH_BYTES));
    int dev = 0;
    RHG_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 256) return fail(RHG_EDEVICE, "rhg_generate_async_noalloc: device index out of range");
    void *ws = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_noalloc_mu);
        if (!g_noalloc_ptr[dev]) {
            void *ptr = nullptr;
            const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(g_noalloc_scratch));
            if (e != hipSuccess || !ptr) return check_hip(e != hipSuccess ? e : hipErrorInvalidSymbol,
                                                          "rhg_generate_async_noalloc (hipGetSymbolAddress)");
            g_noalloc_ptr[dev] = ptr;
        }
        ws = g_noalloc_ptr[dev];
    }
    return rhg_generate_async(p, t, r, theta, ws, RHG_NOALLOC_SCRATCH_BYTES, row_ptr, col_idx, col_capacity, overflow,
                              stream);
}

struct rhg_batch {
    hipGraph_t graph;
    hipGraphExec_t exec;
    int count, streams;
    int small_count;           // graphs generated by the persistent small-graph launch
    void *small_table;         // device: their records
    unsigned int *small_head;  // device: the launch's work counter
    unsigned long long *small_stats;  // device: the decisions' counters (not reported)
};

rhg_status rhg_batch_create(int count, const rhg_params *ps, const rhg_tuning *ts, double *const *r,
                            double *const *theta, void *const *ws, const size_t *ws_bytes, int64_t *const *row_ptr,
                            int32_t *const *col, const int64_t *col_cap, int32_t *overflow, int n_streams,
                            rhg_batch **out)
{
    g_last_error.clear();
    if (!out || !ps || !r || !theta || !ws || !ws_bytes || !row_ptr || !col || !col_cap || !overflow)
        return fail(RHG_EINVAL, "rhg_batch_create: NULL argument");
    if (count < 1) return fail(RHG_EINVAL, "rhg_batch_create: a batch holds at least one graph");
    *out = nullptr;
    if (n_streams < 1) n_streams = 1;
    if (n_streams > 64) n_streams = 64;
    // longest-processing-time-first assignment of graphs to capture streams,
    // by expected work (points plus expected edges)
    std::vector<int> order(count), owner(count);
    std::vector<double> work(count), load(n_streams, 0.0);
    for (int g = 0; g < count; ++g) {
        order[g] = g;
        const double k = std::isnan(ps[g].avg_degree) ? 10.0 : ps[g].avg_degree;
        work[g] = (double)ps[g].n * (4.0 + k);
    }
    // the persistent small-graph launch takes the last stream: charge it
    // the small graphs' work
    if (n_streams > 1)
        for (int g = 0; g < count; ++g)
            if (ps[g].n >= 0 && ps[g].n <= RHG_SMALL_GRAPH) load[n_streams - 1] += work[g];
    std::sort(order.begin(), order.end(), [&](int a, int b) { return work[a] > work[b]; });
    for (int g : order) {
        if (ps[g].n >= 0 && ps[g].n <= RHG_SMALL_GRAPH) {
            owner[g] = n_streams - 1;
            continue;
        }
        int best = 0;
        for (int k = 1; k < n_streams; ++k)
            if (load[k] < load[best]) best = k;
        owner[g] = best;
        load[best] += work[g];
    }
    std::vector<hipStream_t> st(n_streams);
    std::vector<hipEvent_t> ev(n_streams + 1);
    hipStream_t origin;
    RHG_HIP(hipStreamCreateWithFlags(&origin, hipStreamNonBlocking));
    for (int k = 0; k < n_streams; ++k) RHG_HIP(hipStreamCreateWithFlags(&st[k], hipStreamNonBlocking));
    for (int k = 0; k <= n_streams; ++k) RHG_HIP(hipEventCreateWithFlags(&ev[k], hipEventDisableTiming));
    rhg_batch *b = new (std::nothrow) rhg_batch;
    if (!b) return fail(RHG_ENOMEM, "rhg_batch_create: host allocation failed");
    b->count = count;
    b->streams = n_streams;
    b->graph = nullptr;
    b->small_count = 0;
    b->small_table = nullptr;
    b->small_head = nullptr;
    b->small_stats = nullptr;
    rhg_status status = RHG_OK;
    // Small graphs (n <= RHG_SMALL_GRAPH): one persistent launch generates
    // them all, a workgroup per graph, instead of ~50 launches each.
    std::vector<char> small_host;
    std::vector<char> is_small(count, 0);
    {
        const size_t rb = small_graph_record_bytes();
        std::vector<int> small_ids;
        for (int g = 0; g < count; ++g)
            if (ps[g].n >= 0 && ps[g].n <= RHG_SMALL_GRAPH && check_params(&ps[g], "rhg_batch_create") == RHG_OK)
                small_ids.push_back(g);
        if (!small_ids.empty()) {
            hipError_t e = hipMalloc(&b->small_stats, ST_COUNT * 8);
            if (e == hipSuccess) e = hipMemset(b->small_stats, 0, ST_COUNT * 8);
            if (e == hipSuccess) e = hipMalloc((void **)&b->small_head, 16);
            if (e != hipSuccess) status = check_hip(e, "rhg_batch_create (small graphs)");
        }
        for (int g : small_ids) {
            if (status != RHG_OK) break;
            Layout L;
            make_layout(ps[g], ts ? &ts[g] : nullptr, &L);
            const size_t off = small_host.size();
            small_host.resize(off + rb);
            if (!make_small_graph(ps[g], L, r[g], theta[g], ws[g], ws_bytes[g], row_ptr[g], col[g], col_cap[g],
                                  overflow + g, b->small_stats, small_host.data() + off)) {
                status = fail(RHG_ECAPACITY, "rhg_batch_create: workspace of graph " + std::to_string(g) +
                                                 " smaller than rhg_index_workspace_bytes");
                break;
            }
            is_small[g] = 1;
            ++b->small_count;
        }
        if (status == RHG_OK && b->small_count) {
            hipError_t e = hipMalloc(&b->small_table, small_host.size());
            if (e == hipSuccess) e = hipMemcpy(b->small_table, small_host.data(), small_host.size(), hipMemcpyHostToDevice);
            if (e != hipSuccess) status = check_hip(e, "rhg_batch_create (small graphs)");
        }
        if (status != RHG_OK) {
            if (b->small_table) (void)hipFree(b->small_table);
            if (b->small_head) (void)hipFree(b->small_head);
            if (b->small_stats) (void)hipFree(b->small_stats);
            for (int k = 0; k <= n_streams; ++k) (void)hipEventDestroy(ev[k]);
            for (int k = 0; k < n_streams; ++k) (void)hipStreamDestroy(st[k]);
            (void)hipStreamDestroy(origin);
            delete b;
            return status;
        }
    }
    const int prof = g_prof_on;
    g_prof_on = 0;  // no event records inside the captured graph
    hipError_t e = hipStreamBeginCapture(origin, hipStreamCaptureModeRelaxed);
    if (e == hipSuccess) {
        (void)hipEventRecord(ev[n_streams], origin);
        for (int k = 0; k < n_streams; ++k) (void)hipStreamWaitEvent(st[k], ev[n_streams], 0);
        // the persistent launch of the small graphs on a stream of its own
        // (the least loaded one), beside the large graphs' pipelines
        if (b->small_count) {
            const hipError_t e2 = launch_small_batch(b->small_table, b->small_count, b->small_head, st[n_streams - 1]);
            if (e2 != hipSuccess) status = check_hip(e2, "rhg_batch_create (small graphs)");
        }
        for (int g : order) {
            if (status != RHG_OK) break;
            if (is_small[g]) continue;
            status = rhg_generate_async(&ps[g], ts ? &ts[g] : nullptr, r[g], theta[g], ws[g], ws_bytes[g], row_ptr[g],
                                        col[g], col_cap[g], overflow + g, st[owner[g]]);
        }
        for (int k = 0; k < n_streams; ++k) {
            (void)hipEventRecord(ev[k], st[k]);
            (void)hipStreamWaitEvent(origin, ev[k], 0);
        }
        hipGraph_t graph = nullptr;
        const hipError_t e2 = hipStreamEndCapture(origin, &graph);
        b->graph = graph;
        if (status == RHG_OK && e2 != hipSuccess) status = check_hip(e2, "rhg_batch_create (capture)");
        if (status == RHG_OK) {
            const hipError_t e3 = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
            if (e3 != hipSuccess) status = check_hip(e3, "rhg_batch_create (instantiate)");
        }
    } else {
        status = check_hip(e, "rhg_batch_create (begin capture)");
    }
    g_prof_on = prof;
    for (int k = 0; k <= n_streams; ++k) (void)hipEventDestroy(ev[k]);
    for (int k = 0; k < n_streams; ++k) (void)hipStreamDestroy(st[k]);
    (void)hipStreamDestroy(origin);
    if (status != RHG_OK) {
        if (b->graph) (void)hipGraphDestroy(b->graph);
        if (b->small_table) (void)hipFree(b->small_table);
        if (b->small_head) (void)hipFree(b->small_head);
        if (b->small_stats) (void)hipFree(b->small_stats);
        delete b;
        return status;
    }
    *out = b;
    return RHG_OK;
}

rhg_status rhg_batch_launch(rhg_batch *b, void *stream)
{
    g_last_error.clear();
    if (!b) return fail(RHG_EINVAL, "rhg_batch_launch: NULL batch");
    RHG_HIP(hipGraphLaunch(b->exec, (hipStream_t)stream));
    return RHG_OK;
}

void rhg_batch_destroy(rhg_batch *b)
{
    if (!b) return;
    (void)hipGraphExecDestroy(b->exec);
    (void)hipGraphDestroy(b->graph);
    if (b->small_table) (void)hipFree(b->small_table);
    if (b->small_head) (void)hipFree(b->small_head);
    if (b->small_stats) (void)hipFree(b->small_stats);
    delete b;
}

rhg_status rhg_generate(int64_t n, double avg_degree, double gamma, uint64_t seed, const rhg_tuning *t,
                        rhg_alloc_fn alloc, void *alloc_ctx, int canonical_rows, rhg_csr *out, void *stream)
{
    g_last_error.clear();
    if (!alloc || !out) return fail(RHG_EINVAL, "rhg_generate: NULL allocator or output");
    memset(out, 0, sizeof(*out));
    rhg_params p;
    rhg_status st = plan(n, avg_degree, gamma, seed, &p);
    if (st != RHG_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    const size_t N = (size_t)(n > 0 ? n : 1);
    double *r = (double *)alloc(N * 8, alloc_ctx);
    double *th = (double *)alloc(N * 8, alloc_ctx);
    int64_t *row_ptr = (int64_t *)alloc((size_t)(n + 1) * 8, alloc_ctx);
    const size_t wsb = rhg_index_workspace_bytes(&p, t);
    void *ws = alloc(wsb, alloc_ctx);
    if (!r || !th || !row_ptr || !ws) return fail(RHG_ENOMEM, "rhg_generate: allocation callback failed");
    if ((st = rhg_sample_points(&p, r, th, stream)) != RHG_OK) return st;
    rhg_index *idx = nullptr;
    if ((st = rhg_build_index(&p, r, th, t, ws, wsb, 0, &idx, stream)) != RHG_OK) return st;
    if ((st = rhg_count_edges(idx, row_ptr, stream)) != RHG_OK) { rhg_index_free(idx); return st; }
    int64_t nnz = 0;
    hipError_t e = hipMemcpyAsync(&nnz, row_ptr + n, 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) { rhg_index_free(idx); return check_hip(e, "rhg_generate (edge count)"); }
    int32_t *col = (int32_t *)alloc((size_t)(nnz > 0 ? nnz : 1) * 4, alloc_ctx);
    if (!col) { rhg_index_free(idx); return fail(RHG_ENOMEM, "rhg_generate: col_idx allocation failed"); }
    if ((st = rhg_emit_edges(idx, row_ptr, col, nnz, canonical_rows, stream)) != RHG_OK) {
        rhg_index_free(idx);
        return st;
    }
    // the emit pass's row-length check (one more 8-byte read)
    unsigned long long mismatch = 0;
    e = hipMemcpyAsync(&mismatch, idx->stats + ST_EMIT_MISMATCH, 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    rhg_index_free(idx);
    if (e != hipSuccess) return check_hip(e, "rhg_generate (consistency check)");
    if (mismatch) return fail(RHG_EINTERNAL, "rhg_generate: the emit pass disagreed with the count pass");
    out->n = n;
    out->nnz = nnz;
    out->row_ptr = row_ptr;
    out->col_idx = col;
    out->r = r;
    out->theta = th;
    out->params = p;
    return RHG_OK;
}

// ---------------------------------------------------------------- temperature

static rhg_status check_T(double T, const char *who)
{
    if (!(T > 0.0 && T < 1.0)) return fail(RHG_EINVAL, std::string(who) + ": temperature must lie in (0, 1)");
    return RHG_OK;
}

rhg_status rhg_temp_count_edges(rhg_index *idx, double T, int64_t *row_ptr, void *stream)
{
    g_last_error.clear();
    if (!idx || !row_ptr) return fail(RHG_EINVAL, "rhg_temp_count_edges: NULL argument");
    rhg_status st = check_T(T, "rhg_temp_count_edges");
    if (st != RHG_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    RHG_HIP(launch_temp_search(idx, T, row_ptr, nullptr, 0, s, -1));
    idx->counted = 0;  // the per-wavefront tallies are the threshold search's
    idx->count_model = 2;
    idx->count_T = T;
    if (idx->n > 0) {
        PhaseScope ps(RHG_PHASE_SCAN, s);
        RHG_HIP(inclusive_scan_i64(row_ptr + 1, idx->n, idx->tmp, s));
    }
    return RHG_OK;
}

rhg_status rhg_temp_emit_edges(rhg_index *idx, double T, const int64_t *row_ptr, int32_t *col_idx,
                               int64_t col_capacity, int canonical_rows, void *stream)
{
    g_last_error.clear();
    if (!idx || !row_ptr) return fail(RHG_EINVAL, "rhg_temp_emit_edges: NULL argument");
    rhg_status st = check_T(T, "rhg_temp_emit_edges");
    if (st != RHG_OK) return st;
    if (col_capacity < 0) return fail(RHG_EINVAL, "rhg_temp_emit_edges: negative capacity");
    if (idx->count_model != 2 || idx->count_T != T)
        return fail(RHG_EINVAL, "rhg_temp_emit_edges: the index's last count pass was not rhg_temp_count_edges "
                                "at this temperature");
    hipStream_t s = (hipStream_t)stream;
    int64_t nnz = 0;
    RHG_HIP(hipMemcpyAsync(&nnz, row_ptr + idx->n, 8, hipMemcpyDeviceToHost, s));
    RHG_HIP(hipStreamSynchronize(s));
    if (nnz > col_capacity)
        return fail(RHG_ECAPACITY, "rhg_temp_emit_edges: col_idx holds " + std::to_string(col_capacity) +
                                       " entries, the graph needs " + std::to_string(nnz));
    if (nnz > 0 && !col_idx) return fail(RHG_EINVAL, "rhg_temp_emit_edges: col_idx is NULL");
    if (canonical_rows && nnz > idx->rows_nnz_cap)
        return fail(RHG_ECAPACITY, "rhg_temp_emit_edges: canonical rows of " + std::to_string(nnz) +
                                       " entries (over twice the threshold model's expected count) need "
                                       "rhg_sort_rows");
    if (nnz > 0) RHG_HIP(launch_temp_search(idx, T, (int64_t *)row_ptr, col_idx, 1, s, col_capacity));
    if (nnz > 0 && canonical_rows) {
        PhaseScope ps(RHG_PHASE_ROWS, s);
        RHG_HIP(launch_sort_rows(row_ptr, col_idx, idx->n, std::min<int64_t>(nnz, idx->n - 1), idx->rows_aux,
                                 idx->rows_lcap, idx->rows_mapcap, s));
    }
    return RHG_OK;
}

rhg_status rhg_temp_generate(int64_t n, double avg_degree, double gamma, double T, uint64_t seed,
                             const rhg_tuning *t, rhg_alloc_fn alloc, void *alloc_ctx, int canonical_rows,
                             rhg_csr *out, void *stream)
{
    g_last_error.clear();
    if (!alloc || !out) return fail(RHG_EINVAL, "rhg_temp_generate: NULL allocator or output");
    memset(out, 0, sizeof(*out));
    rhg_status st = check_T(T, "rhg_temp_generate");
    if (st != RHG_OK) return st;
    rhg_params p;
    if ((st = plan(n, avg_degree, gamma, seed, &p)) != RHG_OK) return st;
    // the temperature search's windows (radius R + 2T ln(2^53 - 1)) are
    // computed at each band's inner edge, so narrower bands than the
    // threshold search's test fewer candidates outside them
    rhg_tuning tt;
    memset(&tt, 0, sizeof(tt));
    if (t) tt = *t;
    if (!(tt.band_width > 0.0)) tt.band_width = RHG_TEMP_BAND_WIDTH;
    t = &tt;
    hipStream_t s = (hipStream_t)stream;
    const size_t N = (size_t)(n > 0 ? n : 1);
    double *r = (double *)alloc(N * 8, alloc_ctx);
    double *th = (double *)alloc(N * 8, alloc_ctx);
    int64_t *row_ptr = (int64_t *)alloc((size_t)(n + 1) * 8, alloc_ctx);
    const size_t wsb = rhg_index_workspace_bytes(&p, t);
    void *ws = alloc(wsb, alloc_ctx);
    if (!r || !th || !row_ptr || !ws) return fail(RHG_ENOMEM, "rhg_temp_generate: allocation callback failed");
    if ((st = rhg_sample_points(&p, r, th, stream)) != RHG_OK) return st;
    rhg_index *idx = nullptr;
    if ((st = rhg_build_index(&p, r, th, t, ws, wsb, 0, &idx, stream)) != RHG_OK) return st;
    if ((st = rhg_temp_count_edges(idx, T, row_ptr, stream)) != RHG_OK) { rhg_index_free(idx); return st; }
    int64_t nnz = 0;
    hipError_t e = hipMemcpyAsync(&nnz, row_ptr + n, 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) { rhg_index_free(idx); return check_hip(e, "rhg_temp_generate (edge count)"); }
    int32_t *col = (int32_t *)alloc((size_t)(nnz > 0 ? nnz : 1) * 4, alloc_ctx);
    if (!col) { rhg_index_free(idx); return fail(RHG_ENOMEM, "rhg_temp_generate: col_idx allocation failed"); }
    // canonical rows beyond the index's row-sort scratch: a workspace of their own
    const bool own_sort = canonical_rows && nnz > idx->rows_nnz_cap;
    if ((st = rhg_temp_emit_edges(idx, T, row_ptr, col, nnz, canonical_rows && !own_sort, stream)) != RHG_OK) {
        rhg_index_free(idx);
        return st;
    }
    unsigned long long mismatch = 0;
    e = hipMemcpyAsync(&mismatch, idx->stats + ST_EMIT_MISMATCH, 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    rhg_index_free(idx);
    if (e != hipSuccess) return check_hip(e, "rhg_temp_generate (consistency check)");
    if (mismatch) return fail(RHG_EINTERNAL, "rhg_temp_generate: the emit pass disagreed with the count pass");
    if (own_sort) {
        const size_t sb = rhg_sort_rows_workspace_bytes(n, nnz);
        void *sw = alloc(sb, alloc_ctx);
        if (!sw) return fail(RHG_ENOMEM, "rhg_temp_generate: row-sort workspace allocation failed");
        if ((st = rhg_sort_rows(n, row_ptr, col, nnz, sw, sb, stream)) != RHG_OK) return st;
    }
    out->n = n;
    out->nnz = nnz;
    out->row_ptr = row_ptr;
    out->col_idx = col;
    out->r = r;
    out->theta = th;
    out->params = p;
    return RHG_OK;
}

}  // extern "C"
