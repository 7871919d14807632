// rhg_internal.h -- declarations shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>

#include "../../include/rhg.h"
#include "rhg_dd.h"

#define RHG_MAX_BANDS 64
#define RHG_TWO_PI_D 6.283185307179586
#define RHG_TWO_PI_RES_D 2.4492935982947064e-16
#define RHG_HEAVY_CHUNK 8192      // candidates per heavy chunk (at least)
#define RHG_HEAVY_BLOCKS 2048     // workgroups striding over the heavy chunks
#define RHG_HEAVY_EXTRA_CHUNKS (1 << 20)
#define RHG_KAP_SUB 4             // sub-intervals per band of the entry estimate
#define RHG_ROWS_TILE 8192        // LDS tile (entries) of the row sort
#define RHG_SMALL_GRAPH 16384     // a batch's graphs of at most this many points share one persistent launch
#define RHG_TEMP_BAND_WIDTH 0.7   // rhg_temp_generate's default band width

namespace rhg {

// Sets the thread's last-error message and returns the status.
rhg_status fail(rhg_status s, const std::string &msg);
rhg_status check_hip(hipError_t e, const char *what);

#define RHG_HIP(call)                                              \
    do {                                                           \
        hipError_t e_ = (call);                                    \
        if (e_ != hipSuccess) return ::rhg::check_hip(e_, #call); \
    } while (0)

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Radial band layout: band j holds the points with E[j] <= r < E[j+1]
// (E[0] = 0, E[B] = R, and the last band also takes r = R).  Inside a band
// the points are sorted by angle and the angular range [0, 2 pi) is cut into
// 2^cbits[j] equal cells, the polar-quadtree leaves of that band.
struct Layout {
    int B;
    int band_bits;                    // bits of the sort key holding the band
    double E[RHG_MAX_BANDS + 1];      // band edges
    int cbits[RHG_MAX_BANDS];         // log2 of the cell count per band
    int64_t dir_base[RHG_MAX_BANDS + 1];  // offset of band j's directory
    int64_t dir_total;                // entries of the directory (all bands)
    int heavy_band;                   // bands [0, heavy_band) hold the heavy queries
    int64_t heavy_cap;                // at most this many heavy queries
    double entries_est;               // upper estimate of the graph's entries (2m)
    int fp64_only;                    // no FP32 screen
    int no_stream_stage;              // per-query streams never staged in LDS
    int sweep_max;                    // unions of at most this many candidates are swept
    int sweep_linear;                 // swept chunks filtered candidate by candidate
    int exact_inline;                 // undecided pairs decided inside the search kernels
    int64_t defer_cap;                // capacity of the undecided-pair list
    int64_t hset_slots;               // slots of the resolved-edge set (a power of two >= 2 defer_cap)
    int staged;                       // the count pass stages the light rows (the emit pass copies them)
    float lmu_in[RHG_MAX_BANDS];      // staging slots: log2 of the expected degree at band j's edges
    float lmu_out[RHG_MAX_BANDS];     //   (raised to bound the curve between them)
    float stage_f;                    // staging slots: stage_pct / 100
    int64_t stage_cap;                // staging words the workspace holds
};

// Expected degree of a point at radius r (threshold model): the other n - 1
// points are within R when r' <= R - r, and otherwise with probability
// theta_max(r, r') / pi, cos theta_max = (cosh r cosh r' - cosh R) /
// (sinh r sinh r'), r' drawn from the radial density of Eq. (1).  Composite
// 8-point Gauss-Legendre quadrature over 16 panels of [max(0, R - r), R].
// Used only to size the canonical-row workspace.
#define RHG_KAP_NODES 128  // 16 panels x 8 Gauss-Legendre nodes

// Contribution of quadrature node `node` (0 .. RHG_KAP_NODES-1) to the
// probability part of the expected degree at radius r (r > 0, R - r < R).
RHG_HD double degree_node(double alpha, double R, double r, int node)
{
    const double xg[4] = {0.1834346424956498, 0.5255324099163290, 0.7966664774136267, 0.9602898564975363};
    const double wg[4] = {0.3626837833783620, 0.3137066458778873, 0.2223810344533745, 0.1012285362903763};
    const double den = cosh(alpha * R) - 1.0;
    const double lo = fmax(0.0, R - r);
    const double h = (R - lo) / 16.0;
    const int k = node >> 3, g = node & 7;
    const double mid = lo + (k + 0.5) * h;
    const double x = mid + ((g & 1) ? 0.5 : -0.5) * h * xg[g >> 1];
    const double c = (cosh(r) * cosh(x) - cosh(R)) / (sinh(r) * sinh(x));
    const double th = acos(fmin(1.0, fmax(-1.0, c)));
    return 0.5 * h * wg[g >> 1] * (alpha * sinh(alpha * x) / den) * (th / 3.141592653589793);
}

// The part of partners within R - r of the centre (always neighbours).
RHG_HD double degree_inner(double alpha, double R, double r)
{
    return (cosh(alpha * fmax(0.0, R - r)) - 1.0) / (cosh(alpha * R) - 1.0);
}

RHG_HD double expected_degree(double n, double alpha, double R, double r)
{
    double tot = degree_inner(alpha, R, r);
    if (r > 0.0)
        for (int q = 0; q < RHG_KAP_NODES; ++q) tot += degree_node(alpha, R, r, q);
    return (n - 1.0) * fmin(1.0, tot);
}

void make_layout(const rhg_params &p, const rhg_tuning *t, Layout *L);

// Timed phases (rhg_phase_times).
enum { RHG_PHASE_SAMPLE = 0, RHG_PHASE_SORT = 1, RHG_PHASE_INDEX = 2, RHG_PHASE_GATHER = 3,
       RHG_PHASE_PLAN = 4, RHG_PHASE_COUNT_PASS = 5, RHG_PHASE_SCAN = 6, RHG_PHASE_EMIT_PASS = 7,
       RHG_PHASE_ROWS = 8, RHG_PHASE_COUNT = 9 };

// Brackets a phase with HIP events on stream s when profiling is on.
void *phase_begin(int phase, hipStream_t s);
void phase_end(void *rec, hipStream_t s);
struct PhaseScope {
    void *rec;
    hipStream_t s;
    PhaseScope(int phase, hipStream_t st) : rec(phase_begin(phase, st)), s(st) {}
    void end()
    {
        phase_end(rec, s);
        rec = nullptr;
    }
    ~PhaseScope() { end(); }
};

// Device-side counters (one 64-bit word each).
enum { ST_FP32_UNDECIDED = 0, ST_DD = 1, ST_TIES = 2, ST_BAD_INPUT = 3, ST_EMIT_MISMATCH = 4,
       ST_REG_STREAMS = 5, ST_TEMP_CAND = 6, ST_TEMP_COINS = 7, ST_COUNT = 8 };

}  // namespace rhg

// The index handle: host copies of the layout plus device pointers carved
// out of the caller's workspace.
struct rhg_index {
    rhg_params p;
    rhg::Layout L;
    int64_t n;
    uint32_t *keys;        // sorted keys (n)
    uint32_t *ids;         // sorted ids (n): the sort's values, equal to the record's id bits
    int32_t *band_start;   // B + 1 sorted positions
    int32_t *dir;          // directory, dir_total entries
    double *sr, *st;       // sorted r, theta (n each)
    float4 *rec;           // sorted (e^r, e^-r, sinh r) normalised by cosh R, and the id (n)
    int32_t *heavy_end;    // first light position (device scalar)
    int64_t *hplan;        // heavy_cap * B items: candidates, chunks, prefix of chunks
    int64_t *hcnt;         // max_chunks heavy chunks: counts, then their prefix
    int32_t *hitem;        // max_chunks heavy chunks: the item of each
    int64_t *hscal;        // heavy plan scalars
    int64_t heavy_cap;
    int64_t max_chunks;
    double2 *rt;           // (r, theta) interleaved in sample order, for the gather
    unsigned long long *stats;  // ST_COUNT counters
    void *wstat;           // per light wavefront of the last count pass: (tests, candidates swept)
    int counted;           // a count pass has run on this index
    int count_model;       // the model of the last count pass: 0 none, 1 threshold, 2 temperature
    double count_T;        // its temperature (model 2)
    uint64_t *dkeys;       // undecided-pair list (defer_cap): packed sorted positions
    int32_t *dchunk;       // its heavy chunk, or -1
    unsigned long long *dcount;  // [0] pairs listed, [1] overflow flag
    uint64_t *hset;        // resolved edges (hset_slots)
    int64_t *dslot;        // staged count: the listed pair's staging entry (-1: none)
    int32_t *stage;        // staged count: the light rows, one slot per light sorted position
    uint32_t *sslot;       // staged count: per id, the slot's start / 4 + 1 (0: heavy, ~0: none)
    uint8_t *sovf;         // staged count: per light wavefront, a row outgrew its slot
    int64_t *wsum;         // staged count: per wavefront, the inclusive prefix of its slots' words
    int staged_count;      // the last count pass staged its rows
    int64_t hset_slots;
    void *rows_aux;        // row sort: counters, long-row list, tile map
    int64_t rows_lcap;     // long rows the list holds
    int64_t rows_mapcap;   // tiles the map holds
    int64_t rows_nnz_cap;  // canonical rows are sorted here for graphs of up to this many entries
    void *tmp;             // scratch for sort and scan
    size_t tmp_bytes;
};

namespace rhg {

// ---- kernels launched from the C API (defined in the .hip files) ----
hipError_t launch_sample(const rhg_params &p, double *r, double *theta, hipStream_t s);

// LSD radix sort of (key, value) pairs on the low `bits` bits of the keys.
// Buffers k0/v0 hold the input; the sorted output ends in k0/v0.
size_t radix_sort_tmp_bytes(int64_t n);
hipError_t radix_sort_pairs(uint32_t *k0, uint32_t *v0, uint32_t *k1, uint32_t *v1, int64_t n,
                            int bits, void *tmp, hipStream_t s);

// In-place inclusive scan of int64 x[0..n).
size_t scan_tmp_bytes(int64_t n);
hipError_t inclusive_scan_i64(int64_t *x, int64_t n, void *tmp, hipStream_t s);

hipError_t launch_build_index(rhg_index *idx, const double *r, const double *theta, uint32_t *k1,
                              uint32_t *v0, uint32_t *v1, int validate, hipStream_t s);
// Band starts and cell directory of the index's sorted keys (part of the build).
hipError_t launch_index_directory(rhg_index *idx, hipStream_t s);
hipError_t launch_search(rhg_index *idx, int64_t *row_ptr, int32_t *col_idx, int emit, hipStream_t s,
                         int64_t col_cap = -1, int32_t *overflow = nullptr);
// The rows of the vertices at sorted positions qpos[0..k) on the index:
// their lengths into cnt (emit = 0), or the rows into ocol[optr[i] ..).
hipError_t launch_query_rows(rhg_index *idx, const int32_t *qpos, int64_t k, int64_t *cnt, const int64_t *optr,
                             int32_t *ocol, int emit, hipStream_t s);
// The temperature model's count (emit = 0) or emit pass over the index.
// Staged counts (rhg_search.hip): slot starts and cleared overflow flags
// before the count, slot starts split off the degrees after it, and the
// emit pass's copy of the light rows.
hipError_t launch_stage_slots(rhg_index *idx, float scale, hipStream_t s);
hipError_t launch_stage_split(rhg_index *idx, int64_t *row_ptr, hipStream_t s);
hipError_t launch_stage_copy(rhg_index *idx, const int64_t *row_ptr, int32_t *col_idx, int64_t col_cap,
                             hipStream_t s);
hipError_t launch_temp_search(rhg_index *idx, double T, int64_t *row_ptr, int32_t *col_idx, int emit,
                              hipStream_t s, int64_t col_cap);

// The batch's small graphs: a device record per graph, filled on the host by
// make_small_graph (false: workspace too small), and one persistent launch
// over all of them (a device counter `head` hands out the graphs).
size_t small_graph_record_bytes();
bool make_small_graph(const rhg_params &p, const Layout &L, double *r, double *theta, void *ws, size_t ws_bytes,
                      int64_t *row_ptr, int32_t *col, int64_t col_cap, int32_t *overflow,
                      unsigned long long *stats, void *out);
hipError_t launch_small_batch(const void *table, int count, unsigned int *head, hipStream_t s);

// Row sort (ascending rows, in place).  aux: rows_aux_bytes(lcap, mapcap)
// bytes holding counters, up to lcap rows longer than RHG_ROWS_TILE and the
// map of up to mapcap of their tiles.  For a CSR of nnz entries,
// rows_long_bound(nnz) long rows and rows_tile_bound(nnz, lcap) tiles are
// enough.  maxlen_bound: no row is longer.
int64_t rows_long_bound(int64_t nnz);
int64_t rows_tile_bound(int64_t nnz, int64_t lcap);
size_t rows_aux_bytes(int64_t lcap, int64_t mapcap);
hipError_t launch_sort_rows(const int64_t *row_ptr, int32_t *col, int64_t n, int64_t maxlen_bound, void *aux,
                            int64_t lcap, int64_t mapcap, hipStream_t s);

// Graph statistics.  out_i: max degree, tail count, triads, unsorted flag,
// triangles (-1: not counted), vertices of degree >= 2, -, -, then the 33
// histogram bins; out_d: sum ln(d / (kmin - 1/2)) over the tail, sum d^2,
// sum d^3, sum over entries of d_u d_v, sum of local clustering.
// Synchronises.
size_t stats_workspace_bytes(int64_t n, int64_t nnz, int triangles);
hipError_t launch_graph_stats(int64_t n, const int64_t *rp, const int32_t *col, int64_t nnz, double kmin,
                              int triangles, void *workspace, double *out_d, int64_t *out_i, hipStream_t s);

// Long-range augmentation: k extra edges, workspace of lr_workspace_bytes.
size_t lr_workspace_bytes(int64_t n, int64_t k);
hipError_t launch_long_range(int64_t n, const int64_t *row_ptr, const int32_t *col, int64_t nnz, int64_t k,
                             uint64_t seed, void *workspace, int64_t *row_ptr_out, int32_t *col_out, int64_t *added,
                             hipStream_t s);

}  // namespace rhg
