/*
 * rhg.h -- C ABI of the MI355X random hyperbolic graph (RHG) generator.
 *
 * The model (von Looz, Meyerhenke, Prutkin, Staudt, "Fast generation of
 * complex networks with underlying hyperbolic geometry", Sec. 2.1): n points
 * in a hyperbolic disk of radius R, angles uniform, radii with density
 * alpha*sinh(alpha r)/(cosh(alpha R) - 1) (Eq. (1)); two points are joined
 * when their hyperbolic distance is at most R.  Algorithm 1 of the paper
 * takes (n, average degree, alpha) and returns G = (V, E).  This library
 * splits that algorithm into the calls below; rhg_generate chains them.
 *
 * Conventions shared by every call:
 *   - Device pointers are HIP device memory owned by the caller.  The
 *     library never frees caller memory.  Host pointers are marked "host".
 *   - `stream` is a hipStream_t (NULL = the default stream).  Calls are
 *     asynchronous on it unless stated otherwise.
 *   - Every call returns an rhg_status; on failure rhg_last_error() (per
 *     thread) describes it.  No C++ exception crosses this boundary.
 *   - Errors raised on the device (for example an invalid input value seen
 *     by a kernel) are reported by the next call that synchronises.
 *   - Vertex ids are 0 .. n-1.  Ids are int32, so n <= 2^31 - 1.  Edge
 *     counts and CSR offsets are int64.
 *
 * Edge rule.  Pair {i, j}, i != j, is an edge iff the exact hyperbolic
 * distance of the two binary64 points is <= R, where
 *     cosh d = cosh r_i cosh r_j - sinh r_i sinh r_j cos(theta_i - theta_j)
 * (native representation, Sec. 2.1; equal to the Poincare metric of Eq. (2)
 * on the points mapped by mapToPoincare, Appendix B.2).  The library decides
 * it exactly: an FP32 screen and an FP64 evaluation settle all pairs away
 * from the threshold, and the rare pairs within a relative 2^-30 of it are
 * re-evaluated in double-double arithmetic.  Pairs that even double-double
 * cannot separate from the threshold (relative 1e-26) are counted in
 * rhg_index_stats and resolved by the double-double comparison.
 */
#ifndef RHG_H
#define RHG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RHG_OK = 0,
    RHG_EINVAL = 1,     /* an argument is out of range or inconsistent       */
    RHG_ENOMEM = 2,     /* an allocation (callback or host) failed           */
    RHG_ECAPACITY = 3,  /* an output buffer is smaller than required         */
    RHG_EDEVICE = 4,    /* a HIP runtime call failed                         */
    RHG_ENOROOT = 5,    /* Eq. (22) has no radius for the requested degree   */
    RHG_EINTERNAL = 6,  /* a device-side consistency check failed            */
    RHG_EBUSY = 7       /* the object is still in use (a running request)    */
} rhg_status;

/* Parameters of one graph.  Filled by rhg_plan / rhg_plan_radius; the
 * derived fields are what the kernels use and are exposed for tests. */
typedef struct {
    int64_t n;             /* vertices                                        */
    double avg_degree;     /* target average degree (NaN if R was given)      */
    double gamma;          /* power-law exponent (NaN if alpha was given)     */
    uint64_t seed;         /* Philox4x32-10 key                               */
    double alpha;          /* (gamma - 1) / 2                                 */
    double R;              /* disk radius = distance threshold                */
    double cosh_R;         /* cosh(R) rounded to binary64                     */
    double cosh_R_lo;      /* cosh(R) - cosh_R (double-double tail)           */
    double cosh_aR_m1;     /* cosh(alpha R) - 1 rounded to binary64           */
    double cosh_aR_m1_lo;  /* its double-double tail                          */
} rhg_params;

/* Tuning of the index and search.  Zero fields mean "choose automatically".
 * The edge set never depends on the tuning; only speed and the order of
 * neighbours inside a CSR row do. */
typedef struct {
    double band_width;     /* radial width of the outer bands                 */
    double inner_radius;   /* radius below which all points share one band    */
    int32_t cell_target;   /* mean points per angular cell                    */
    int32_t heavy_points;  /* expected points searched one per workgroup      */
    int32_t sweep_max;     /* a wavefront's union window (all its queries'
                            * windows in one band) of at most this many
                            * candidates is read once and swept by every
                            * lane; 0: automatic (128); negative: swept only
                            * where the queries' windows overlap           */
    int32_t sweep_linear;  /* nonzero: lanes filter every candidate of a
                            * swept chunk instead of binary-searching their
                            * window's start (slower; same bytes out)       */
    int32_t fp64_only;     /* nonzero: no FP32 screen, every candidate is
                            * decided in binary64 (double-double near the
                            * threshold): the plain path, same edge set      */
    int32_t no_stream_stage; /* nonzero: a wavefront's per-query candidate
                            * streams are always read through registers one
                            * step ahead, never staged in LDS (the path the
                            * longest streams take); same bytes out         */
    int32_t exact_inline;  /* nonzero: pairs the FP32 screen leaves undecided
                            * are decided inside the search kernels instead
                            * of being listed for a separate exact pass;
                            * same bytes out                                */
    int32_t defer_cap;     /* capacity of that list (0: automatic,
                            * 65536 + n/1024); when the count pass finds
                            * more, both passes rerun with in-place
                            * decisions; same bytes out                     */
    int32_t stage;         /* 1: the count pass also writes each light
                            * query's row into a staging area of the index
                            * (a slot per query sized from its expected
                            * degree mu at its radius: mu + 5 sqrt(mu) + 8
                            * entries) and the emit pass copies the rows out
                            * instead of searching again (a wavefront with a
                            * row that outgrew its slot is searched again);
                            * -1: count and search again; 0: automatic
                            * (staged from n = 2^19).  Same bytes out; the
                            * workspace grows by the slots, about 4 (2m +
                            * 30n) bytes at mean degree 20 (26.5 GB instead
                            * of 6.4 GB at n = 1e8)                         */
    int32_t stage_pct;     /* slot size, percent of mu + 5 sqrt(mu) + 8
                            * (0: 100)                                      */
} rhg_tuning;

/* Device-side diagnostics of the count and emit passes over an index.  The
 * first three and register_streams are summed since the index was built
 * (rhg_build_index clears them); swept and tests are those of the most
 * recent count pass (0 before one). */
typedef struct {
    int64_t fp32_undecided;  /* pairs the FP32 screen passed to FP64          */
    int64_t dd_fallbacks;    /* pairs FP64 passed to double-double            */
    int64_t ties;            /* pairs double-double could not separate        */
    int64_t swept;           /* candidates the light queries' wavefronts read
                              * into swept chunks                             */
    int64_t tests;           /* pair tests of the light queries (the
                              * candidates inside a query's window)           */
    int64_t register_streams; /* per-query candidate streams (one per light
                              * wavefront and band) read through registers:
                              * those longer than 4096 entries, or all of
                              * them with no_stream_stage; the rest are
                              * staged in LDS                                 */
    int64_t temp_candidates; /* the last temperature count pass: pairs
                              * inside the windows of radius
                              * R + 2T ln(2^53 - 1) that were screened     */
    int64_t temp_coins;      /* the last temperature count pass: coins drawn
                              * (screened pairs closer than that radius)  */
    int64_t staged_waves;    /* the last threshold count pass, when staged:
                              * light wavefronts (64 sorted positions)       */
    int64_t stage_overflows; /* of those, wavefronts with a row longer than
                              * its slot (the emit pass searches them again) */
} rhg_stats;

typedef struct rhg_index rhg_index;  /* opaque, host-side handle */

/* ------------------------------------------------------------------ */
/* Planning (host only, synchronous, no device work).                  */
/* ------------------------------------------------------------------ */

/* alpha = (gamma - 1)/2 (Sec. 2.1: gamma = 2 alpha + 1 with curvature 1).
 * R is the smallest binary64 value on the decreasing branch of Eq. (22)
 * (Appendix B.1, "getTargetRadius"; Algorithm 1, first step) whose expected
 * degree is <= avg_degree, Eq. (22) being read with the middle term
 * (pi - 1) * zeta/alpha, zeta = 1, and evaluated in double-double.
 * Errors: RHG_EINVAL if n < 0 or n > 2^31 - 1, gamma <= 2 or NaN,
 * avg_degree <= 0 or NaN, or avg_degree >= n - 1 when n >= 2, or if the
 * solved R is 80 or more (the range of the search's FP32 records and of
 * the screen's error bound; every call taking rhg_params refuses it too);
 * RHG_ENOROOT if the target exceeds the peak of Eq. (22).
 * n = 0 or 1 is valid (R is then that of n = 2 and the graph is empty). */
rhg_status rhg_plan(int64_t n, double avg_degree, double gamma, uint64_t seed,
                    rhg_params *out /* host */);

/* Same with alpha and R given directly (0.5 < alpha, 0 < R < 80). */
rhg_status rhg_plan_radius(int64_t n, double alpha, double R, uint64_t seed,
                           rhg_params *out /* host */);

/* The radial band layout the index would use for these parameters and
 * tuning (NULL = automatic): the flat-array form of the polar quadtree's
 * rings (Sec. 3.1).  Band j holds E[j] <= r < E[j+1] (the last band also
 * r = R).  *bands receives B; edges (host, cap doubles) receives
 * E[0 .. min(B + 1, cap)).  Host only, no device work; for tests and tools
 * that place points on band edges.  Errors: RHG_EINVAL for NULL pointers
 * or invalid params. */
rhg_status rhg_layout_bands(const rhg_params *p /* host */, const rhg_tuning *t /* host, may be NULL */,
                            double *edges /* host */, int cap, int *bands /* host */);

/* ------------------------------------------------------------------ */
/* Sampling (Algorithm 1, angular and radial draws; Eq. (1)).          */
/* ------------------------------------------------------------------ */

/* Writes n points: theta[i] = fl(TWO_PI_D * u_theta(i)) in [0, 2 pi) and
 * r[i] = acosh(1 + u_r(i) (cosh(alpha R) - 1)) / alpha in [0, R], the inverse
 * of the radial CDF (Appendix C, cell probability with the full angle), where
 * (u_theta, u_r) are the two 53-bit uniforms of Philox4x32-10 with key
 * (seed_lo, seed_hi) and counter (i_lo, i_hi, 0, 0): words (x1:x0) >> 11 and
 * (x3:x2) >> 11 times 2^-53.  r and theta: device, n doubles each, SoA. */
rhg_status rhg_sample_points(const rhg_params *p /* host */, double *r, double *theta,
                             void *stream);

/* ------------------------------------------------------------------ */
/* Index: the polar quadtree of Sec. 3.1 rebuilt as a flat array of     */
/* radial bands, each sorted by angle, with an angular cell directory.  */
/* ------------------------------------------------------------------ */

/* Bytes of device workspace rhg_build_index needs for these parameters
 * and tuning (NULL = automatic).  Host only. */
size_t rhg_index_workspace_bytes(const rhg_params *p /* host */,
                                 const rhg_tuning *t /* host, may be NULL */);

/* Builds the index of n points (r, theta: device, n doubles each, read
 * during this call's stream work only).  workspace: device, at least
 * rhg_index_workspace_bytes bytes, must stay allocated and untouched until
 * rhg_index_free.  Inputs must satisfy 0 <= r <= R and 0 <= theta < 2 pi
 * (finite); validate != 0 checks this on the device and synchronises the
 * stream once (RHG_EINVAL on violation).  *out receives a host handle. */
rhg_status rhg_build_index(const rhg_params *p /* host */, const double *r,
                           const double *theta, const rhg_tuning *t /* host, may be NULL */,
                           void *workspace, size_t workspace_bytes, int validate,
                           rhg_index **out /* host */, void *stream);

/* ------------------------------------------------------------------ */
/* Count pass and scan (Algorithm 1, query loop, counting).            */
/* ------------------------------------------------------------------ */

/* Runs the neighbour search and writes the CSR row offsets: row_ptr[0] = 0,
 * row_ptr[i + 1] - row_ptr[i] = deg(i) (device, n + 1 int64); row_ptr[n] =
 * 2m.  Unstaged, nothing but the degrees is kept and the emit pass
 * searches again; staged (rhg_tuning.stage), the light rows also go to
 * their slots in the index's workspace for the emit pass to copy.
 * Asynchronous. */
rhg_status rhg_count_edges(rhg_index *idx, int64_t *row_ptr, void *stream);

/* ------------------------------------------------------------------ */
/* Emit pass (Algorithm 1, edge insertion for each query).             */
/* ------------------------------------------------------------------ */

/* Writes the neighbours of vertex i to col_idx[row_ptr[i] .. row_ptr[i+1])
 * (device, int32) by repeating the count pass's search in the same order,
 * or, after a staged count, by searching the heavy queries' chunks again
 * and copying the light rows from their slots (the same bytes either way).
 * row_ptr must be the output of rhg_count_edges on the same index.  Each
 * undirected edge appears in both rows; there are no self-loops.
 * canonical_rows = 0: rows are in search order, deterministic for a given
 * tuning.  canonical_rows = 1: every row is then sorted ascending
 * (rhg_sort_rows on the index's own scratch), so col_idx is the same bytes
 * for every tuning.  col_capacity is the number of int32 slots in col_idx;
 * the call reads row_ptr[n] back (one synchronisation) and returns
 * RHG_ECAPACITY if it exceeds col_capacity, or if canonical rows are asked
 * for a graph with more entries than the index's row-sort scratch was sized
 * for (twice the planner's upper estimate of 2m, plus 2^23; sort such a
 * graph with rhg_sort_rows instead).  The emit kernels check every row they
 * write against its count; a disagreement is RHG_EINTERNAL from the next
 * rhg_index_stats (rhg_generate checks it itself).  RHG_EINVAL if the
 * index's last count pass was not rhg_count_edges. */
rhg_status rhg_emit_edges(rhg_index *idx, const int64_t *row_ptr, int32_t *col_idx,
                          int64_t col_capacity, int canonical_rows, void *stream);

/* ------------------------------------------------------------------ */
/* Canonical rows.                                                     */
/* ------------------------------------------------------------------ */

/* Sorts every row of a CSR ascending, in place: the canonical layout of the
 * edge set of Prop. 2 (the pairs within distance R), identical for every
 * tuning.  row_ptr: device, n + 1 non-decreasing int64 offsets into col_idx;
 * col_idx: device int32 entries, compared as signed integers (equal entries
 * are allowed).  nnz must be at least row_ptr[n] - row_ptr[0]: it sizes the
 * list of rows longer than 8192 entries and the merge levels; with a smaller
 * value some long rows stay unsorted (no access leaves the rows).
 * workspace: device, rhg_sort_rows_workspace_bytes(n, nnz) bytes, scratch
 * only.  Asynchronous on `stream`, no allocation and no host synchronisation.
 * Errors: RHG_EINVAL for n < 0, n > 2^31 - 1, nnz < 0 or a NULL pointer
 * (nothing is needed when n or nnz is 0); RHG_ECAPACITY for a smaller
 * workspace. */
size_t rhg_sort_rows_workspace_bytes(int64_t n, int64_t nnz);
rhg_status rhg_sort_rows(int64_t n, const int64_t *row_ptr, int32_t *col_idx, int64_t nnz,
                         void *workspace, size_t workspace_bytes, void *stream);

/* ------------------------------------------------------------------ */
/* Long-range augmentation (RHG-LR).                                   */
/* ------------------------------------------------------------------ */

/* Adds k random edges to a graph, as the paper does to correct the
 * diameter of random hyperbolic graphs (0.5 % of the edges in its
 * experiment: Sec. 4.2; the RHG-LR row of the generator table, Sec. 4.3;
 * Appendix I).  Candidate j = 0, 1, 2, ... is the vertex pair
 * (floor(w0 n / 2^64), floor(w1 n / 2^64)) for the words w0 = (x1:x0),
 * w1 = (x3:x2) of the Philox4x32-10 block with counter (j_lo, j_hi, 1, 0)
 * and key (seed_lo, seed_hi).  A candidate is rejected if it is a self-loop,
 * an edge of the input, or a pair an earlier candidate gave; the first k
 * accepted pairs are added, drawing at most the candidates j < 2k + 4096
 * (so fewer than k are added only when over half of those pairs are
 * rejected, in very dense or tiny graphs).
 * Input: row_ptr (device, n + 1 int64, row_ptr[0] = 0), col_idx (device,
 * nnz = row_ptr[n] int32 entries, a simple symmetric graph in any row
 * order).  Output: row_ptr_out (device, n + 1), col_out (device,
 * col_out_capacity >= nnz + 2k int32 slots): every input row, unchanged,
 * followed by its added neighbours in the order their pairs were accepted;
 * *added (device int64) = the number of added edges.  workspace: device,
 * rhg_long_range_workspace_bytes(n, k) bytes (about 40 B per candidate
 * plus 48 B per added edge).  Asynchronous, no allocation.
 * Errors: RHG_EINVAL for n < 0, n > 2^31 - 1, nnz < 0, k < 0,
 * k > (2^31 - 4097) / 2 or a NULL pointer; RHG_ECAPACITY for a small
 * col_out or workspace. */
size_t rhg_long_range_workspace_bytes(int64_t n, int64_t k);
rhg_status rhg_long_range(int64_t n, const int64_t *row_ptr, const int32_t *col_idx, int64_t nnz, int64_t k,
                          uint64_t seed, void *workspace, size_t workspace_bytes, int64_t *row_ptr_out,
                          int32_t *col_out, int64_t col_out_capacity, int64_t *added, void *stream);

/* ------------------------------------------------------------------ */
/* Validation statistics (Sec. 4.1).                                   */
/* ------------------------------------------------------------------ */

typedef struct {
    int64_t n, nnz;
    int64_t max_degree;
    int64_t hist[33];            /* [0]: degree 0; [b]: degree in [2^(b-1), 2^b)  */
    double kmin;                 /* the power-law fit uses degrees >= kmin        */
    int64_t tail_count;          /* vertices of degree >= kmin                    */
    double gamma_mle;            /* 1 + tail / sum ln(d / (kmin - 1/2)); NaN if no tail */
    double assortativity;        /* degree correlation over edge ends; NaN if undefined */
    int64_t triads;              /* sum over vertices of d (d - 1) / 2            */
    int64_t triangles;           /* -1 when not counted                           */
    double transitivity;         /* 3 triangles / triads (NaN if not counted)     */
    double avg_local_clustering; /* mean of t(v) / C(d, 2) over degree >= 2       */
    int32_t ascending_rows;      /* 1 if every row is strictly ascending          */
    int32_t reserved;
} rhg_graph_summary;

/* Statistics of a simple symmetric CSR (row_ptr: device n + 1 int64 with
 * row_ptr[0] = 0, col_idx: device nnz = row_ptr[n] int32), the properties
 * the paper reports for generated graphs (Sec. 4.1): the degree histogram;
 * the power-law exponent of the degrees >= kmin by the usual discrete
 * maximum-likelihood approximation (Clauset, Shalizi and Newman, 2009);
 * degree assortativity (Newman, 2002) over both directions of every edge;
 * and, when `triangles` is set, the triangles, the clustering coefficient
 * as the fraction of closed triangles to triads, and the average local
 * clustering.  Triangles need ascending rows (canonical rows): otherwise
 * the other fields are filled and RHG_EINVAL is returned.  Floating-point
 * sums are reduced in a fixed order (the same result on every run).
 * workspace: device, rhg_graph_stats_workspace_bytes(n, nnz, triangles)
 * bytes (about 4n, plus 14 B per entry and 20n with triangles).
 * Synchronises; *out is host memory.
 * Errors: RHG_EINVAL for n < 0, n > 2^31 - 1, nnz < 0, kmin < 1 or a NULL
 * pointer; RHG_ECAPACITY for a small workspace. */
size_t rhg_graph_stats_workspace_bytes(int64_t n, int64_t nnz, int triangles);
rhg_status rhg_graph_stats(int64_t n, const int64_t *row_ptr, const int32_t *col_idx, int64_t nnz, double kmin,
                           int triangles, void *workspace, size_t workspace_bytes, rhg_graph_summary *out,
                           void *stream);

/* Diagnostics accumulated by the count and emit passes (synchronises). */
rhg_status rhg_index_stats(rhg_index *idx, rhg_stats *out /* host */, void *stream);

void rhg_index_free(rhg_index *idx);

/* ------------------------------------------------------------------ */
/* Whole generator (Algorithm 1).                                      */
/* ------------------------------------------------------------------ */

/* Device allocator supplied by the caller: returns `bytes` of device memory
 * (256-byte aligned) or NULL.  The memory must stay valid until the caller
 * releases it; the library never frees it. */
typedef void *(*rhg_alloc_fn)(size_t bytes, void *ctx);

typedef struct {
    int64_t n;
    int64_t nnz;        /* 2m: entries of col_idx                            */
    int64_t *row_ptr;   /* device, n + 1                                     */
    int32_t *col_idx;   /* device, nnz                                       */
    double *r;          /* device, n: the sampled radii                      */
    double *theta;      /* device, n: the sampled angles                     */
    rhg_params params;
} rhg_csr;

/* Plans, samples, indexes, counts, scans and emits one graph.  All device
 * memory (points, index workspace, CSR) comes from `alloc`; the host
 * synchronises for the 8-byte read of 2m before col_idx is allocated and
 * for the 8-byte read of the emit pass's row-length check at the end.
 * canonical_rows as for rhg_emit_edges.
 * Errors: those of rhg_plan, RHG_ENOMEM if `alloc` returns NULL, and
 * RHG_EINTERNAL if an emitted row's length disagrees with its count. */
rhg_status rhg_generate(int64_t n, double avg_degree, double gamma, uint64_t seed,
                        const rhg_tuning *t /* host, may be NULL */,
                        rhg_alloc_fn alloc, void *alloc_ctx, int canonical_rows,
                        rhg_csr *out /* host */, void *stream);

/* ------------------------------------------------------------------ */
/* Temperature model.                                                  */
/* ------------------------------------------------------------------ */

/* The more general model of Krioukov et al. that Sec. 2.1 mentions and sets
 * aside: a pair is joined with a probability that depends on its distance.
 * Read here as their Fermi-Dirac form with curvature 1,
 *     p(d) = 1 / (1 + e^{(d - R) / (2T)}),  temperature 0 < T < 1,
 * which tends to the threshold rule d <= R as T -> 0.  Pair {i, j} draws one
 * coin u = a 2^-53, a = k + 1 in [1, 2^53], k = the word (x1:x0) >> 11 of the
 * Philox4x32-10 block with key (seed_lo, seed_hi) of the index's params and
 * counter (min(i,j), max(i,j), 2, 0); the pair is an edge iff u < p(d),
 * decided exactly on the binary64 points and the coin (an FP32 screen,
 * binary64, then double-double; pairs that double-double cannot separate
 * within a relative 1e-26 are counted as ties in rhg_index_stats).  Only
 * pairs with d < R + 2T ln(2^53 - 1) can satisfy it (p(d) > 2^-53), so the
 * search covers exactly those.  The disk is the threshold model's: R comes
 * from the params as planned for the target degree (Eq. (22)), and at T > 0
 * the mean degree is larger (by about pi T / sin(pi T) for large n).
 *
 * rhg_temp_count_edges: as rhg_count_edges for this rule (row_ptr: device,
 * n + 1 int64, row_ptr[n] = 2m).  rhg_temp_emit_edges: as rhg_emit_edges;
 * row_ptr must come from rhg_temp_count_edges on the same index at the same
 * T with no other count pass in between (the two models share the index's
 * search scratch), else RHG_EINVAL.  Rows are in search order, or ascending
 * with canonical_rows = 1 (RHG_ECAPACITY if the graph has more entries than
 * the index's row-sort scratch, which is sized from the threshold model:
 * sort such a graph with rhg_sort_rows).  The innermost queries (the
 * tuning's heavy_points) are split over workgroups; at larger T a larger
 * heavy_points keeps the wider windows balanced.  On a staged index
 * (rhg_tuning.stage) the count pass also writes the light rows into the
 * staging slots, scaled by pi T' / sin(pi T') for T' = min(2T, 0.45), and
 * the emit pass copies them (rows beyond their slot searched again); the
 * same bytes out.  Same diagnostics and row-length check as the threshold
 * passes.
 * Errors: RHG_EINVAL for a NULL argument or T outside (0, 1) (or NaN).
 *
 * rhg_temp_generate: rhg_generate with this rule (plan, sample, index,
 * count, scan, emit; canonical rows beyond the index's scratch get a row-sort
 * workspace of their own from `alloc`).  A band_width of 0 (or a NULL
 * tuning) means 0.7 here: the windows are taken at each band's inner edge,
 * and narrower bands than the threshold search's default leave fewer
 * candidates outside them. */
rhg_status rhg_temp_count_edges(rhg_index *idx, double T, int64_t *row_ptr, void *stream);
rhg_status rhg_temp_emit_edges(rhg_index *idx, double T, const int64_t *row_ptr, int32_t *col_idx,
                               int64_t col_capacity, int canonical_rows, void *stream);
rhg_status rhg_temp_generate(int64_t n, double avg_degree, double gamma, double T, uint64_t seed,
                             const rhg_tuning *t /* host, may be NULL */, rhg_alloc_fn alloc, void *alloc_ctx,
                             int canonical_rows, rhg_csr *out /* host */, void *stream);

/* ------------------------------------------------------------------ */
/* Dynamic model: vertices move, the graph follows.                    */
/* ------------------------------------------------------------------ */

/* Sec. 5 notes that the incremental construction of the polar quadtree
 * admits a dynamic model with vertex movement (future work there).  Here a
 * state holds n points, their index and the threshold graph on them as a
 * CSR with ascending rows; each rhg_dyn_move applies a batch of moves (ids
 * with new coordinates) and leaves exactly the graph that generation from
 * scratch on the moved points gives (same edge rule and exactness as
 * rhg_count_edges), updating the index by a merge instead of a rebuild and
 * recomputing only the rows that change (the moved vertices' rows and the
 * rows that lose or gain a moved neighbour).  The movement itself is the
 * caller's: the paper fixes none.
 *
 * The state's device memory is the library's own (hipMalloc at creation,
 * grown when a step needs more, released by rhg_dyn_free); about
 * 100 B per point plus two CSR column buffers.
 *
 * rhg_dyn_create: p (host) as from rhg_plan / rhg_plan_radius with
 * 1 <= n <= 2^31 - 1; r, theta: device, n doubles each, copied (the caller
 * keeps them); 0 <= r <= R and 0 <= theta < 2 pi are checked (RHG_EINVAL).
 * Synchronises.  *out receives the state.
 *
 * rhg_dyn_move: k moves (0 <= k <= n; k = 0 does nothing): ids (device
 * int32, distinct, in [0, n)), r and theta (device doubles, the new
 * coordinates, 0 <= r <= R, 0 <= theta < 2 pi).  A batch that breaks these
 * rules is refused with RHG_EINVAL and leaves the state unchanged.  Runs on
 * `stream` and synchronises it a few times (to size the step's buffers).
 * Calls on one state must not overlap.  After a device error the state is
 * undefined.
 *
 * rhg_dyn_graph: the current graph (*out, host): device pointers to
 * row_ptr (n + 1), col_idx (nnz, ascending rows), r and theta (the current
 * points), and the params.  Valid until the next rhg_dyn_move or
 * rhg_dyn_free; the caller must not write through them.
 *
 * A batch with k (1 + mean degree) above share * n (share = 1/8 unless
 * rhg_dyn_set_regenerate_share says otherwise; 0: always) is applied by
 * regeneration instead (index rebuilt, both passes, rows sorted): same
 * graph, less work when most rows would change.
 *
 * rhg_dyn_last_step: rows rewritten by the last move (the changed unmoved
 * rows plus the k moved rows, or n after a regeneration) and entries of
 * the moved rows (or all entries). */
typedef struct rhg_dyn rhg_dyn;
rhg_status rhg_dyn_create(const rhg_params *p /* host */, const rhg_tuning *t /* host, may be NULL */,
                          const double *r, const double *theta, rhg_dyn **out /* host */, void *stream);
rhg_status rhg_dyn_move(rhg_dyn *d, int64_t k, const int32_t *ids, const double *r, const double *theta,
                        void *stream);
rhg_status rhg_dyn_graph(rhg_dyn *d, rhg_csr *out /* host */);
rhg_status rhg_dyn_set_regenerate_share(rhg_dyn *d, double share);
rhg_status rhg_dyn_last_step(rhg_dyn *d, int64_t *changed_rows /* host */, int64_t *moved_entries /* host */);
void rhg_dyn_free(rhg_dyn *d);

/* ------------------------------------------------------------------ */
/* Phase timing (HIP events on the caller's stream).                   */
/* ------------------------------------------------------------------ */

/* Turns event timing of the library's phases on (1) or off (0) and clears
 * the record ring (512 entries).  Turning it on creates the events once;
 * call it outside any timed region.  Process-wide, not thread-safe. */
rhg_status rhg_set_profiling(int on);

/* Average duration in ms and number of recorded launches of each phase
 * since profiling was last turned on (synchronises on the events).  Phases:
 * 0 sample, 1 keys+sort, 2 index (band starts + directory), 3 gather,
 * 4 plan (the small kernels around the searches: heavy-work plan, its
 * scans, heavy degrees, capacity check), 5 count (the search kernel of the
 * count pass), 6 scan (row offsets), 7 emit (the search kernel of the emit
 * pass), 8 rows (the row sort of canonical rows).  Each of 5 and 7 brackets
 * exactly one kernel launch.  avg_ms, count: host arrays of at least 9
 * entries (cap). */
rhg_status rhg_phase_times(double *avg_ms /* host */, int64_t *count /* host */, int cap);

/* Name of a phase index ("" if out of range). */
const char *rhg_phase_name(int phase);

/* ------------------------------------------------------------------ */
/* Batches: many graphs, one launch.                                   */
/* ------------------------------------------------------------------ */

/* The whole pipeline of one graph (sample, index, count, scan, emit) into
 * caller buffers, fully asynchronous on `stream`: no allocation, no host
 * synchronisation, no memset, so it can be captured into a HIP graph.
 * r, theta: n doubles; workspace: rhg_index_workspace_bytes(p, t) bytes;
 * row_ptr: n + 1 int64; col_idx: col_capacity int32 slots.  *overflow
 * (device int32) is set to 1 when 2m > col_capacity -- then row_ptr is
 * valid but col_idx is left unwritten, and the caller can emit again into a
 * buffer of row_ptr[n] slots -- and to 0 otherwise.  After the emit, bit 1
 * (value 2) is added when an emitted row's length disagreed with its count
 * (an internal error; the rows are then not to be trusted). */
rhg_status rhg_generate_async(const rhg_params *p /* host */, const rhg_tuning *t /* host, may be NULL */,
                              double *r, double *theta, void *workspace, size_t workspace_bytes,
                              int64_t *row_ptr, int32_t *col_idx, int64_t col_capacity,
                              int32_t *overflow, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * rhg_generate_async with the index workspace taken from the library's own
 * device array of RHG_NOALLOC_SCRATCH_BYTES bytes, one per GPU, held from
 * the library's first use of that GPU until the process ends.  The caller
 * still passes the points, the CSR and the overflow flag exactly as for
 * rhg_generate_async (same meaning, same results, bit for bit); the stream
 * must belong to the current device.  Allocates no device memory.  Every
 * call on one GPU uses the same array, so calls whose stream work overlaps
 * on a GPU race and must be ordered by the caller.
 * Errors: those of rhg_generate_async; RHG_ECAPACITY when
 * rhg_index_workspace_bytes(p, t) exceeds RHG_NOALLOC_SCRATCH_BYTES (about
 * n = 7e5 points); RHG_EDEVICE when the array's address cannot be read. */
#define RHG_NOALLOC_SCRATCH_BYTES (64ull << 20)
rhg_status rhg_generate_async_noalloc(const rhg_params *p /* host */, const rhg_tuning *t /* host, may be NULL */,
                                      double *r, double *theta, int64_t *row_ptr, int32_t *col_idx,
                                      int64_t col_capacity, int32_t *overflow, void *stream);

typedef struct rhg_batch rhg_batch;  /* opaque, host-side handle */

/* Captures rhg_generate_async for `count` graphs into one HIP graph (one
 * submission for the whole batch).  The graphs are spread over n_streams
 * capture streams (1..64), largest expected work first, so independent
 * graphs run concurrently.  All arrays are host arrays of `count` entries
 * (ts may be NULL; a zero field of ts[g] takes the default); the device
 * buffers they point to must stay allocated while the batch exists;
 * overflow: device, count int32 flags, flag g set on each launch to whether
 * graph g's 2m exceeded col_capacity[g] (its emit then writes nothing).
 * Errors: RHG_EINVAL for count < 1, a NULL array or any graph's invalid
 * arguments (no batch is created, *out stays NULL); RHG_EDEVICE if capture
 * or instantiation fails.  Creation allocates host objects and the
 * executable graph; it launches no work. */
rhg_status rhg_batch_create(int count, const rhg_params *ps, const rhg_tuning *ts, double *const *r,
                            double *const *theta, void *const *workspace, const size_t *workspace_bytes,
                            int64_t *const *row_ptr, int32_t *const *col_idx, const int64_t *col_capacity,
                            int32_t *overflow, int n_streams, rhg_batch **out /* host */);

/* Launches the captured batch on `stream` (asynchronous; replayable). */
rhg_status rhg_batch_launch(rhg_batch *b, void *stream);

void rhg_batch_destroy(rhg_batch *b);

/* ------------------------------------------------------------------ */
/* Serving: continuous batching of generation requests on one GPU.     */
/* ------------------------------------------------------------------ */

/* A request server.  Requests (n, avg_degree, gamma, seed; planned as in
 * rhg_plan) are queued first come, first served; the head is admitted as
 * soon as one of `slots` HIP streams is free and its device memory fits in
 * the server's arena beside what admitted and unreleased requests hold.
 * Each admitted request runs the whole pipeline of rhg_generate_async on its
 * own stream, so requests that arrive while others run overlap with them on
 * the device.  The arena (budget_bytes of device memory) is allocated once,
 * at creation, and handed out on the host: admission allocates nothing.  A
 * request holds (r, theta), row_ptr and col_idx slots for its target degree
 * times n (with a 1.3 slack) until it is released, and its index workspace
 * until it completes; a graph with more edges than its slots is run again
 * into exactly 2m slots before it completes.  The server is the natural
 * boundary of the paper's generator (Algorithm 1) put behind a request
 * queue; it is single-threaded: calls on one server must not overlap.
 * Errors (create): RHG_EINVAL for slots outside 1 .. 64 or a budget below
 * 1 MiB; RHG_ENOMEM when the arena cannot be allocated. */
typedef struct rhg_server rhg_server;  /* opaque, host-side handle */

typedef struct {
    int64_t req_id;
    rhg_status status;        /* RHG_OK, or the error that ended the request  */
    int32_t reserved;
    int64_t n;
    int64_t nnz;              /* 2m                                           */
    const int64_t *row_ptr;   /* device, n + 1 (valid until released)          */
    const int32_t *col_idx;   /* device, nnz                                   */
    const double *r;          /* device, n: the sampled points                 */
    const double *theta;
    double latency_ms;        /* from submission to completion seen by a poll  */
    rhg_params params;
} rhg_completion;

typedef struct {
    int64_t submitted, completed, failed, rejected, refills;
    int64_t edges;            /* undirected edges of the completed requests   */
    int64_t max_inflight, max_reserved_bytes;
    int64_t reserved_bytes, inflight, queued;  /* now                         */
} rhg_server_stats;

rhg_status rhg_server_create(size_t budget_bytes, int slots, rhg_server **out /* host */);

/* Plans and queues a request, then admits what fits.  req_id: the caller's
 * key (unique among unreleased requests).  Errors: those of rhg_plan;
 * RHG_EINVAL for an id in use; RHG_ECAPACITY when the request could not fit
 * even into the empty arena (it is not queued). */
rhg_status rhg_server_submit(rhg_server *s, int64_t req_id, int64_t n, double avg_degree, double gamma,
                             uint64_t seed, const rhg_tuning *t /* host, may be NULL */);

/* Collects the requests whose work has finished (by querying their events;
 * no blocking), admits queued requests into the freed slots and memory, and
 * writes up to cap completions to out (host) with their count in *count
 * (the rest come with the next polls). */
rhg_status rhg_server_poll(rhg_server *s, rhg_completion *out /* host */, int cap, int *count /* host */);

/* Returns a completed request's memory to the arena (or withdraws a queued
 * one).  Errors: RHG_EINVAL for an unknown id; RHG_EBUSY while it runs or
 * before a poll has handed out its completion. */
rhg_status rhg_server_release(rhg_server *s, int64_t req_id);

rhg_status rhg_server_get_stats(rhg_server *s, rhg_server_stats *out /* host */);

/* Waits for the server's streams and frees everything it holds. */
void rhg_server_destroy(rhg_server *s);

/* Message of the last failed call on this thread ("" if none). */
const char *rhg_last_error(void);

/* Library version string. */
const char *rhg_version(void);

#ifdef __cplusplus
}
#endif
#endif /* RHG_H */
