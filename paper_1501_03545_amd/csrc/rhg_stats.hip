// rhg_stats.hip -- validation statistics of a generated graph on the device
// (the properties of Sec. 4.1): the degree histogram and the power-law
// exponent of the degrees, degree assortativity, and the clustering
// coefficient as the fraction of closed triangles to triads (paths of
// length 2), with the triangles through every vertex for the average local
// clustering.
//
// Floating-point sums are reduced in a fixed order (per-block partials, then
// one block), so the results do not change from run to run.  Triangles are
// counted once each on the degree-oriented graph: every edge points from the
// lower to the higher (degree, id) rank, so each triangle {u, v, w} with
// u < v < w in rank is found once, at the edge u -> v, as the common
// out-neighbour w; out-degrees stay small even at the hubs.  Out-rows keep
// the order of the input rows, which must be ascending for the merge
// intersection.
#include "rhg_internal.h"

namespace rhg {

namespace {

constexpr int ST_TILE = 4096;      // entries per workgroup in the entry passes (256 threads x 16)
constexpr int ST_PER = 16;         // consecutive entries per thread
constexpr int ST_ROWS_CAP = 4096;  // rows staged in LDS per tile (more: binary search in global memory)
constexpr int ST_VBLOCK = 256;     // vertices per workgroup in the vertex passes

// Device results (one array of 8-byte words).
enum {
    SR_MAXDEG = 0, SR_TAIL = 1, SR_TRIADS = 2, SR_UNSORTED = 3, SR_TRIANGLES = 4, SR_KEPT = 5,
    SR_SUMLOG = 8, SR_SUMD2 = 9, SR_SUMD3 = 10, SR_SUMXY = 11, SR_LCC = 12, SR_LCC_N = 13,
    SR_HIST = 16, SR_WORDS = 16 + 33
};

__device__ __forceinline__ double block_sum_d(double x, double *lds)
{
    // fixed-order reduction over a workgroup of 256: wavefront tree, then
    // the four wavefront sums in order
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x += __shfl_down(x, d);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) lds[wv] = x;
    __syncthreads();
    const double s = ((lds[0] + lds[1]) + lds[2]) + lds[3];
    __syncthreads();
    return s;
}

__device__ __forceinline__ int64_t block_sum_i(int64_t x, int64_t *lds)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x += __shfl_down(x, d);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) lds[wv] = x;
    __syncthreads();
    const int64_t s = lds[0] + lds[1] + lds[2] + lds[3];
    __syncthreads();
    return s;
}

// Index of the last row starting at or before position p (rows [lo, hi)).
__device__ __forceinline__ int64_t row_of(const int64_t *rp, int64_t lo, int64_t hi, int64_t p)
{
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (rp[mid] <= p) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Calls f(e, u) for every entry e of this workgroup's tile [p0, p1) of a
// CSR (rp: n + 1 offsets), with u the row holding e.  Each thread takes 16
// consecutive entries; the rows spanning the tile are staged in LDS.
template <class F>
__device__ void for_tile_entries(const int64_t *__restrict__ rp, int64_t n, int64_t nnz, F f)
{
    __shared__ int64_t srp[ST_ROWS_CAP + 1];
    __shared__ int64_t su0, scnt;
    const int64_t p0 = (int64_t)blockIdx.x * ST_TILE;
    const int64_t p1 = min(nnz, p0 + ST_TILE);
    if (threadIdx.x == 0) {
        const int64_t u0 = row_of(rp, 0, n, p0);
        const int64_t u1 = row_of(rp, u0, n, p1 - 1);
        su0 = u0;
        scnt = u1 - u0 + 1;
    }
    __syncthreads();
    const int64_t u0 = su0, cnt = scnt;
    const bool staged = cnt + 1 <= ST_ROWS_CAP + 1;
    if (staged)
        for (int64_t i = threadIdx.x; i <= cnt; i += blockDim.x) srp[i] = rp[u0 + i];
    __syncthreads();
    const int64_t e0 = p0 + (int64_t)threadIdx.x * ST_PER;
    if (e0 < p1) {
        const int64_t e1 = min(p1, e0 + ST_PER);
        int64_t u, next;
        if (staged) {
            int64_t lo = 0, hi = cnt;
            while (hi - lo > 1) {
                const int64_t mid = (lo + hi) >> 1;
                if (srp[mid] <= e0) lo = mid;
                else hi = mid;
            }
            u = u0 + lo;
            next = srp[lo + 1];
        } else {
            u = row_of(rp, u0, u0 + cnt, e0);
            next = rp[u + 1];
        }
        for (int64_t e = e0; e < e1; ++e) {
            while (e >= next) {  // empty rows are skipped
                ++u;
                next = staged ? srp[u - u0 + 1] : rp[u + 1];
            }
            f(e, u);
        }
    }
    __syncthreads();
}

__global__ void __launch_bounds__(256) st_deg_kernel(int64_t n, const int64_t *__restrict__ rp, int32_t *__restrict__ deg)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) deg[v] = (int32_t)(rp[v + 1] - rp[v]);
}

// Histogram, maximum, power-law tail sums, triads, sums of d^2 and d^3.
__global__ void __launch_bounds__(256) st_vertex_kernel(int64_t n, const int32_t *__restrict__ deg, double kmin,
                                                        double *__restrict__ part, unsigned long long *__restrict__ res)
{
    __shared__ unsigned long long hist[33];
    __shared__ double ld[4];
    __shared__ int64_t li[4];
    if (threadIdx.x < 33) hist[threadIdx.x] = 0ull;
    __syncthreads();
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double slog = 0.0, d2 = 0.0, d3 = 0.0;
    int64_t tail = 0, triads = 0;
    int d = 0;
    if (v < n) {
        d = deg[v];
        const int b = d == 0 ? 0 : 32 - __clz((unsigned)d);  // degree in [2^(b-1), 2^b)
        atomicAdd(&hist[b], 1ull);
        const double x = (double)d;
        if (x >= kmin) {
            tail = 1;
            slog = log(x / (kmin - 0.5));
        }
        d2 = x * x;
        d3 = d2 * x;
        triads = (int64_t)d * (d - 1) / 2;
    }
    unsigned long long mx = (unsigned long long)d;
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) mx = max(mx, (unsigned long long)__shfl_down(mx, s));
    if ((threadIdx.x & 63) == 0) atomicMax(&res[SR_MAXDEG], mx);
    const double a = block_sum_d(slog, ld), b2 = block_sum_d(d2, ld), b3 = block_sum_d(d3, ld);
    const int64_t t = block_sum_i(tail, li), tr = block_sum_i(triads, li);
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x + 0] = a;
        part[3 * blockIdx.x + 1] = b2;
        part[3 * blockIdx.x + 2] = b3;
        atomicAdd(&res[SR_TAIL], (unsigned long long)t);
        atomicAdd(&res[SR_TRIADS], (unsigned long long)tr);
    }
    if (threadIdx.x < 33 && hist[threadIdx.x]) atomicAdd(&res[SR_HIST + threadIdx.x], hist[threadIdx.x]);
}

// Sum over entries of d_u d_v, and whether every row is strictly ascending.
__global__ void __launch_bounds__(256) st_edge_kernel(int64_t n, int64_t nnz, const int64_t *__restrict__ rp,
                                                      const int32_t *__restrict__ col,
                                                      const int32_t *__restrict__ deg, double *__restrict__ part,
                                                      unsigned long long *__restrict__ res)
{
    __shared__ double ld[4];
    double sxy = 0.0;
    int unsorted = 0;
    for_tile_entries(rp, n, nnz, [&](int64_t e, int64_t u) {
        const int32_t v = col[e];
        sxy += (double)deg[u] * (double)deg[v];
        if (e + 1 < rp[u + 1] && col[e + 1] <= v) unsorted = 1;
    });
    const double s = block_sum_d(sxy, ld);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
    if (unsorted) atomicOr(&res[SR_UNSORTED], 1ull);
}

// Partials summed in index order by one workgroup: out = sum of part[k * stride + off].
__global__ void __launch_bounds__(256) st_reduce_kernel(const double *__restrict__ part, int64_t count, int stride,
                                                        int off, unsigned long long *__restrict__ res, int slot)
{
    // each thread sums a contiguous stretch, then the stretches in order
    const int64_t per = (count + 255) / 256;
    const int64_t a = (int64_t)threadIdx.x * per, b = min(count, a + per);
    double s = 0.0;
    for (int64_t k = a; k < b; ++k) s += part[k * stride + off];
    __shared__ double all[256];
    all[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < 256; ++k) t += all[k];
        ((double *)res)[slot] = t;
    }
}

__device__ __forceinline__ bool rank_less(int32_t du, int64_t u, int32_t dv, int64_t v)
{
    return du < dv || (du == dv && u < v);
}

// Kept entries (u -> v with v above u in rank) per tile.
__global__ void __launch_bounds__(256) st_orient_count_kernel(int64_t n, int64_t nnz, const int64_t *__restrict__ rp,
                                                              const int32_t *__restrict__ col,
                                                              const int32_t *__restrict__ deg,
                                                              int64_t *__restrict__ tcnt)
{
    __shared__ int64_t li[4];
    int64_t c = 0;
    for_tile_entries(rp, n, nnz, [&](int64_t e, int64_t u) {
        const int32_t v = col[e];
        c += rank_less(deg[u], u, deg[v], v);
    });
    const int64_t s = block_sum_i(c, li);
    if (threadIdx.x == 0) tcnt[blockIdx.x] = s;
}

// Out-rows: kept entries in input order at tile offset + their rank in the
// tile; pre[e] = kept entries of the tile before e.
__global__ void __launch_bounds__(256) st_orient_fill_kernel(int64_t n, int64_t nnz, const int64_t *__restrict__ rp,
                                                             const int32_t *__restrict__ col,
                                                             const int32_t *__restrict__ deg,
                                                             const int64_t *__restrict__ tscan,
                                                             uint16_t *__restrict__ pre, int32_t *__restrict__ ocol)
{
    __shared__ int wcnt[4];
    // pass 1: kept entries per thread (16 consecutive entries each)
    uint32_t keep = 0;
    int mine = 0;
    int idx = 0;
    for_tile_entries(rp, n, nnz, [&](int64_t e, int64_t u) {
        const int32_t v = col[e];
        const bool k = rank_less(deg[u], u, deg[v], v);
        keep |= (uint32_t)k << idx;
        mine += k;
        ++idx;
    });
    // exclusive scan of the per-thread counts, in thread order
    int inc = mine;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int y = __shfl_up(inc, d);
        if ((int)(threadIdx.x & 63) >= d) inc += y;
    }
    if ((threadIdx.x & 63) == 63) wcnt[threadIdx.x >> 6] = inc;
    __syncthreads();
    int before = 0;
    for (int w = 0; w < (int)(threadIdx.x >> 6); ++w) before += wcnt[w];
    const int excl = before + inc - mine;
    const int64_t off = blockIdx.x ? tscan[blockIdx.x - 1] : 0;
    const int64_t p0 = (int64_t)blockIdx.x * ST_TILE;
    const int64_t e0 = p0 + (int64_t)threadIdx.x * ST_PER;
    const int64_t e1 = min(min(nnz, p0 + ST_TILE), e0 + ST_PER);
    int r = excl;
    for (int64_t e = e0; e < e1; ++e) {
        pre[e] = (uint16_t)r;
        if ((keep >> (e - e0)) & 1u) ocol[off + r++] = col[e];
    }
}

// Out-row offsets: orp[u] = kept entries before row u's first entry.
__global__ void __launch_bounds__(256) st_optr_kernel(int64_t n, int64_t nnz, const int64_t *__restrict__ rp,
                                                      const int64_t *__restrict__ tscan, int64_t ntiles,
                                                      const uint16_t *__restrict__ pre, int64_t *__restrict__ orp)
{
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u > n) return;
    const int64_t p = rp[u];
    if (p >= nnz) {
        orp[u] = ntiles ? tscan[ntiles - 1] : 0;
    } else {
        const int64_t t = p / ST_TILE;
        orp[u] = (t ? tscan[t - 1] : 0) + pre[p];
    }
}

// Triangles: for every out-edge u -> v, the common out-neighbours w of u and
// v by merging the two ascending out-rows; each adds one to t(u), t(v), t(w).
__global__ void __launch_bounds__(256) st_triangle_kernel(int64_t n, int64_t m, const int64_t *__restrict__ orp,
                                                          const int32_t *__restrict__ ocol,
                                                          unsigned long long *__restrict__ tv,
                                                          unsigned long long *__restrict__ res)
{
    __shared__ int64_t li[4];
    int64_t total = 0;
    for_tile_entries(orp, n, m, [&](int64_t e, int64_t u) {
        const int32_t v = ocol[e];
        int64_t i = orp[u], ie = orp[u + 1], j = orp[v], je = orp[v + 1];
        unsigned long long c = 0;
        while (i < ie && j < je) {
            const int32_t a = ocol[i], b = ocol[j];
            if (a < b) ++i;
            else if (b < a) ++j;
            else {
                atomicAdd(&tv[a], 1ull);
                ++c;
                ++i;
                ++j;
            }
        }
        if (c) {
            atomicAdd(&tv[u], c);
            atomicAdd(&tv[v], c);
        }
        total += (int64_t)c;
    });
    const int64_t s = block_sum_i(total, li);
    if (threadIdx.x == 0 && s) atomicAdd(&res[SR_TRIANGLES], (unsigned long long)s);
}

// Local clustering t(v) / C(d, 2) over vertices of degree >= 2.
__global__ void __launch_bounds__(256) st_local_kernel(int64_t n, const int32_t *__restrict__ deg,
                                                       const unsigned long long *__restrict__ tv,
                                                       double *__restrict__ part, unsigned long long *__restrict__ res)
{
    __shared__ double ld[4];
    __shared__ int64_t li[4];
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double x = 0.0;
    int64_t c = 0;
    if (v < n) {
        const int64_t d = deg[v];
        if (d >= 2) {
            x = (double)tv[v] / ((double)d * (double)(d - 1) * 0.5);
            c = 1;
        }
    }
    const double s = block_sum_d(x, ld);
    const int64_t cs = block_sum_i(c, li);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = s;
        atomicAdd(&res[SR_LCC_N], (unsigned long long)cs);
    }
}

__global__ void st_zero_kernel(unsigned long long *p, int64_t count)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) p[i] = 0ull;
}

struct StPlan {
    int64_t vblocks, tiles, otiles, m;
    size_t deg, res, vpart, epart, tcnt, pre, ocol, orp, tv, lpart, tmp, total;
};

StPlan st_plan(int64_t n, int64_t nnz, int tri)
{
    StPlan p;
    p.vblocks = std::max<int64_t>(1, (n + ST_VBLOCK - 1) / ST_VBLOCK);
    p.tiles = std::max<int64_t>(1, (nnz + ST_TILE - 1) / ST_TILE);
    p.m = nnz;  // out-entries: nnz / 2 for a symmetric graph, at most nnz
    p.otiles = std::max<int64_t>(1, (p.m + ST_TILE - 1) / ST_TILE);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes, 256);
        return o;
    };
    const size_t N = (size_t)std::max<int64_t>(n, 1);
    p.deg = take(N * 4);
    p.res = take(SR_WORDS * 8);
    p.vpart = take((size_t)p.vblocks * 3 * 8);
    p.epart = take((size_t)p.tiles * 8);
    p.tcnt = p.pre = p.ocol = p.orp = p.tv = p.lpart = p.tmp = 0;
    if (tri) {
        p.tcnt = take((size_t)p.tiles * 8);
        p.pre = take((size_t)std::max<int64_t>(nnz, 1) * 2);
        p.ocol = take((size_t)std::max<int64_t>(p.m, 1) * 4);
        p.orp = take((N + 1) * 8);
        p.tv = take(N * 8);
        p.lpart = take((size_t)p.vblocks * 8);
        p.tmp = take(scan_tmp_bytes(p.tiles));
    }
    p.total = off + 256;
    return p;
}

unsigned grid_n(int64_t x) { return (unsigned)std::max<int64_t>(1, (x + 255) / 256); }

}  // namespace

size_t stats_workspace_bytes(int64_t n, int64_t nnz, int triangles) { return st_plan(n, nnz, triangles).total; }

hipError_t launch_graph_stats(int64_t n, const int64_t *rp, const int32_t *col, int64_t nnz, double kmin,
                              int triangles, void *workspace, double *out_d, int64_t *out_i, hipStream_t s)
{
    const StPlan P = st_plan(n, nnz, triangles);
    char *base = (char *)align_up((size_t)workspace, 256);
    int32_t *deg = (int32_t *)(base + P.deg);
    auto *res = (unsigned long long *)(base + P.res);
    double *vpart = (double *)(base + P.vpart), *epart = (double *)(base + P.epart);
    hipError_t e;
    hipLaunchKernelGGL(st_zero_kernel, dim3(1), dim3(64), 0, s, res, (int64_t)SR_WORDS);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (n > 0) {
        hipLaunchKernelGGL(st_deg_kernel, dim3(grid_n(n)), dim3(256), 0, s, n, rp, deg);
        hipLaunchKernelGGL(st_vertex_kernel, dim3((unsigned)P.vblocks), dim3(256), 0, s, n, (const int32_t *)deg, kmin,
                           vpart, res);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        for (int k = 0; k < 3; ++k)
            hipLaunchKernelGGL(st_reduce_kernel, dim3(1), dim3(256), 0, s, (const double *)vpart, P.vblocks, 3, k, res,
                               SR_SUMLOG + k);
    }
    if (nnz > 0) {
        hipLaunchKernelGGL(st_edge_kernel, dim3((unsigned)P.tiles), dim3(256), 0, s, n, nnz, rp, col,
                           (const int32_t *)deg, epart, res);
        hipLaunchKernelGGL(st_reduce_kernel, dim3(1), dim3(256), 0, s, (const double *)epart, P.tiles, 1, 0, res,
                           SR_SUMXY);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    // copy back: the unsorted flag decides whether triangles can be counted
    unsigned long long h[SR_WORDS];
    if ((e = hipMemcpyAsync(h, res, sizeof(h), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    int64_t tri_count = (triangles && n == 0) ? 0 : -1;
    double lcc = 0.0;
    int64_t lcc_n = 0;
    if (triangles && !h[SR_UNSORTED] && n > 0) {
        auto *tcnt = (int64_t *)(base + P.tcnt);
        auto *pre = (uint16_t *)(base + P.pre);
        auto *ocol = (int32_t *)(base + P.ocol);
        auto *orp = (int64_t *)(base + P.orp);
        auto *tv = (unsigned long long *)(base + P.tv);
        double *lpart = (double *)(base + P.lpart);
        int64_t kept = 0;
        if (nnz > 0) {
            hipLaunchKernelGGL(st_orient_count_kernel, dim3((unsigned)P.tiles), dim3(256), 0, s, n, nnz, rp, col,
                               (const int32_t *)deg, tcnt);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            if ((e = inclusive_scan_i64(tcnt, P.tiles, base + P.tmp, s)) != hipSuccess) return e;
            hipLaunchKernelGGL(st_orient_fill_kernel, dim3((unsigned)P.tiles), dim3(256), 0, s, n, nnz, rp, col,
                               (const int32_t *)deg, (const int64_t *)tcnt, pre, ocol);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            if ((e = hipMemcpyAsync(&kept, tcnt + P.tiles - 1, 8, hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
        }
        hipLaunchKernelGGL(st_optr_kernel, dim3(grid_n(n + 1)), dim3(256), 0, s, n, nnz, rp, (const int64_t *)tcnt,
                           nnz > 0 ? P.tiles : (int64_t)0, (const uint16_t *)pre, orp);
        hipLaunchKernelGGL(st_zero_kernel, dim3(1024), dim3(256), 0, s, tv, n);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
        if (kept > 0) {
            const int64_t otiles = (kept + ST_TILE - 1) / ST_TILE;
            hipLaunchKernelGGL(st_triangle_kernel, dim3((unsigned)otiles), dim3(256), 0, s, n, kept,
                               (const int64_t *)orp, (const int32_t *)ocol, tv, res);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
        hipLaunchKernelGGL(st_local_kernel, dim3((unsigned)P.vblocks), dim3(256), 0, s, n, (const int32_t *)deg,
                           (const unsigned long long *)tv, lpart, res);
        hipLaunchKernelGGL(st_reduce_kernel, dim3(1), dim3(256), 0, s, (const double *)lpart, P.vblocks, 1, 0, res,
                           SR_LCC);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = hipMemcpyAsync(h, res, sizeof(h), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
        tri_count = (int64_t)h[SR_TRIANGLES];
        lcc = ((double *)h)[SR_LCC];
        lcc_n = (int64_t)h[SR_LCC_N];
    }
    const double *hd = (const double *)h;
    out_i[0] = (int64_t)h[SR_MAXDEG];
    out_i[1] = (int64_t)h[SR_TAIL];
    out_i[2] = (int64_t)h[SR_TRIADS];
    out_i[3] = (int64_t)h[SR_UNSORTED];
    out_i[4] = tri_count;
    out_i[5] = lcc_n;
    for (int b = 0; b < 33; ++b) out_i[8 + b] = (int64_t)h[SR_HIST + b];
    out_d[0] = hd[SR_SUMLOG];
    out_d[1] = hd[SR_SUMD2];
    out_d[2] = hd[SR_SUMD3];
    out_d[3] = hd[SR_SUMXY];
    out_d[4] = lcc;
    return hipSuccess;
}

}  // namespace rhg
