// rhg_index.hip -- the flat polar index (Sec. 3.1 "Data structure" rebuilt
// for a GPU).
//
// The paper's polar quadtree splits cells at the angular midpoint and at the
// equal-mass radius of Eq. (3), so a cell at depth i holds a point with
// probability 4^-i (Lemma 1).  Here the radial direction is cut once into
// bands (E[j] <= r < E[j+1]) and each band's angular range into 2^cbits equal
// cells; points are sorted by (band, angle) with one radix sort, and a
// directory gives, for every cell, the first sorted position at or after it.
// A range query then reads whole runs of sorted points instead of walking a
// tree.
#include "rhg_geom.h"
#include "rhg_internal.h"

namespace rhg {

struct KeyArgs {
    double E[RHG_MAX_BANDS + 1];
    int B;
    int band_bits;
    double R;
};

// rt (may be NULL): (r, theta) interleaved in sample order, so that the
// gather after the sort reads each point with one 16-byte access.
__global__ void __launch_bounds__(256) key_kernel(KeyArgs A, int64_t n, const double *__restrict__ r,
                                                  const double *__restrict__ theta, uint32_t *__restrict__ keys,
                                                  uint32_t *__restrict__ vals, double2 *__restrict__ rt,
                                                  int validate, unsigned long long *stats)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double ri = r[i], ti = theta[i];
        if (rt) rt[i] = make_double2(ri, ti);
        if (validate && !(ri >= 0.0 && ri <= A.R && ti >= 0.0 && ti <= RHG_TWO_PI_D))
            atomicAdd(&stats[ST_BAD_INPUT], 1ull);
        keys[i] = point_key(A.E, A.B, A.band_bits, ri, ti);
        vals[i] = (uint32_t)i;
    }
}

// First sorted position whose key is >= k, searched in [lo, hi).
__device__ __forceinline__ int64_t lower_bound_key(const uint32_t *keys, int64_t lo, int64_t hi, uint64_t k)
{
    while (lo < hi) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        if ((uint64_t)keys[mid] < k) lo = mid + 1; else hi = mid;
    }
    return lo;
}

__global__ void band_start_kernel(const uint32_t *__restrict__ keys, int64_t n, int B, int band_bits,
                                  int32_t *__restrict__ band_start)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j > B) return;
    int64_t p;
    if (j == 0) p = 0;
    else if (j == B) p = n;
    else p = lower_bound_key(keys, 0, n, (uint64_t)j << (32 - band_bits));
    band_start[j] = (int32_t)p;
}

struct DirArgs {
    int64_t dir_base[RHG_MAX_BANDS + 1];
    int cbits[RHG_MAX_BANDS];
    int B;
    int band_bits;
    int64_t total;
};

// dir[dir_base[j] + c] = first sorted position of band j whose cell is >= c,
// for c = 0 .. 2^cbits[j] (the last entry is the band's end).  One pass over
// the sorted keys: position p writes the entries of the cells after its
// predecessor's cell up to its own (and the last position of a band those
// up to the band's end), so every entry is written once.
__global__ void __launch_bounds__(256) dir_fill_kernel(DirArgs A, int64_t n, const uint32_t *__restrict__ keys,
                                                       const int32_t *__restrict__ band_start,
                                                       int32_t *__restrict__ dir)
{
    const int ab = 32 - A.band_bits;  // angle bits of a key
    const uint32_t amask = ab >= 32 ? 0xffffffffu : ((1u << ab) - 1u);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) {
        const uint32_t k = keys[p];
        const int j = A.band_bits ? (int)(k >> ab) : 0;
        const int cb = A.cbits[j];
        const int64_t s = band_start[j], t = band_start[j + 1];
        const int64_t c = cb ? (int64_t)((k & amask) >> (ab - cb)) : 0;
        const int64_t cp = (p > s) ? (cb ? (int64_t)((keys[p - 1] & amask) >> (ab - cb)) : 0) : -1;
        int32_t *d = dir + A.dir_base[j];
        for (int64_t cc = cp + 1; cc <= c; ++cc) d[cc] = (int32_t)p;
        if (p == t - 1)
            for (int64_t cc = c + 1; cc <= ((int64_t)1 << cb); ++cc) d[cc] = (int32_t)t;
    }
}

// Empty bands have no position to write their directory: all of it is the
// band's (empty) start.  One block per band.
__global__ void __launch_bounds__(256) dir_empty_kernel(DirArgs A, const int32_t *__restrict__ band_start,
                                                        int32_t *__restrict__ dir)
{
    const int j = blockIdx.x;
    if (j >= A.B) return;
    const int32_t s = band_start[j];
    if (s != band_start[j + 1]) return;
    const int64_t m = ((int64_t)1 << A.cbits[j]) + 1;
    for (int64_t c = threadIdx.x; c < m; c += 256) dir[A.dir_base[j] + c] = s;
}

// Sorted per-point records: r, theta (binary64) and the FP32 screen record
// (e^r / sqrt(2 cosh R), e^-r / sqrt(2 cosh R), sinh r sqrt(2 / cosh R),
// original id as raw bits).
__global__ void __launch_bounds__(256) gather_kernel(int64_t n, const double *__restrict__ r,
                                                     const double *__restrict__ theta,
                                                     const double2 *__restrict__ rt,
                                                     const uint32_t *__restrict__ perm, double inv, double sc,
                                                     double *__restrict__ sr, double *__restrict__ st,
                                                     float4 *__restrict__ rec)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) {
        uint32_t id = perm[p];
        if (id >= (uint64_t)n) id = 0;  // unreachable for a valid permutation; keeps reads in bounds
        double ri, ti;
        if (rt) {
            const double2 x = rt[id];
            ri = x.x;
            ti = x.y;
        } else {
            ri = r[id];
            ti = theta[id];
        }
        sr[p] = ri;
        st[p] = ti;
        rec[p] = point_record(ri, id, inv, sc);
    }
}

static unsigned grid_for(int64_t n, int64_t cap = 65536)
{
    int64_t b = (n + 255) / 256;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (unsigned)b;
}

// Band starts and the cell directory of the sorted keys idx->keys.
hipError_t launch_index_directory(rhg_index *idx, hipStream_t s)
{
    const int64_t n = idx->n;
    const Layout &L = idx->L;
    hipLaunchKernelGGL(band_start_kernel, dim3(1), dim3(128), 0, s, idx->keys, n, L.B, L.band_bits,
                       idx->band_start);
    hipError_t e;
    if ((e = hipGetLastError()) != hipSuccess) return e;
    DirArgs da;
    for (int j = 0; j <= L.B; ++j) da.dir_base[j] = L.dir_base[j];
    for (int j = 0; j < L.B; ++j) da.cbits[j] = L.cbits[j];
    da.B = L.B;
    da.band_bits = L.band_bits;
    da.total = L.dir_total;
    if (n > 0)
        hipLaunchKernelGGL(dir_fill_kernel, dim3(grid_for(n)), dim3(256), 0, s, da, n, idx->keys, idx->band_start,
                           idx->dir);
    hipLaunchKernelGGL(dir_empty_kernel, dim3((unsigned)L.B), dim3(256), 0, s, da, idx->band_start, idx->dir);
    return hipGetLastError();
}

hipError_t launch_build_index(rhg_index *idx, const double *r, const double *theta, uint32_t *k1,
                              uint32_t *v0, uint32_t *v1, int validate, hipStream_t s)
{
    const int64_t n = idx->n;
    const Layout &L = idx->L;
    KeyArgs ka;
    for (int j = 0; j <= L.B; ++j) ka.E[j] = L.E[j];
    ka.B = L.B;
    ka.band_bits = L.band_bits;
    ka.R = idx->p.R;
    hipError_t e;
    double2 *rt = idx->rt;
    if (n > 0) {
        PhaseScope ps(RHG_PHASE_SORT, s);
        hipLaunchKernelGGL(key_kernel, dim3(grid_for(n)), dim3(256), 0, s, ka, n, r, theta, idx->keys, v0, rt,
                           validate, idx->stats);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = radix_sort_pairs(idx->keys, v0, k1, v1, n, 32, idx->tmp, s)) != hipSuccess) return e;
    }
    PhaseScope ps_index(RHG_PHASE_INDEX, s);
    if ((e = launch_index_directory(idx, s)) != hipSuccess) return e;
    phase_end(ps_index.rec, s);
    ps_index.rec = nullptr;
    if (n > 0) {
        PhaseScope ps(RHG_PHASE_GATHER, s);
        const double inv = 1.0 / sqrt(2.0 * idx->p.cosh_R), sc = sqrt(2.0 / idx->p.cosh_R);
        hipLaunchKernelGGL(gather_kernel, dim3(grid_for(n)), dim3(256), 0, s, n, r, theta, (const double2 *)rt, v0,
                           inv, sc, idx->sr, idx->st, idx->rec);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace rhg
