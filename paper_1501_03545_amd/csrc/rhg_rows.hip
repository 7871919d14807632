// rhg_rows.hip -- ascending (canonical) rows of a CSR adjacency, in place.
//
// The search emits each row in search order, which depends on the tuning.
// Sorting every row gives one canonical layout: the same bytes for every
// tuning, and the layout of the plain pairwise definition of the edge set
// (Prop. 2: the generator returns exactly the pairs within distance R).
//
// Rows are sorted by length class:
//   2 .. 64 entries     a workgroup takes 128 consecutive rows, stages their
//                       entries in LDS and writes each entry at its rank
//                       (the number of smaller entries, ties by position);
//   65 .. 512           one wavefront per row, a sorting network in LDS;
//   513 .. 8192         one workgroup per row, the same network in LDS;
//   longer              every 8192-entry tile is sorted in LDS, then each
//                       further merge level runs its long strides over
//                       global memory and its strides below the tile size
//                       in LDS again.
// The network is the bitonic sorter in the form whose comparators all point
// the same way: level k first compares entry i of every block of 2^k with its
// mirror in that block, then halves the stride down to 1.  In that form a
// row of any length sorts as if padded with +infinity, so no padding is
// stored and every comparator with a partner past the row's end is skipped.
#include "rhg_internal.h"

namespace rhg {

namespace {

constexpr int RS_ROWS = 128;           // rows per workgroup in the short-row kernel
constexpr int RS_SMALL = 64;           // rows up to this length are ranked
constexpr int RS_WAVE = 512;           // rows up to this length: one wavefront each
constexpr int RS_TILE = RHG_ROWS_TILE; // LDS tile (entries) of the workgroup network
static_assert((RS_TILE & (RS_TILE - 1)) == 0, "tile must be a power of two");

// Counters at the head of the auxiliary buffer (64-bit words).
enum { RC_WAVE = 0, RC_BLOCK = 1, RC_LONG = 2, RC_TILES = 3, RC_MAXLEN = 4, RC_WORDS = 8 };

__device__ __forceinline__ void wsync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Order-preserving map of int32 onto uint32 (flip the sign bit).
__device__ __forceinline__ uint32_t okey(int32_t v) { return (uint32_t)v ^ 0x80000000u; }
__device__ __forceinline__ int32_t oval(uint32_t k) { return (int32_t)(k ^ 0x80000000u); }

__device__ __forceinline__ int pow2_at_least(int x)
{
    int p = 1;
    while (p < x) p <<= 1;
    return p;
}

__device__ __forceinline__ void cmpx(uint32_t *b, int i, int j)
{
    const uint32_t x = b[i], y = b[j];
    if (x > y) {
        b[i] = y;
        b[j] = x;
    }
}

// One stage of the network over b[0, L), P = pow2_at_least(L): pair t of the
// P/2 pairs is handled by lane/thread t (strided by `step`).  blk > 0: the
// mirror step of level blk; otherwise the stride-s step.
__device__ __forceinline__ void net_stage(uint32_t *b, int L, int P, int blk, int s, int t0, int step)
{
    if (blk) {
        const int h = blk >> 1;
        for (int t = t0; t < (P >> 1); t += step) {
            const int loc = t & (h - 1);
            const int i = ((t - loc) << 1) + loc;
            const int j = i - loc + blk - 1 - loc;
            if (j < L) cmpx(b, i, j);
        }
    } else {
        for (int t = t0; t < (P >> 1); t += step) {
            const int i = ((t & ~(s - 1)) << 1) | (t & (s - 1));
            if (i + s < L) cmpx(b, i, i + s);
        }
    }
}

// Full sort of b[0, L) by one wavefront.
__device__ void wave_sort(uint32_t *b, int L, int lane)
{
    const int P = pow2_at_least(L);
    for (int blk = 2; blk <= P; blk <<= 1) {
        net_stage(b, L, P, blk, 0, lane, 64);
        wsync();
        for (int s = blk >> 2; s >= 1; s >>= 1) {
            net_stage(b, L, P, 0, s, lane, 64);
            wsync();
        }
    }
}

// Full sort of b[0, L) (full = true), or only the strides P/2 .. 1 (the tail
// of a merge level whose longer strides ran in global memory), by the whole
// workgroup.  L is uniform over the workgroup.
__device__ void block_sort(uint32_t *b, int L, bool full)
{
    const int P = pow2_at_least(L);
    if (full) {
        for (int blk = 2; blk <= P; blk <<= 1) {
            net_stage(b, L, P, blk, 0, threadIdx.x, blockDim.x);
            __syncthreads();
            for (int s = blk >> 2; s >= 1; s >>= 1) {
                net_stage(b, L, P, 0, s, threadIdx.x, blockDim.x);
                __syncthreads();
            }
        }
    } else {
        for (int s = P >> 1; s >= 1; s >>= 1) {
            net_stage(b, L, P, 0, s, threadIdx.x, blockDim.x);
            __syncthreads();
        }
    }
}

// Index k of the long row whose tiles hold tile number g: the largest k
// with prefix[k] <= g (prefixes are strictly increasing, each long row has
// at least two tiles).
__device__ int64_t find_long(const int32_t *lp, int64_t nl, int64_t g)
{
    int64_t lo = 0, hi = nl - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if ((int64_t)lp[2 * mid + 1] <= g) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ void rows_init_kernel(unsigned long long *cnt)
{
    if (threadIdx.x < RC_WORDS) cnt[threadIdx.x] = 0ull;
}

// Short rows in place, and the lists of the longer ones: wavefront rows grow
// from the front of ids, workgroup rows from its back (together at most n),
// long rows go to lp[2k] (at most lcap of them).
__global__ void __launch_bounds__(256) rows_short_kernel(const int64_t *__restrict__ row_ptr, int32_t *__restrict__ col,
                                                         int64_t n, int32_t *__restrict__ ids, int32_t *__restrict__ lp,
                                                         int64_t lcap, unsigned long long *__restrict__ cnt)
{
    __shared__ int32_t vals[RS_ROWS * RS_SMALL];
    __shared__ uint8_t rowof[RS_ROWS * RS_SMALL];
    __shared__ int off[RS_ROWS + 1];
    __shared__ int slen[RS_ROWS];
    __shared__ int64_t rst[RS_ROWS];
    const int t = threadIdx.x, lane = t & 63;
    if (t < RS_ROWS) {  // wavefronts 0 and 1: one row per lane
        const int64_t r = (int64_t)blockIdx.x * RS_ROWS + t;
        int64_t s0 = 0, len = 0;
        if (r < n) {
            s0 = row_ptr[r];
            len = row_ptr[r + 1] - s0;
        }
        const int cls = len <= 1 ? -1 : len <= RS_SMALL ? 0 : len <= RS_WAVE ? 1 : len <= RS_TILE ? 2 : 3;
        const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
#pragma unroll
        for (int c = 1; c <= 3; ++c) {
            const uint64_t m = __ballot(cls == c);
            if (m) {
                const int leader = __ffsll((unsigned long long)m) - 1;
                unsigned long long base = 0;
                if (lane == leader) base = atomicAdd(&cnt[c == 1 ? RC_WAVE : c == 2 ? RC_BLOCK : RC_LONG],
                                                     (unsigned long long)__popcll(m));
                base = __shfl(base, leader);
                if (cls == c) {
                    const int64_t pos = (int64_t)base + __popcll(m & below);
                    if (c == 1) ids[pos] = (int32_t)r;
                    else if (c == 2) ids[n - 1 - pos] = (int32_t)r;
                    else if (pos < lcap) lp[2 * pos] = (int32_t)r;
                }
            }
        }
        if (cls == 3) atomicMax(&cnt[RC_MAXLEN], (unsigned long long)len);
        rst[t] = s0;
        slen[t] = cls == 0 ? (int)len : 0;
    }
    __syncthreads();
    if (t < 64) {  // exclusive scan of the 128 short lengths, two per lane
        const int a = slen[2 * t], b = slen[2 * t + 1];
        int inc = a + b;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int y = __shfl_up(inc, d);
            if (t >= d) inc += y;
        }
        const int exc = inc - a - b;
        off[2 * t] = exc;
        off[2 * t + 1] = exc + a;
        if (t == 63) off[RS_ROWS] = inc;
    }
    __syncthreads();
    if (t < RS_ROWS)
        for (int q = 0; q < slen[t]; ++q) rowof[off[t] + q] = (uint8_t)t;
    __syncthreads();
    const int total = off[RS_ROWS];
    for (int k = t; k < total; k += 256) {
        const int tr = rowof[k];
        vals[k] = col[rst[tr] + (k - off[tr])];
    }
    __syncthreads();
    for (int k = t; k < total; k += 256) {
        const int tr = rowof[k];
        const int b = off[tr], L = slen[tr];
        const int32_t v = vals[k];
        int rank = 0;
        for (int q = 0; q < L; ++q) {
            const int32_t w = vals[b + q];
            rank += (w < v) | ((w == v) & (b + q < k));
        }
        col[rst[tr] + rank] = v;
    }
}

// Tile counts of the long rows and their exclusive prefix (lp[2k + 1]); the
// total goes to cnt[RC_TILES].  One workgroup of 1024.
__global__ void __launch_bounds__(1024) rows_lscan_kernel(const int64_t *__restrict__ row_ptr, int32_t *__restrict__ lp,
                                                          int64_t lcap, unsigned long long *__restrict__ cnt)
{
    __shared__ int64_t wsum[16];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int64_t nl = min((int64_t)cnt[RC_LONG], lcap);
    int64_t run = 0;
    for (int64_t b0 = 0; b0 < nl; b0 += 1024) {
        const int64_t k = b0 + t;
        int64_t tiles = 0;
        if (k < nl) {
            const int r = lp[2 * k];
            const int64_t len = row_ptr[r + 1] - row_ptr[r];
            tiles = (len + RS_TILE - 1) / RS_TILE;
        }
        int64_t inc = tiles;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int64_t y = __shfl_up(inc, d);
            if (lane >= d) inc += y;
        }
        if (lane == 63) wsum[wv] = inc;
        __syncthreads();
        int64_t before = 0, all = 0;
#pragma unroll
        for (int w = 0; w < 16; ++w) {
            const int64_t x = wsum[w];
            if (w < wv) before += x;
            all += x;
        }
        if (k < nl) lp[2 * k + 1] = (int32_t)(run + before + inc - tiles);
        run += all;
        __syncthreads();
    }
    if (t == 0) cnt[RC_TILES] = (unsigned long long)run;
}

// Rows of 65 .. 512 entries: one wavefront each.
__global__ void __launch_bounds__(256) rows_wave_kernel(const int64_t *__restrict__ row_ptr, int32_t *__restrict__ col,
                                                        const int32_t *__restrict__ ids,
                                                        const unsigned long long *__restrict__ cnt)
{
    __shared__ uint32_t buf[4][RS_WAVE];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t nw = (int64_t)cnt[RC_WAVE];
    uint32_t *b = buf[wv];
    for (int64_t w = (int64_t)blockIdx.x * 4 + wv; w < nw; w += (int64_t)gridDim.x * 4) {
        const int r = ids[w];
        const int64_t s0 = row_ptr[r];
        const int L = (int)(row_ptr[r + 1] - s0);
        for (int q = lane; q < L; q += 64) b[q] = okey(col[s0 + q]);
        wsync();
        wave_sort(b, L, lane);
        for (int q = lane; q < L; q += 64) col[s0 + q] = oval(b[q]);
        wsync();
    }
}

// Unit u: a workgroup row (u < nb) or tile u - nb of the long rows.  Sets
// the tile's first entry, its length, and the row's length.
__device__ void unit_of(int64_t u, int64_t nb, const int64_t *row_ptr, const int32_t *ids, int64_t n,
                        const int32_t *lp, int64_t nl, int64_t *st, int *L, int64_t *len)
{
    if (u < nb) {
        const int r = ids[n - 1 - u];
        *st = row_ptr[r];
        *len = row_ptr[r + 1] - *st;
        *L = (int)*len;
    } else {
        const int64_t g = u - nb;
        const int64_t k = find_long(lp, nl, g);
        const int r = lp[2 * k];
        const int64_t tile = g - lp[2 * k + 1];
        const int64_t rs = row_ptr[r];
        *len = row_ptr[r + 1] - rs;
        *st = rs + tile * RS_TILE;
        *L = (int)min((int64_t)RS_TILE, *len - tile * RS_TILE);
    }
}

// Rows of 513 .. 8192 entries, and every tile of the long rows: a full sort
// in LDS.  merge_blk > 0: only the long rows' tiles of rows that take part in
// merge level merge_blk, and only the strides below the tile size.
__global__ void __launch_bounds__(512) rows_tile_kernel(const int64_t *__restrict__ row_ptr, int32_t *__restrict__ col,
                                                        const int32_t *__restrict__ ids, int64_t n,
                                                        const int32_t *__restrict__ lp, int64_t lcap,
                                                        const unsigned long long *__restrict__ cnt, int64_t merge_blk)
{
    __shared__ uint32_t buf[RS_TILE];
    __shared__ int64_t seg_st, seg_len;
    __shared__ int seg_L;
    const int64_t nb = merge_blk ? 0 : (int64_t)cnt[RC_BLOCK];
    const int64_t nl = min((int64_t)cnt[RC_LONG], lcap), tt = (int64_t)cnt[RC_TILES];
    if (merge_blk && 2 * (int64_t)cnt[RC_MAXLEN] <= merge_blk) return;
    for (int64_t u = blockIdx.x; u < nb + tt; u += gridDim.x) {
        if (threadIdx.x == 0) {
            int64_t st, len;
            int L;
            unit_of(u, nb, row_ptr, ids, n, lp, nl, &st, &L, &len);
            seg_st = st;
            seg_L = L;
            seg_len = len;
        }
        __syncthreads();
        const int64_t st = seg_st, len = seg_len;
        const int L = seg_L;
        __syncthreads();
        if (merge_blk && 2 * len <= merge_blk) continue;  // uniform: the row is already sorted
        for (int q = threadIdx.x; q < L; q += blockDim.x) buf[q] = okey(col[st + q]);
        __syncthreads();
        block_sort(buf, L, merge_blk == 0);
        for (int q = threadIdx.x; q < L; q += blockDim.x) col[st + q] = oval(buf[q]);
        __syncthreads();
    }
}

// One network step over global memory for the long rows: the mirror step of
// level blk (s == 0) or the stride-s step (s >= tile size).  The lower entry
// of each pair does the compare-exchange; pairs are disjoint.
__global__ void __launch_bounds__(256) rows_gstep_kernel(const int64_t *__restrict__ row_ptr, int32_t *__restrict__ col,
                                                         const int32_t *__restrict__ lp, int64_t lcap,
                                                         const unsigned long long *__restrict__ cnt, int64_t blk,
                                                         int64_t s)
{
    __shared__ int64_t seg_base, seg_len, seg_i0;
    if (2 * (int64_t)cnt[RC_MAXLEN] <= blk) return;
    const int64_t nl = min((int64_t)cnt[RC_LONG], lcap), tt = (int64_t)cnt[RC_TILES];
    for (int64_t g = blockIdx.x; g < tt; g += gridDim.x) {
        if (threadIdx.x == 0) {
            const int64_t k = find_long(lp, nl, g);
            const int r = lp[2 * k];
            seg_base = row_ptr[r];
            seg_len = row_ptr[r + 1] - seg_base;
            seg_i0 = (g - lp[2 * k + 1]) * RS_TILE;
        }
        __syncthreads();
        const int64_t base = seg_base, len = seg_len, i0 = seg_i0;
        __syncthreads();
        if (2 * len <= blk) continue;
        int32_t *p = col + base;
        const int64_t iend = min(len, i0 + RS_TILE);
        for (int64_t i = i0 + threadIdx.x; i < iend; i += blockDim.x) {
            int64_t j;
            if (s == 0) {
                const int64_t loc = i & (blk - 1);
                if (loc >= (blk >> 1)) continue;
                j = i - loc + blk - 1 - loc;
            } else {
                if (i & s) continue;
                j = i + s;
            }
            if (j < len) {
                const int32_t x = p[i], y = p[j];
                if (x > y) {
                    p[i] = y;
                    p[j] = x;
                }
            }
        }
    }
}

}  // namespace

size_t rows_aux_bytes(int64_t lcap) { return 256 + (size_t)(lcap > 0 ? lcap : 0) * 8; }

int64_t rows_long_bound(int64_t nnz) { return nnz / (RS_TILE + 1) + 1; }

hipError_t launch_sort_rows(const int64_t *row_ptr, int32_t *col, int64_t n, int64_t maxlen_bound, int32_t *ids,
                            void *aux, int64_t lcap, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipError_t e;
    auto *cnt = (unsigned long long *)aux;
    int32_t *lp = (int32_t *)((char *)aux + 256);
    hipLaunchKernelGGL(rows_init_kernel, dim3(1), dim3(64), 0, s, cnt);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(rows_short_kernel, dim3((unsigned)((n + RS_ROWS - 1) / RS_ROWS)), dim3(256), 0, s, row_ptr, col,
                       n, ids, lp, lcap, cnt);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(rows_lscan_kernel, dim3(1), dim3(1024), 0, s, row_ptr, lp, lcap, cnt);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(rows_wave_kernel, dim3(2048), dim3(256), 0, s, row_ptr, col, ids, cnt);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(rows_tile_kernel, dim3(1024), dim3(512), 0, s, row_ptr, col, ids, n, lp, lcap, cnt,
                       (int64_t)0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // merge levels of the long rows; a level no row reaches exits at once
    for (int64_t blk = 2 * (int64_t)RS_TILE; blk / 2 < maxlen_bound; blk *= 2) {
        hipLaunchKernelGGL(rows_gstep_kernel, dim3(1024), dim3(256), 0, s, row_ptr, col, lp, lcap, cnt, blk,
                           (int64_t)0);
        for (int64_t st = blk / 4; st >= RS_TILE; st /= 2)
            hipLaunchKernelGGL(rows_gstep_kernel, dim3(1024), dim3(256), 0, s, row_ptr, col, lp, lcap, cnt, blk, st);
        hipLaunchKernelGGL(rows_tile_kernel, dim3(1024), dim3(512), 0, s, row_ptr, col, (const int32_t *)nullptr, n,
                           lp, lcap, cnt, blk);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace rhg
