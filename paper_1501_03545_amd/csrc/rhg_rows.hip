// rhg_rows.hip -- ascending (canonical) rows of a CSR adjacency, in place.
//
// The search emits each row in search order, which depends on the tuning.
// Sorting every row gives one canonical layout: the same bytes for every
// tuning, and the layout of the plain pairwise definition of the edge set
// (Prop. 2: the generator returns exactly the pairs within distance R).
//
// Rows are sorted by length class, each class by its own kernel scanning
// the row offsets:
//   2 .. 64 entries     64 rows per workgroup, staged in LDS, each entry
//                       written at its rank (the number of smaller entries,
//                       ties by position);
//   65 .. 512           one wavefront per row, a sorting network in LDS;
//   513 .. 8192         one workgroup per row, the same network;
//   longer              listed; every 8192-entry tile of them is sorted in
//                       LDS, then each further merge level runs its long
//                       strides over global memory and its strides below the
//                       tile size in LDS again.
// The network is the bitonic sorter in the form whose comparators all point
// the same way: level k first compares entry i of every block of 2^k with its
// mirror in that block, then halves the stride down to 1.  In that form a
// row of any length sorts as if padded with +infinity, so no padding is
// stored and every comparator with a partner past the row's end is skipped.
#include "rhg_internal.h"

namespace rhg {

namespace {

constexpr int RS_ROWS = 64;            // rows per workgroup of the short-row kernel
constexpr int RS_SHORT_THREADS = 128;  // its workgroup size
constexpr int RS_SMALL = 64;           // rows up to this length are ranked
constexpr int RS_WAVE = 512;           // rows up to this length: one wavefront each
constexpr int RS_TILE = RHG_ROWS_TILE; // LDS tile (entries) of the workgroup network
static_assert((RS_TILE & (RS_TILE - 1)) == 0, "tile must be a power of two");

// Counters at the head of the auxiliary buffer (64-bit words).
enum { RC_LONG = 0, RC_TILES = 1, RC_MAXLEN = 2, RC_WORDS = 8 };

// Order-preserving map of int32 onto uint32 (flip the sign bit).
__device__ __forceinline__ uint32_t okey(int32_t v) { return (uint32_t)v ^ 0x80000000u; }
__device__ __forceinline__ int32_t oval(uint32_t k) { return (int32_t)(k ^ 0x80000000u); }

__device__ __forceinline__ void wsync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

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
// workgroup (a multiple of 64 threads).  L is uniform over the workgroup.
// With pair t handled by thread t mod blockDim, a stage of stride <= 64 (or
// a mirror step of level <= 128) keeps every wavefront inside its own runs
// of 128 keys, so between two such stages a wavefront barrier suffices.
__device__ __forceinline__ void stage_sync(bool wide)
{
    if (wide) __syncthreads();
    else wsync();
}

__device__ void block_sort(uint32_t *b, int L, bool full)
{
    const int P = pow2_at_least(L);
    if (full) {
        for (int blk = 2; blk <= P; blk <<= 1) {
            net_stage(b, L, P, blk, 0, threadIdx.x, blockDim.x);
            // next stage: stride blk / 4, or the next level's mirror step
            stage_sync(blk > 128 || (blk >= 4 ? blk / 4 >= 128 : 2 * blk > 128));
            for (int s = blk >> 2; s >= 1; s >>= 1) {
                net_stage(b, L, P, 0, s, threadIdx.x, blockDim.x);
                stage_sync(s >= 128 || (s > 1 ? s / 2 >= 128 : 2 * blk > 128));
            }
        }
        __syncthreads();
    } else {
        for (int s = P >> 1; s >= 1; s >>= 1) {
            net_stage(b, L, P, 0, s, threadIdx.x, blockDim.x);
            stage_sync(s >= 128 || s / 2 >= 128);
        }
        __syncthreads();
    }
}

__global__ void rows_init_kernel(unsigned long long *cnt)
{
    if (threadIdx.x < RC_WORDS) cnt[threadIdx.x] = 0ull;
}

// Rows of 2 .. 64 entries, 128 consecutive rows per workgroup: the entries
// are staged in LDS and each is written at its rank.  Rows longer than the
// tile go to the long-row list lp[2k] (at most lcap of them).
__global__ void __launch_bounds__(RS_SHORT_THREADS) rows_short_kernel(const int64_t *__restrict__ row_ptr, int32_t *__restrict__ col,
                                                         int64_t n, int32_t *__restrict__ lp, int64_t lcap,
                                                         unsigned long long *__restrict__ cnt)
{
    __shared__ int32_t vals[RS_ROWS * RS_SMALL];
    __shared__ uint8_t rowof[RS_ROWS * RS_SMALL];
    __shared__ int off[RS_ROWS + 1];
    __shared__ int slen[RS_ROWS];
    __shared__ int64_t rst[RS_ROWS];
    const int t = threadIdx.x;
    if (t < RS_ROWS) {
        const int64_t r = (int64_t)blockIdx.x * RS_ROWS + t;
        int64_t s0 = 0, len = 0;
        if (r < n) {
            s0 = row_ptr[r];
            len = row_ptr[r + 1] - s0;
        }
        rst[t] = s0;
        slen[t] = (len >= 2 && len <= RS_SMALL) ? (int)len : 0;
        if (len > RS_TILE) {  // rare: one atomic per long row
            const int64_t pos = (int64_t)atomicAdd(&cnt[RC_LONG], 1ull);
            if (pos < lcap) lp[2 * pos] = (int32_t)r;
            atomicMax(&cnt[RC_MAXLEN], (unsigned long long)len);
        }
    }
    __syncthreads();
    if (t < 64) {  // exclusive scan of the short lengths, RS_ROWS / 64 per lane
        constexpr int PL = RS_ROWS / 64;
        int a[PL], sum = 0;
#pragma unroll
        for (int k = 0; k < PL; ++k) {
            a[k] = slen[PL * t + k];
            sum += a[k];
        }
        int inc = sum;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int y = __shfl_up(inc, d);
            if (t >= d) inc += y;
        }
        int run = inc - sum;
#pragma unroll
        for (int k = 0; k < PL; ++k) {
            off[PL * t + k] = run;
            run += a[k];
        }
        if (t == 63) off[RS_ROWS] = inc;
    }
    __syncthreads();
    if (t < RS_ROWS)
        for (int q = 0; q < slen[t]; ++q) rowof[off[t] + q] = (uint8_t)t;
    __syncthreads();
    const int total = off[RS_ROWS];
    for (int k = t; k < total; k += RS_SHORT_THREADS) {
        const int tr = rowof[k];
        vals[k] = col[rst[tr] + (k - off[tr])];
    }
    __syncthreads();
    for (int k = t; k < total; k += RS_SHORT_THREADS) {
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

// Rows of 65 .. 512 entries: each wavefront scans chunks of 64 rows (one
// per lane) and sorts the ones of this class one after another.
__global__ void __launch_bounds__(256) rows_wave_kernel(const int64_t *__restrict__ row_ptr, int32_t *__restrict__ col,
                                                        int64_t n)
{
    __shared__ uint32_t buf[4][RS_WAVE];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    uint32_t *b = buf[wv];
    for (int64_t c0 = ((int64_t)blockIdx.x * 4 + wv) * 64; c0 < n; c0 += (int64_t)gridDim.x * 256) {
        const int64_t r = c0 + lane;
        int64_t s0 = 0, len = 0;
        if (r < n) {
            s0 = row_ptr[r];
            len = row_ptr[r + 1] - s0;
        }
        uint64_t m = __ballot(len > RS_SMALL && len <= RS_WAVE);
        while (m) {
            const int src = __ffsll((unsigned long long)m) - 1;
            m &= m - 1;
            const int64_t st = __shfl(s0, src);
            const int L = __shfl((int)len, src);
            for (int q = lane; q < L; q += 64) b[q] = okey(col[st + q]);
            wsync();
            wave_sort(b, L, lane);
            for (int q = lane; q < L; q += 64) col[st + q] = oval(b[q]);
            wsync();
        }
    }
}

// Rows of 513 .. 8192 entries: each workgroup scans chunks of 512 rows (one
// per thread) and sorts the ones of this class one after another.
__global__ void __launch_bounds__(512) rows_group_kernel(const int64_t *__restrict__ row_ptr, int32_t *__restrict__ col,
                                                         int64_t n)
{
    __shared__ uint32_t buf[RS_TILE];
    __shared__ int64_t gst[512];
    __shared__ int glen[512];
    __shared__ int ng;
    for (int64_t c0 = (int64_t)blockIdx.x * 512; c0 < n; c0 += (int64_t)gridDim.x * 512) {
        if (threadIdx.x == 0) ng = 0;
        __syncthreads();
        const int64_t r = c0 + threadIdx.x;
        if (r < n) {
            const int64_t s0 = row_ptr[r], len = row_ptr[r + 1] - s0;
            if (len > RS_WAVE && len <= RS_TILE) {
                const int k = atomicAdd(&ng, 1);
                gst[k] = s0;
                glen[k] = (int)len;
            }
        }
        __syncthreads();
        const int cnt = ng;
        for (int x = 0; x < cnt; ++x) {
            const int64_t st = gst[x];
            const int L = glen[x];
            for (int q = threadIdx.x; q < L; q += 512) buf[q] = okey(col[st + q]);
            __syncthreads();
            block_sort(buf, L, true);
            for (int q = threadIdx.x; q < L; q += 512) col[st + q] = oval(buf[q]);
            __syncthreads();
        }
        __syncthreads();  // every thread has read ng and gst before they are rewritten
    }
}

// Tile counts of the long rows, their exclusive prefix (lp[2k + 1]) and the
// tile map (row, tile number within the row) of every tile; the total goes to
// cnt[RC_TILES].  One workgroup of 1024.
__global__ void __launch_bounds__(1024) rows_lscan_kernel(const int64_t *__restrict__ row_ptr, int32_t *__restrict__ lp,
                                                          int64_t lcap, int2 *__restrict__ tmap, int64_t mapcap,
                                                          unsigned long long *__restrict__ cnt)
{
    __shared__ int64_t wsum[16];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int64_t nl = min((int64_t)cnt[RC_LONG], lcap);
    int64_t run = 0;
    for (int64_t b0 = 0; b0 < nl; b0 += 1024) {
        const int64_t k = b0 + t;
        int64_t tiles = 0;
        int r = 0;
        if (k < nl) {
            r = lp[2 * k];
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
        if (k < nl) {
            const int64_t first = run + before + inc - tiles;
            lp[2 * k + 1] = (int32_t)first;
            for (int64_t q = 0; q < tiles && first + q < mapcap; ++q) tmap[first + q] = make_int2(r, (int)q);
        }
        run += all;
        __syncthreads();
    }
    if (t == 0) cnt[RC_TILES] = (unsigned long long)min(run, mapcap);
}

// Every tile of the long rows: a full sort in LDS (merge_blk == 0), or, for
// the rows that take part in merge level merge_blk, the strides below the
// tile size.
__global__ void __launch_bounds__(512) rows_tile_kernel(const int64_t *__restrict__ row_ptr, int32_t *__restrict__ col,
                                                        const int2 *__restrict__ tmap,
                                                        const unsigned long long *__restrict__ cnt, int64_t merge_blk)
{
    constexpr int PER = RS_TILE / 512;
    __shared__ uint32_t buf[RS_TILE];
    const int64_t tt = (int64_t)cnt[RC_TILES];
    if (merge_blk && 2 * (int64_t)cnt[RC_MAXLEN] <= merge_blk) return;
    for (int64_t u = blockIdx.x; u < tt; u += gridDim.x) {
        const int2 m = tmap[u];
        const int64_t rs = row_ptr[m.x], len = row_ptr[m.x + 1] - rs;
        if (merge_blk && 2 * len <= merge_blk) continue;  // uniform: the row is already sorted
        const int64_t st = rs + (int64_t)m.y * RS_TILE;
        const int L = (int)min((int64_t)RS_TILE, len - (int64_t)m.y * RS_TILE);
        int32_t v[PER];
#pragma unroll
        for (int c = 0; c < PER; ++c) {
            const int q = threadIdx.x + 512 * c;
            v[c] = q < L ? col[st + q] : 0;
        }
#pragma unroll
        for (int c = 0; c < PER; ++c) {
            const int q = threadIdx.x + 512 * c;
            if (q < L) buf[q] = okey(v[c]);
        }
        __syncthreads();
        block_sort(buf, L, merge_blk == 0);
        for (int q = threadIdx.x; q < L; q += 512) col[st + q] = oval(buf[q]);
        __syncthreads();
    }
}

// One network step over global memory for the long rows: the mirror step of
// level blk (s == 0) or the stride-s step (s >= tile size).  blk and s are
// multiples of the tile size, so a tile holds only lower or only upper
// entries of its pairs; the lower tiles do the compare-exchanges, loading all
// their pairs before storing.
__global__ void __launch_bounds__(256) rows_gstep_kernel(const int64_t *__restrict__ row_ptr, int32_t *__restrict__ col,
                                                         const int2 *__restrict__ tmap,
                                                         const unsigned long long *__restrict__ cnt, int64_t blk,
                                                         int64_t s)
{
    constexpr int PER = RS_TILE / 256;
    if (2 * (int64_t)cnt[RC_MAXLEN] <= blk) return;
    const int64_t tt = (int64_t)cnt[RC_TILES];
    for (int64_t g = blockIdx.x; g < tt; g += gridDim.x) {
        const int2 m = tmap[g];
        const int64_t base = row_ptr[m.x], len = row_ptr[m.x + 1] - base;
        const int64_t i0 = (int64_t)m.y * RS_TILE;
        if (2 * len <= blk) continue;
        if (s == 0 ? (i0 & (blk - 1)) >= (blk >> 1) : (i0 & s) != 0) continue;  // an upper tile
        int32_t *p = col + base;
        // entry e of the tile is i = i0 + e; its partner j = j0 + e (stride)
        // or j0 - e (mirror), kept as an offset f(e) >= 0 from pj.  Valid e:
        // i < len and j < len.
        const int64_t j0 = s == 0 ? i0 - 2 * (i0 & (blk - 1)) + blk - 1 : i0 + s;
        const int32_t *pi = p + i0;
        int32_t *pj;
        int emin, emax;
        if (s == 0) {
            pj = p + (j0 - (RS_TILE - 1));
            emin = (int)min((int64_t)RS_TILE, max((int64_t)0, j0 - len + 1));
            emax = (int)min((int64_t)RS_TILE, len - i0);
        } else {
            pj = p + j0;
            emin = 0;
            emax = (int)max((int64_t)0, min((int64_t)RS_TILE, min(len - i0, len - j0)));
        }
        int32_t *qi = p + i0;
#pragma unroll 1
        for (int c0 = 0; c0 < PER; c0 += 8) {  // 8 pairs per thread in flight
            int32_t x[8], y[8];
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const int e = threadIdx.x + 256 * (c0 + c);
                const int f = s == 0 ? RS_TILE - 1 - e : e;
                const bool ok = e >= emin && e < emax;
                x[c] = ok ? pi[e] : 0;
                y[c] = ok ? pj[f] : 0;
            }
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const int e = threadIdx.x + 256 * (c0 + c);
                const int f = s == 0 ? RS_TILE - 1 - e : e;
                if (e >= emin && e < emax && x[c] > y[c]) {
                    qi[e] = y[c];
                    pj[f] = x[c];
                }
            }
        }
    }
}

}  // namespace

int64_t rows_long_bound(int64_t nnz) { return nnz / (RS_TILE + 1) + 1; }

int64_t rows_tile_bound(int64_t nnz, int64_t lcap) { return nnz / RS_TILE + lcap + 1; }

size_t rows_aux_bytes(int64_t lcap, int64_t mapcap)
{
    return 256 + align_up((size_t)(lcap > 0 ? lcap : 0) * 8, 256) + (size_t)(mapcap > 0 ? mapcap : 0) * 8;
}

hipError_t launch_sort_rows(const int64_t *row_ptr, int32_t *col, int64_t n, int64_t maxlen_bound, void *aux,
                            int64_t lcap, int64_t mapcap, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipError_t e;
    auto *cnt = (unsigned long long *)aux;
    int32_t *lp = (int32_t *)((char *)aux + 256);
    int2 *tmap = (int2 *)((char *)aux + 256 + align_up((size_t)lcap * 8, 256));
    hipLaunchKernelGGL(rows_init_kernel, dim3(1), dim3(64), 0, s, cnt);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(rows_short_kernel, dim3((unsigned)((n + RS_ROWS - 1) / RS_ROWS)), dim3(RS_SHORT_THREADS), 0, s, row_ptr, col,
                       n, lp, lcap, cnt);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (maxlen_bound <= RS_SMALL) return hipSuccess;
    const unsigned wgrid = (unsigned)std::min<int64_t>(4096, (n + 255) / 256);
    hipLaunchKernelGGL(rows_wave_kernel, dim3(wgrid), dim3(256), 0, s, row_ptr, col, n);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (maxlen_bound <= RS_WAVE) return hipSuccess;
    const unsigned ggrid = (unsigned)std::min<int64_t>(2048, (n + 511) / 512);
    hipLaunchKernelGGL(rows_group_kernel, dim3(ggrid), dim3(512), 0, s, row_ptr, col, n);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (maxlen_bound <= RS_TILE) return hipSuccess;  // no long rows
    hipLaunchKernelGGL(rows_lscan_kernel, dim3(1), dim3(1024), 0, s, row_ptr, lp, lcap, tmap, mapcap, cnt);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(rows_tile_kernel, dim3(1024), dim3(512), 0, s, row_ptr, col, (const int2 *)tmap, cnt,
                       (int64_t)0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // merge levels of the long rows; a level no row reaches exits at once
    for (int64_t blk = 2 * (int64_t)RS_TILE; blk / 2 < maxlen_bound; blk *= 2) {
        hipLaunchKernelGGL(rows_gstep_kernel, dim3(1024), dim3(256), 0, s, row_ptr, col, (const int2 *)tmap, cnt, blk,
                           (int64_t)0);
        for (int64_t st = blk / 4; st >= RS_TILE; st /= 2)
            hipLaunchKernelGGL(rows_gstep_kernel, dim3(1024), dim3(256), 0, s, row_ptr, col, (const int2 *)tmap, cnt,
                               blk, st);
        hipLaunchKernelGGL(rows_tile_kernel, dim3(1024), dim3(512), 0, s, row_ptr, col, (const int2 *)tmap, cnt, blk);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace rhg
