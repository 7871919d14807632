// rhg_sort.hip -- device-wide scan and LSD radix sort (wave64 kernels).
//
// Scan: reduce-then-scan over tiles of 2048 elements, recursive on the tile
// sums.  Tiles are staged through LDS so global loads and stores stay
// coalesced.
//
// Radix sort: least-significant-digit first, 8-bit digits, stable.  Each pass
// is (1) a per-tile digit histogram, (2) an exclusive scan of the digit-major
// histogram table, (3) a stable scatter in which every wavefront ranks its
// 64-element chunks with eight ballots (lanes holding the same digit find
// each other bit by bit), so equal keys keep their input order.
#include "rhg_internal.h"

namespace rhg {

// ------------------------------------------------------------------ scan

constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_BLOCK * SCAN_ITEMS;

template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T x, int lane)
{
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        T y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    return x;
}

// Exclusive scan of one value per thread across the 256-thread block.
template <typename T>
__device__ __forceinline__ T block_exclusive_scan(T v, T *wave_tot, T *total)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    T inc = wave_inclusive_scan(v, lane);
    if (lane == 63) wave_tot[wave] = inc;
    __syncthreads();
    T off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < SCAN_BLOCK / 64; ++w) {
        T t = wave_tot[w];
        if (w < wave) off += t;
        tot += t;
    }
    *total = tot;
    __syncthreads();
    return off + inc - v;
}

template <typename T>
__global__ void __launch_bounds__(SCAN_BLOCK) scan_reduce_kernel(const T *__restrict__ x, int64_t n,
                                                                T *__restrict__ part)
{
    __shared__ T wave_tot[SCAN_BLOCK / 64];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    T s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        int64_t i = base + k * SCAN_BLOCK + threadIdx.x;
        if (i < n) s += x[i];
    }
    T tot;
    block_exclusive_scan<T>(s, wave_tot, &tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

template <typename T, bool INCLUSIVE>
__global__ void __launch_bounds__(SCAN_BLOCK) scan_tile_kernel(const T *__restrict__ in, T *__restrict__ out,
                                                              int64_t n, const T *__restrict__ carry)
{
    __shared__ T tile[SCAN_TILE];
    __shared__ T wave_tot[SCAN_BLOCK / 64];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        int64_t i = base + k * SCAN_BLOCK + threadIdx.x;
        tile[k * SCAN_BLOCK + threadIdx.x] = (i < n) ? in[i] : (T)0;
    }
    __syncthreads();
    T v[SCAN_ITEMS];
    T s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        v[k] = tile[threadIdx.x * SCAN_ITEMS + k];
        s += v[k];
    }
    T tot;
    T run = block_exclusive_scan<T>(s, wave_tot, &tot);
    if (carry) run += carry[blockIdx.x];
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        if (INCLUSIVE) { run += v[k]; tile[threadIdx.x * SCAN_ITEMS + k] = run; }
        else { tile[threadIdx.x * SCAN_ITEMS + k] = run; run += v[k]; }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        int64_t i = base + k * SCAN_BLOCK + threadIdx.x;
        if (i < n) out[i] = tile[k * SCAN_BLOCK + threadIdx.x];
    }
}

template <typename T>
static size_t scan_tmp_bytes_t(int64_t n)
{
    size_t bytes = 0;
    int64_t m = n;
    while (m > SCAN_TILE) {
        m = (m + SCAN_TILE - 1) / SCAN_TILE;
        bytes += align_up((size_t)m * sizeof(T), 256);
    }
    return bytes + 256;
}

template <typename T, bool INCLUSIVE>
static hipError_t scan_t(T *x, int64_t n, char *tmp, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (nb == 1) {
        hipLaunchKernelGGL((scan_tile_kernel<T, INCLUSIVE>), dim3(1), dim3(SCAN_BLOCK), 0, s, x, x, n,
                           (const T *)nullptr);
        return hipGetLastError();
    }
    T *part = (T *)tmp;
    char *next = tmp + align_up((size_t)nb * sizeof(T), 256);
    hipLaunchKernelGGL((scan_reduce_kernel<T>), dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, s, x, n, part);
    hipError_t e = scan_t<T, false>(part, nb, next, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((scan_tile_kernel<T, INCLUSIVE>), dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, s, x, x, n,
                       (const T *)part);
    return hipGetLastError();
}

size_t scan_tmp_bytes(int64_t n) { return scan_tmp_bytes_t<int64_t>(n); }

hipError_t inclusive_scan_i64(int64_t *x, int64_t n, void *tmp, hipStream_t s)
{
    return scan_t<int64_t, true>(x, n, (char *)tmp, s);
}

// ------------------------------------------------------------ radix sort

constexpr int RS_BLOCK = 256;
constexpr int RS_WAVES = RS_BLOCK / 64;
constexpr int RS_ITEMS = 16;                 // 64-element chunks per wave
constexpr int RS_WAVE_TILE = 64 * RS_ITEMS;  // 1024
constexpr int RS_TILE = RS_WAVES * RS_WAVE_TILE;  // 4096

__global__ void __launch_bounds__(RS_BLOCK) radix_hist_kernel(const uint32_t *__restrict__ keys, int64_t n,
                                                             int shift, uint32_t *__restrict__ counts,
                                                             int64_t nblocks)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
#pragma unroll 4
    for (int k = 0; k < RS_TILE / RS_BLOCK; ++k) {
        int64_t i = base + k * RS_BLOCK + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    counts[(int64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// Lanes of the wave whose 8-bit digit equals this lane's digit.
__device__ __forceinline__ uint64_t match_digit(uint32_t d, uint64_t valid)
{
    uint64_t m = valid;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const uint64_t bal = __ballot((d >> b) & 1u);
        m &= ((d >> b) & 1u) ? bal : ~bal;
    }
    return m;
}

// One LSD pass over a tile of RS_TILE elements: the tile is first sorted by
// the digit in LDS (stably: by wave, chunk and lane, as in the input), then
// written out in LDS order, so that consecutive threads write consecutive
// addresses of the same digit's run.
__global__ void __launch_bounds__(RS_BLOCK) radix_scatter_kernel(
    const uint32_t *__restrict__ kin, const uint32_t *__restrict__ vin, uint32_t *__restrict__ kout,
    uint32_t *__restrict__ vout, int64_t n, int shift, const uint32_t *__restrict__ offsets, int64_t nblocks)
{
    __shared__ uint32_t wh[RS_WAVES][256];
    __shared__ uint32_t lstart[256], gbase[256], tot[256];
    __shared__ uint32_t lk[RS_TILE], lv[RS_TILE];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int d = threadIdx.x; d < RS_WAVES * 256; d += RS_BLOCK) (&wh[0][0])[d] = 0;
    __syncthreads();
    const int64_t tbase = (int64_t)blockIdx.x * RS_TILE;
    const int64_t wbase = tbase + (int64_t)wave * RS_WAVE_TILE;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint32_t key[RS_ITEMS], val[RS_ITEMS];
#pragma unroll 4
    for (int c = 0; c < RS_ITEMS; ++c) {
        const int64_t i = wbase + c * 64 + lane;
        key[c] = (i < n) ? kin[i] : 0u;
        val[c] = (i < n) ? vin[i] : 0u;
    }
    // per-wave digit histogram
#pragma unroll 4
    for (int c = 0; c < RS_ITEMS; ++c) {
        const int64_t i = wbase + c * 64 + lane;
        const uint64_t valid = __ballot(i < n);
        const uint32_t d = (key[c] >> shift) & 255u;
        const uint64_t m = match_digit(d, valid);
        if (i < n && (m & lt) == 0) wh[wave][d] += (uint32_t)__popcll(m);
    }
    __syncthreads();
    // digit totals of the tile, their exclusive prefix (the digit runs in
    // LDS), and each wave's start inside its digits' runs
    const int dt = threadIdx.x;  // RS_BLOCK == 256 digits
    uint32_t sum = 0;
#pragma unroll
    for (int w = 0; w < RS_WAVES; ++w) sum += wh[w][dt];
    tot[dt] = sum;
    gbase[dt] = offsets[(int64_t)dt * nblocks + blockIdx.x];
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const uint32_t add = dt >= o ? tot[dt - o] : 0u;
        __syncthreads();
        tot[dt] += add;
        __syncthreads();
    }
    {
        uint32_t run = tot[dt] - sum;  // exclusive prefix
        lstart[dt] = run;
#pragma unroll
        for (int w = 0; w < RS_WAVES; ++w) {
            const uint32_t t = wh[w][dt];
            wh[w][dt] = run;
            run += t;
        }
    }
    __syncthreads();
#pragma unroll 4
    for (int c = 0; c < RS_ITEMS; ++c) {
        const int64_t i = wbase + c * 64 + lane;
        const uint64_t valid = __ballot(i < n);
        const uint32_t d = (key[c] >> shift) & 255u;
        const uint64_t m = match_digit(d, valid);
        const uint32_t rank = (uint32_t)__popcll(m & lt);
        const uint32_t pos = wh[wave][d] + rank;
        __builtin_amdgcn_wave_barrier();
        if (i < n && pos < (uint32_t)RS_TILE) {
            lk[pos] = key[c];
            lv[pos] = val[c];
            if (rank == 0) wh[wave][d] = pos + (uint32_t)__popcll(m);
        }
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    const int64_t count = n - tbase < (int64_t)RS_TILE ? n - tbase : (int64_t)RS_TILE;
    for (int t = threadIdx.x; t < count; t += RS_BLOCK) {
        const uint32_t k = lk[t];
        const uint32_t d = (k >> shift) & 255u;
        const uint64_t pos = (uint64_t)gbase[d] + (uint32_t)t - lstart[d];
        if (pos < (uint64_t)n) {
            kout[pos] = k;
            vout[pos] = lv[t];
        }
    }
}

size_t radix_sort_tmp_bytes(int64_t n)
{
    const int64_t nb = (n + RS_TILE - 1) / RS_TILE;
    const int64_t cnt = nb * 256;
    return align_up((size_t)cnt * sizeof(uint32_t), 256) + scan_tmp_bytes_t<uint32_t>(cnt);
}

hipError_t radix_sort_pairs(uint32_t *k0, uint32_t *v0, uint32_t *k1, uint32_t *v1, int64_t n, int bits,
                            void *tmp, hipStream_t s)
{
    if (n <= 1) return hipSuccess;
    const int64_t nb = (n + RS_TILE - 1) / RS_TILE;
    const int64_t cnt = nb * 256;
    uint32_t *counts = (uint32_t *)tmp;
    char *scan_tmp = (char *)tmp + align_up((size_t)cnt * sizeof(uint32_t), 256);
    uint32_t *ka = k0, *va = v0, *kb = k1, *vb = v1;
    int passes = 0;
    for (int shift = 0; shift < bits; shift += 8, ++passes) {
        hipLaunchKernelGGL(radix_hist_kernel, dim3((unsigned)nb), dim3(RS_BLOCK), 0, s, ka, n, shift, counts, nb);
        hipError_t e = scan_t<uint32_t, false>(counts, cnt, scan_tmp, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(radix_scatter_kernel, dim3((unsigned)nb), dim3(RS_BLOCK), 0, s, ka, va, kb, vb, n,
                           shift, counts, nb);
        uint32_t *t;
        t = ka; ka = kb; kb = t;
        t = va; va = vb; vb = t;
    }
    if (passes & 1) {
        hipError_t e = hipMemcpyAsync(k0, ka, (size_t)n * 4, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
        e = hipMemcpyAsync(v0, va, (size_t)n * 4, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

}  // namespace rhg
