// rhg_lr.hip -- long-range augmentation of a generated graph (RHG-LR).
//
// The paper corrects the one unrealistic property of random hyperbolic
// graphs, their large diameter, by adding a small share of edges between
// uniformly chosen vertex pairs (0.5 % in its experiment: Sec. 4.2, the
// RHG-LR row of the generator table in Sec. 4.3, Appendix I).  It fixes
// neither the generator nor what happens to self-loops and repeated pairs;
// the definition used here:
//   candidate j = 0, 1, 2, ... is the pair of vertices floor(w * n / 2^64)
//   for the two 64-bit words w of the Philox4x32-10 block with counter
//   (j_lo, j_hi, 1, 0) and the graph's key (seed_lo, seed_hi) -- third word
//   1, where the points use 0;
//   a candidate is rejected if it is a self-loop, an edge of the graph, or a
//   pair an earlier candidate already gave; the first k accepted are added;
//   at most the candidates j < 2k + 4096 are drawn.
// The output CSR holds every input row followed by its added neighbours in
// the order their pairs were accepted.
//
// On the device all 2k + 4096 candidates are drawn at once.  Membership in
// the graph is a scan of the shorter of the two rows (one thread; one
// workgroup when that row is long).  Repeats are found with a hash table
// keyed by the pair that keeps the smallest candidate index.  A scan over the
// candidate flags ranks the accepted ones, the directed entries are sorted
// by source vertex (stable, so each row's extras stay in candidate order),
// and the CSR is rebuilt: with ins[e] = row_ptr[src[e] + 1] the old end of
// the row that receives sorted extra e, old entry p moves to
// p + #{e : ins[e] <= p} and extra e lands at ins[e] + e.
#include "rhg_internal.h"
#include "rhg_philox.h"

namespace rhg {

namespace {

constexpr int LR_SHORT = 256;     // rows up to this length are scanned by one thread
constexpr int LR_TILE = 4096;     // old entries per workgroup in the copy
constexpr int LR_TILE_INS = 2048; // insertion points staged in LDS per tile
constexpr uint64_t LR_EMPTY = ~0ull;

enum { LC_LONG = 0, LC_WORDS = 8 };

struct LrWs {
    int32_t *ca, *cb;          // candidate pair (a < b), J each
    int8_t *vflag;             // 1 admissible so far, 0 rejected, 2 waiting for the long check
    int64_t *pos;              // accepted-candidate flags, then their inclusive scan
    int32_t *lchk;             // candidates whose membership check needs a workgroup
    uint64_t *hkey;            // hash table: pair keys
    int32_t *hmin;             // hash table: smallest candidate index per key
    uint32_t *src, *dst, *src1, *dst1;  // directed extra entries (2k) and sort buffers
    int64_t *ins;              // insertion points of the sorted extras (2k)
    unsigned long long *cnt;
    void *tmp;
};

__device__ __forceinline__ uint64_t mix64(uint64_t x)
{
    // splitmix64's finaliser: a bijection that spreads the pair keys
    x ^= x >> 30;
    x *= 0xBF58476D1CE4E5B9ull;
    x ^= x >> 27;
    x *= 0x94D049BB133111EBull;
    x ^= x >> 31;
    return x;
}

__global__ void lr_init_kernel(uint64_t *hkey, int32_t *hmin, int64_t hsize, uint32_t *src, uint32_t *dst,
                               int64_t m2, uint32_t n, unsigned long long *cnt)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t i = i0; i < hsize; i += stride) {
        hkey[i] = LR_EMPTY;
        hmin[i] = INT32_MAX;
    }
    for (int64_t i = i0; i < m2; i += stride) {
        src[i] = n;  // sentinel: sorts after every vertex
        dst[i] = 0;
    }
    if (i0 < LC_WORDS) cnt[i0] = 0ull;
}

// Draws candidate j, rejects self-loops, and checks membership by scanning
// the shorter row (long rows are left to lr_long_kernel).
__global__ void __launch_bounds__(256) lr_draw_kernel(uint64_t seed, int64_t n, int64_t J,
                                                      const int64_t *__restrict__ row_ptr,
                                                      const int32_t *__restrict__ col, LrWs w)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= J) return;
    uint32_t x0 = (uint32_t)(uint64_t)j, x1 = (uint32_t)((uint64_t)j >> 32), x2 = 1u, x3 = 0u;
    philox4x32_10(x0, x1, x2, x3, (uint32_t)seed, (uint32_t)(seed >> 32));
    const uint64_t w0 = ((uint64_t)x1 << 32) | x0, w1 = ((uint64_t)x3 << 32) | x2;
    const uint64_t u = __umul64hi(w0, (uint64_t)n), v = __umul64hi(w1, (uint64_t)n);
    const int32_t a = (int32_t)min(u, v), b = (int32_t)max(u, v);
    w.ca[j] = a;
    w.cb[j] = b;
    int8_t flag = 0;
    if (a != b) {
        const int64_t sa = row_ptr[a], la = row_ptr[a + 1] - sa;
        const int64_t sb = row_ptr[b], lb = row_ptr[b + 1] - sb;
        const int64_t s0 = la <= lb ? sa : sb, len = la <= lb ? la : lb;
        const int32_t other = la <= lb ? b : a;
        if (len <= LR_SHORT) {
            flag = 1;
            for (int64_t q = 0; q < len; ++q)
                if (col[s0 + q] == other) {
                    flag = 0;
                    break;
                }
        } else {
            flag = 2;
            const unsigned long long k = atomicAdd(&w.cnt[LC_LONG], 1ull);
            w.lchk[k] = (int32_t)j;
        }
    }
    w.vflag[j] = flag;
}

// Membership of the candidates whose shorter row is long: one workgroup each.
__global__ void __launch_bounds__(256) lr_long_kernel(const int64_t *__restrict__ row_ptr,
                                                      const int32_t *__restrict__ col, LrWs w)
{
    __shared__ int found;
    const int64_t nl = (int64_t)w.cnt[LC_LONG];
    for (int64_t x = blockIdx.x; x < nl; x += gridDim.x) {
        const int32_t j = w.lchk[x];
        const int32_t a = w.ca[j], b = w.cb[j];
        const int64_t sa = row_ptr[a], la = row_ptr[a + 1] - sa;
        const int64_t sb = row_ptr[b], lb = row_ptr[b + 1] - sb;
        const int64_t s0 = la <= lb ? sa : sb, len = la <= lb ? la : lb;
        const int32_t other = la <= lb ? b : a;
        if (threadIdx.x == 0) found = 0;
        __syncthreads();
        int hit = 0;
        for (int64_t q = threadIdx.x; q < len; q += blockDim.x) hit |= col[s0 + q] == other;
        if (hit) atomicOr(&found, 1);
        __syncthreads();
        if (threadIdx.x == 0) w.vflag[j] = found ? 0 : 1;
        __syncthreads();
    }
}

// Admissible candidates enter the hash table, which keeps the smallest
// candidate index per pair (an order-independent result).
__global__ void __launch_bounds__(256) lr_hash_kernel(int64_t J, int64_t hmask, LrWs w)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= J || w.vflag[j] != 1) return;
    const uint64_t key = ((uint64_t)(uint32_t)w.ca[j] << 32) | (uint32_t)w.cb[j];
    for (int64_t h = (int64_t)(mix64(key) & (uint64_t)hmask);; h = (h + 1) & hmask) {
        const uint64_t prev = atomicCAS((unsigned long long *)&w.hkey[h], (unsigned long long)LR_EMPTY,
                                        (unsigned long long)key);
        if (prev == LR_EMPTY || prev == key) {
            atomicMin(&w.hmin[h], (int32_t)j);
            return;
        }
    }
}

// pos[j] = 1 for the first candidate of every admissible pair.
__global__ void __launch_bounds__(256) lr_first_kernel(int64_t J, int64_t hmask, LrWs w)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= J) return;
    int64_t first = 0;
    if (w.vflag[j] == 1) {
        const uint64_t key = ((uint64_t)(uint32_t)w.ca[j] << 32) | (uint32_t)w.cb[j];
        int64_t h = (int64_t)(mix64(key) & (uint64_t)hmask);
        while (w.hkey[h] != key) h = (h + 1) & hmask;
        first = w.hmin[h] == (int32_t)j;
    }
    w.pos[j] = first;
}

// The accepted candidates (rank < k after the scan) as directed entries
// 2t, 2t + 1 of accepted pair t; the count goes to *added.
__global__ void __launch_bounds__(256) lr_pairs_kernel(int64_t J, int64_t k, LrWs w, int64_t *added)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j == 0) *added = min(k, w.pos[J - 1]);
    if (j >= J) return;
    const int64_t before = j ? w.pos[j - 1] : 0;
    if (w.pos[j] == before || w.pos[j] > k) return;
    const int64_t t = before;
    const uint32_t a = (uint32_t)w.ca[j], b = (uint32_t)w.cb[j];
    w.src[2 * t] = a;
    w.dst[2 * t] = b;
    w.src[2 * t + 1] = b;
    w.dst[2 * t + 1] = a;
}

__global__ void __launch_bounds__(256) lr_ins_kernel(int64_t m2, uint32_t n, const int64_t *__restrict__ row_ptr,
                                                     LrWs w)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m2) return;
    const uint32_t s = w.src[e];
    w.ins[e] = s < n ? row_ptr[s + 1] : INT64_MAX;
}

// Number of sorted sources below v.
__device__ __forceinline__ int64_t lower_src(const uint32_t *src, int64_t m2, uint32_t v)
{
    int64_t lo = 0, hi = m2;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (src[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Number of insertion points at or before p, in ins[lo, hi).
__device__ __forceinline__ int64_t upper_ins(const int64_t *ins, int64_t lo, int64_t hi, int64_t p)
{
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (ins[mid] <= p) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__global__ void __launch_bounds__(256) lr_rowptr_kernel(int64_t n, const int64_t *__restrict__ row_ptr, int64_t m2,
                                                        LrWs w, int64_t *__restrict__ row_ptr_out)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v > n) return;
    row_ptr_out[v] = row_ptr[v] + lower_src(w.src, m2, (uint32_t)v);
}

// Old entries [p0, p0 + LR_TILE) per workgroup: entry p moves to
// p + #{e : ins[e] <= p}.
__global__ void __launch_bounds__(256) lr_copy_kernel(const int32_t *__restrict__ col, int64_t p_begin, int64_t p_end,
                                                      int64_t m2, LrWs w, int32_t *__restrict__ col_out)
{
    __shared__ int64_t sins[LR_TILE_INS];
    __shared__ int64_t lo_s, hi_s;
    const int64_t p0 = p_begin + (int64_t)blockIdx.x * LR_TILE;
    if (p0 >= p_end) return;
    const int64_t p1 = min(p_end, p0 + LR_TILE);
    if (threadIdx.x == 0) {
        lo_s = upper_ins(w.ins, 0, m2, p0 - 1);
        hi_s = upper_ins(w.ins, lo_s, m2, p1 - 1);
    }
    __syncthreads();
    const int64_t lo = lo_s, hi = hi_s;
    const bool staged = hi - lo <= LR_TILE_INS;
    if (staged)
        for (int64_t e = lo + threadIdx.x; e < hi; e += blockDim.x) sins[e - lo] = w.ins[e];
    __syncthreads();
    for (int64_t p = p0 + threadIdx.x; p < p1; p += blockDim.x) {
        int64_t sh;
        if (staged) {
            int a = 0, b = (int)(hi - lo);
            while (a < b) {
                const int mid = (a + b) >> 1;
                if (sins[mid] <= p) a = mid + 1;
                else b = mid;
            }
            sh = lo + a;
        } else {
            sh = upper_ins(w.ins, lo, hi, p);
        }
        col_out[p + sh] = col[p];
    }
}

__global__ void __launch_bounds__(256) lr_extra_kernel(const int64_t *__restrict__ added, LrWs w,
                                                       int32_t *__restrict__ col_out)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 2 * *added) return;
    col_out[w.ins[e] + e] = (int32_t)w.dst[e];
}

struct LrPlan {
    int64_t J, hsize, m2;
    size_t ca, cb, vflag, pos, lchk, hkey, hmin, src, dst, src1, dst1, ins, cnt, tmp, total;
};

LrPlan lr_plan(int64_t n, int64_t k)
{
    LrPlan p;
    p.J = 2 * k + 4096;
    p.m2 = 2 * k;
    p.hsize = 1;
    while (p.hsize < 2 * p.J) p.hsize <<= 1;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes, 256);
        return o;
    };
    const size_t M2 = (size_t)(p.m2 > 0 ? p.m2 : 1);
    p.ca = take((size_t)p.J * 4);
    p.cb = take((size_t)p.J * 4);
    p.vflag = take((size_t)p.J);
    p.pos = take((size_t)p.J * 8);
    p.lchk = take((size_t)p.J * 4);
    p.hkey = take((size_t)p.hsize * 8);
    p.hmin = take((size_t)p.hsize * 4);
    p.src = take(M2 * 4);
    p.dst = take(M2 * 4);
    p.src1 = take(M2 * 4);
    p.dst1 = take(M2 * 4);
    p.ins = take(M2 * 8);
    p.cnt = take(LC_WORDS * 8);
    p.tmp = take(std::max(scan_tmp_bytes(p.J), radix_sort_tmp_bytes(p.m2)));
    p.total = off + 256;
    (void)n;
    return p;
}

unsigned grid_of(int64_t x) { return (unsigned)std::max<int64_t>(1, (x + 255) / 256); }

}  // namespace

size_t lr_workspace_bytes(int64_t n, int64_t k) { return lr_plan(n, k).total; }

hipError_t launch_long_range(int64_t n, const int64_t *row_ptr, const int32_t *col, int64_t nnz, int64_t k,
                             uint64_t seed, void *workspace, int64_t *row_ptr_out, int32_t *col_out, int64_t *added,
                             hipStream_t s)
{
    const LrPlan P = lr_plan(n, k);
    char *base = (char *)align_up((size_t)workspace, 256);
    LrWs w;
    w.ca = (int32_t *)(base + P.ca);
    w.cb = (int32_t *)(base + P.cb);
    w.vflag = (int8_t *)(base + P.vflag);
    w.pos = (int64_t *)(base + P.pos);
    w.lchk = (int32_t *)(base + P.lchk);
    w.hkey = (uint64_t *)(base + P.hkey);
    w.hmin = (int32_t *)(base + P.hmin);
    w.src = (uint32_t *)(base + P.src);
    w.dst = (uint32_t *)(base + P.dst);
    w.src1 = (uint32_t *)(base + P.src1);
    w.dst1 = (uint32_t *)(base + P.dst1);
    w.ins = (int64_t *)(base + P.ins);
    w.cnt = (unsigned long long *)(base + P.cnt);
    w.tmp = base + P.tmp;
    const int64_t hmask = P.hsize - 1;
    hipError_t e;
    const int64_t init_n = std::max(P.hsize, P.m2);
    hipLaunchKernelGGL(lr_init_kernel, dim3((unsigned)std::min<int64_t>(65536, (init_n + 255) / 256)), dim3(256), 0,
                       s, w.hkey, w.hmin, P.hsize, w.src, w.dst, P.m2, (uint32_t)n, w.cnt);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(lr_draw_kernel, dim3(grid_of(P.J)), dim3(256), 0, s, seed, n, P.J, row_ptr, col, w);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(lr_long_kernel, dim3(1024), dim3(256), 0, s, row_ptr, col, w);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(lr_hash_kernel, dim3(grid_of(P.J)), dim3(256), 0, s, P.J, hmask, w);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(lr_first_kernel, dim3(grid_of(P.J)), dim3(256), 0, s, P.J, hmask, w);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = inclusive_scan_i64(w.pos, P.J, w.tmp, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(lr_pairs_kernel, dim3(grid_of(P.J)), dim3(256), 0, s, P.J, k, w, added);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    int bits = 1;
    while (bits < 32 && ((int64_t)1 << bits) <= n) ++bits;  // sources 0 .. n (n: sentinel)
    if ((e = radix_sort_pairs(w.src, w.dst, w.src1, w.dst1, P.m2, bits, w.tmp, s)) != hipSuccess) return e;
    if (P.m2 > 0) {
        hipLaunchKernelGGL(lr_ins_kernel, dim3(grid_of(P.m2)), dim3(256), 0, s, P.m2, (uint32_t)n, row_ptr, w);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(lr_rowptr_kernel, dim3(grid_of(n + 1)), dim3(256), 0, s, n, row_ptr, P.m2, w, row_ptr_out);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (nnz > 0) {
        const int64_t tiles = (nnz + LR_TILE - 1) / LR_TILE;
        for (int64_t t0 = 0; t0 < tiles; t0 += 1 << 30) {  // grid dimension limit
            const int64_t tn = std::min<int64_t>(tiles - t0, 1 << 30);
            hipLaunchKernelGGL(lr_copy_kernel, dim3((unsigned)tn), dim3(256), 0, s, col, t0 * LR_TILE, nnz, P.m2, w,
                               col_out);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
    }
    if (P.m2 > 0) {
        hipLaunchKernelGGL(lr_extra_kernel, dim3(grid_of(P.m2)), dim3(256), 0, s, (const int64_t *)added, w, col_out);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace rhg
