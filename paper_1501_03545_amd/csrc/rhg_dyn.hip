// rhg_dyn.hip -- the dynamic model: vertices move and the graph follows.
//
// Sec. 5 notes that the incremental construction of the polar quadtree
// admits a dynamic model with vertex movement and leaves it to future work.
// Here a step takes a batch of moves (vertex ids with new coordinates) and
// brings the whole state to what generation from scratch on the moved points
// gives: the index is updated in place of a rebuild and only the rows that
// change are recomputed.
//
// State: the points by id, the index (sorted (key, id) order, cell
// directory, FP32 records), the sorted position of every id, and the graph
// as a CSR with ascending rows.  A step:
//   1. checks the moves (ids in range and distinct, coordinates in the disk),
//      marks the moved ids and stores their new coordinates;
//   2. updates the index by a merge: the k moved entries are sorted by their
//      new (key, id); every unmoved entry moves to p - (moved entries before
//      it) + (new entries before it), every new entry to its rank plus the
//      unmoved entries before it (binary searches), and the cell directory is
//      recomputed from the merged keys;
//   3. searches the moved vertices' rows on the updated index (exact);
//   4. counts, per unmoved vertex, the moved neighbours it loses (the moved
//      vertices' old rows) and gains (their new rows), listing the vertices
//      whose rows change;
//   5. scans the new degrees, copies every unchanged row to its new place,
//      assembles the changed rows (kept entries plus gained neighbours, or the
//      moved vertex's new row) in a compact buffer, sorts them and copies them
//      into place.
// The work besides the O(n + m) copies is proportional to the moves and
// their neighbourhoods.
#include <string.h>

#include <algorithm>
#include <vector>

#include "rhg_geom.h"
#include "rhg_internal.h"

namespace rhg {
namespace {

struct DynArgs {
    double E[RHG_MAX_BANDS + 1];
    int B, band_bits;
    double R, inv, sc;
    int64_t n;
};

// Number of entries of the ascending array a[0..m) below x.
__device__ __forceinline__ int64_t count_below_u32(const uint32_t *a, int64_t m, uint32_t x)
{
    int64_t lo = 0, hi = m;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (a[mid] < x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

__global__ void __launch_bounds__(256) dyn_fill_i32(int32_t *p, int64_t n, int32_t v)
{
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) p[i] = v;
}

// Step 1: the moves' checks.  err bit 0: an id out of range or a coordinate
// outside the disk; bit 1: an id listed twice.  Valid ids are marked moved.
__global__ void __launch_bounds__(256) dyn_check_kernel(DynArgs A, const int32_t *__restrict__ mid,
                                                        const double *__restrict__ mr, const double *__restrict__ mt,
                                                        int64_t k, int32_t *__restrict__ moved, int32_t *err)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= k) return;
    const int32_t id = mid[i];
    const double r = mr[i], t = mt[i];
    if (id < 0 || (int64_t)id >= A.n || !(r >= 0.0 && r <= A.R && t >= 0.0 && t < RHG_TWO_PI_D)) {
        atomicOr(err, 1);
        return;
    }
    if (atomicExch(&moved[id], 1) != 0) atomicOr(err, 2);
}

// Undo the marks of a refused batch.
__global__ void __launch_bounds__(256) dyn_unmark_kernel(DynArgs A, const int32_t *__restrict__ mid, int64_t k,
                                                         int32_t *__restrict__ moved)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= k) return;
    const int32_t id = mid[i];
    if (id >= 0 && (int64_t)id < A.n) moved[id] = 0;
}

__device__ __forceinline__ uint64_t comp(uint32_t key, uint32_t id) { return ((uint64_t)key << 32) | id; }

// Number of (key, id) entries of the ascending arrays below x.
__device__ __forceinline__ int64_t count_below_comp(const uint32_t *keys, const uint32_t *ids, int64_t m, uint64_t x)
{
    int64_t lo = 0, hi = m;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (comp(keys[mid], ids[mid]) < x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// The moved entries' old positions (found by their old (key, id) in the
// sorted arrays), their new keys, and the new coordinates.
__global__ void __launch_bounds__(256) dyn_prepare_kernel(DynArgs A, const int32_t *__restrict__ mid,
                                                          const double *__restrict__ mr,
                                                          const double *__restrict__ mt, int64_t k,
                                                          double *__restrict__ r, double *__restrict__ theta,
                                                          const uint32_t *__restrict__ okey,
                                                          const uint32_t *__restrict__ oid,
                                                          uint32_t *__restrict__ gone, uint32_t *__restrict__ nkey,
                                                          uint32_t *__restrict__ nid, uint32_t *__restrict__ gval,
                                                          int32_t *err)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= k) return;
    const int32_t id = mid[i];
    const uint32_t okk = point_key(A.E, A.B, A.band_bits, r[id], theta[id]);
    const int64_t p = count_below_comp(okey, oid, A.n, comp(okk, (uint32_t)id));
    if (p >= A.n || okey[p] != okk || oid[p] != (uint32_t)id) atomicOr(err, 4);  // only an inconsistent state
    const double ri = mr[i], ti = mt[i];
    r[id] = ri;
    theta[id] = ti;
    gone[i] = (uint32_t)min<int64_t>(p, A.n - 1);
    gval[i] = (uint32_t)id;
    nkey[i] = point_key(A.E, A.B, A.band_bits, ri, ti);
    nid[i] = (uint32_t)id;
}

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Step 2, unmoved entries: old position p -> p - (gone positions below p) +
// (new entries below p's (key, id)).  A wavefront takes 64 consecutive
// positions; where no gone position and no insertion point falls among them
// (almost everywhere for small batches) one shift serves all 64.
__global__ void __launch_bounds__(256) dyn_merge_old_kernel(
    int64_t n, int64_t k, const uint32_t *__restrict__ okey, const uint32_t *__restrict__ oid,
    const double *__restrict__ osr, const double *__restrict__ ost, const float4 *__restrict__ orec,
    const uint32_t *__restrict__ gone_s, const uint32_t *__restrict__ nkey_s, const uint32_t *__restrict__ nid_s,
    uint32_t *__restrict__ key2, uint32_t *__restrict__ id2, double *__restrict__ sr2, double *__restrict__ st2,
    float4 *__restrict__ rec2, int32_t *err)
{
    const int lane = threadIdx.x & 63;
    const int64_t wstride = (int64_t)gridDim.x * 256;
    for (int64_t base = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 64; base < n; base += wstride) {
        const int64_t last = min(base + 63, n - 1);
        const int64_t p = base + lane;
        const bool valid = p < n;
        const uint32_t key = valid ? okey[p] : 0u, id = valid ? oid[p] : 0u;
        // the wave's ends (every lane computes the same values)
        const int64_t g0 = count_below_u32(gone_s, k, (uint32_t)base);
        const int64_t g1 = count_below_u32(gone_s, k, (uint32_t)(last + 1));
        const int64_t i0 = count_below_comp(nkey_s, nid_s, k, comp(okey[base], oid[base]));
        const int64_t i1 = count_below_comp(nkey_s, nid_s, k, comp(okey[last], oid[last]));
        if (!valid) continue;
        int64_t gb = g0, ib = i0;
        if (g1 != g0) {  // a gone position among the 64
            gb = count_below_u32(gone_s, k, (uint32_t)p);
            if (gb < k && gone_s[gb] == (uint32_t)p) continue;  // a moved entry leaves
        }
        if (i1 != i0) ib = count_below_comp(nkey_s, nid_s, k, comp(key, id));
        const int64_t np = p - gb + ib;
        if (np < 0 || np >= n) {  // only an inconsistent state gets here
            atomicOr(err, 4);
            continue;
        }
        key2[np] = key;
        id2[np] = id;
        sr2[np] = osr[p];
        st2[np] = ost[p];
        rec2[np] = orec[p];
    }
}

// Step 2, new entries: rank i -> i + unmoved entries below.
__global__ void __launch_bounds__(256) dyn_merge_new_kernel(
    DynArgs A, int64_t k, const uint32_t *__restrict__ okey, const uint32_t *__restrict__ oid,
    const uint32_t *__restrict__ gone_s, const uint32_t *__restrict__ nkey_s, const uint32_t *__restrict__ nid_s,
    const double *__restrict__ r, const double *__restrict__ theta, uint32_t *__restrict__ key2,
    uint32_t *__restrict__ id2, double *__restrict__ sr2, double *__restrict__ st2, float4 *__restrict__ rec2,
    int32_t *__restrict__ qpos, int32_t *err)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= k) return;
    const uint32_t key = nkey_s[i], id = nid_s[i];
    const int64_t below = count_below_comp(okey, oid, A.n, comp(key, id));
    const int64_t np = i + below - count_below_u32(gone_s, k, (uint32_t)below);
    if (np < 0 || np >= A.n) {  // only an inconsistent state gets here
        atomicOr(err, 4);
        qpos[i] = 0;
        return;
    }
    const double ri = r[id], ti = theta[id];
    key2[np] = key;
    id2[np] = id;
    sr2[np] = ri;
    st2[np] = ti;
    rec2[np] = point_record(ri, id, A.inv, A.sc);
    qpos[i] = (int32_t)np;
}

// Appends v to the changed-row list the first time it is touched.
__device__ __forceinline__ void touch(int32_t *touched, int32_t *changed, unsigned long long *nchanged, int32_t v)
{
    if (atomicExch(&touched[v], 1) == 0) changed[atomicAdd(nchanged, 1ull)] = v;
}

// Step 4, losses: a wavefront per moved vertex walks its old row; each
// unmoved neighbour w loses u, recorded as the pair (w, u).
__global__ void __launch_bounds__(256) dyn_losses_kernel(const uint32_t *__restrict__ nid_s, int64_t k,
                                                         const int64_t *__restrict__ orp,
                                                         const int32_t *__restrict__ ocol,
                                                         const int32_t *__restrict__ moved, int32_t *__restrict__ rem,
                                                         int32_t *touched, int32_t *changed,
                                                         unsigned long long *counters, uint32_t *__restrict__ qv,
                                                         uint32_t *__restrict__ qu)
{
    const int lane = threadIdx.x & 63;
    const int64_t waves = (int64_t)gridDim.x * 4;
    for (int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); i < k; i += waves) {
        const uint32_t u = nid_s[i];
        const int64_t s = orp[u], e = orp[u + 1];
        for (int64_t x = s + lane; x < e; x += 64) {
            const int32_t w = ocol[x];
            if (moved[w]) continue;
            atomicAdd(&rem[w], 1);
            touch(touched, changed, &counters[0], w);
            const unsigned long long slot = atomicAdd(&counters[5], 1ull);
            qv[slot] = (uint32_t)w;
            qu[slot] = u;
        }
    }
}

// Before the losses: the old degrees of the moved vertices, summed (one
// atomic per workgroup) into *sum.
__global__ void __launch_bounds__(256) dyn_olddeg_kernel(const uint32_t *__restrict__ nid_s, int64_t k,
                                                         const int64_t *__restrict__ orp, unsigned long long *sum)
{
    __shared__ unsigned long long part[4];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    unsigned long long d = 0;
    if (i < k) {
        const uint32_t u = nid_s[i];
        d = (unsigned long long)(orp[u + 1] - orp[u]);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) d += __shfl_xor(d, o, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = d;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long t = part[0] + part[1] + part[2] + part[3];
        if (t) atomicAdd(sum, t);
    }
}

// Step 4, gains: a wavefront per moved vertex walks its new row; each
// unmoved neighbour v gains u, recorded as the pair (v, u).
__global__ void __launch_bounds__(256) dyn_gains_kernel(const uint32_t *__restrict__ nid_s, int64_t k,
                                                        const int64_t *__restrict__ mrp,
                                                        const int32_t *__restrict__ mcol,
                                                        const int32_t *__restrict__ moved, int32_t *__restrict__ add,
                                                        int32_t *touched, int32_t *changed,
                                                        unsigned long long *counters, uint32_t *__restrict__ pv,
                                                        uint32_t *__restrict__ pu)
{
    const int lane = threadIdx.x & 63;
    const int64_t waves = (int64_t)gridDim.x * 4;
    for (int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); i < k; i += waves) {
        const uint32_t u = nid_s[i];
        const int64_t s = mrp[i], e = mrp[i + 1];
        for (int64_t x = s + lane; x < e; x += 64) {
            const int32_t v = mcol[x];
            if (moved[v]) continue;
            atomicAdd(&add[v], 1);
            touch(touched, changed, &counters[0], v);
            const unsigned long long slot = atomicAdd(&counters[1], 1ull);
            pv[slot] = (uint32_t)v;
            pu[slot] = u;
        }
    }
}

// Step 5: new degrees into nrp[id + 1]; mrow[id] = the moved vertex's row in
// the moved rows' CSR.
__global__ void __launch_bounds__(256) dyn_degree_kernel(int64_t n, const int64_t *__restrict__ orp,
                                                         const int32_t *__restrict__ moved,
                                                         const int32_t *__restrict__ mrow,
                                                         const int64_t *__restrict__ mrp,
                                                         const int32_t *__restrict__ rem,
                                                         const int32_t *__restrict__ add, int64_t *__restrict__ nrp)
{
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x; v < n; v += stride) {
        int64_t d;
        if (moved[v]) {
            const int32_t i = mrow[v];
            d = mrp[i + 1] - mrp[i];
        } else {
            d = orp[v + 1] - orp[v] - rem[v] + add[v];
        }
        nrp[v + 1] = d;
        if (v == 0) nrp[0] = 0;
    }
}

__global__ void __launch_bounds__(256) dyn_mrow_kernel(const uint32_t *__restrict__ nid_s, int64_t k,
                                                       int32_t *__restrict__ mrow)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < k) mrow[nid_s[i]] = (int32_t)i;
}

// Pairs (v, u) sorted by v, then u: the segment of v.
__device__ __forceinline__ void pair_segment(const uint32_t *pv, int64_t m, uint32_t v, int64_t &s, int64_t &e)
{
    s = count_below_u32(pv, m, v);
    int64_t lo = s, hi = m;  // first entry above v
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (pv[mid] <= v) lo = mid + 1; else hi = mid;
    }
    e = lo;
}

constexpr int HUB_DEG = 2048;  // rows longer than this are rewritten in tiles
constexpr int HUB_TILE = 4096;

// The new place of entry e at old offset x of an unmoved row v whose old
// row starts at o and new row at nn: shifted by the row's move, and in a
// changed row corrected by the losses before it and the gains below it
// (losses qu[a..b), gains pu[c..d) of v, both ascending).  -1: e is lost.
__device__ __forceinline__ int64_t new_place(int64_t x, uint32_t e, int64_t o, int64_t nn, int changed, int64_t a,
                                             int64_t b, int64_t c, int64_t d, const uint32_t *qu, const uint32_t *pu)
{
    int64_t dst = nn + (x - o);
    if (changed) {
        const int64_t lost = a + count_below_u32(qu + a, b - a, e);
        if (lost < b && qu[lost] == e) return -1;
        dst += count_below_u32(pu + c, d - c, e) - (lost - a);
    }
    return dst;
}

// Step 5: every old entry of the unmoved rows, to its new place.  A
// wavefront takes 64 consecutive rows: with none changed, moved or long,
// their entries move by one shift (a straight copy); otherwise each entry
// finds its row among the 64 (offsets in LDS).  Rows longer than HUB_DEG
// are left to the tile pass (their tiles listed here).
__global__ void __launch_bounds__(256) dyn_rewrite_rows_kernel(
    int64_t n, const int64_t *__restrict__ orp, const int32_t *__restrict__ ocol, const int64_t *__restrict__ nrp,
    const int32_t *__restrict__ moved, const int32_t *__restrict__ touched, const uint32_t *__restrict__ qv,
    const uint32_t *__restrict__ qu, int64_t nq, const uint32_t *__restrict__ pv, const uint32_t *__restrict__ pu,
    int64_t np, int32_t *__restrict__ ncol, int2 *__restrict__ hub_tiles, unsigned long long *nhub_tiles)
{
    __shared__ int64_t so[4][65], sn[4][64];
    __shared__ int32_t kd[4][64];
    __shared__ int64_t sg[4][64][4];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t wstride = (int64_t)gridDim.x * 4;
    for (int64_t g = (int64_t)blockIdx.x * 4 + w; g * 64 < n; g += wstride) {
        const int64_t v = g * 64 + lane;
        const bool valid = v < n;
        const int64_t o = orp[valid ? v : n], o1 = valid ? orp[v + 1] : o;
        const int64_t nn = valid ? nrp[v] : 0;
        // 0 unchanged, 1 changed, 2 moved (written whole), 3 long (tiles)
        int kind = 0;
        if (valid) kind = moved[v] ? 2 : (o1 - o > HUB_DEG ? 3 : (touched[v] ? 1 : 0));
        if (kind == 3) {
            const int64_t nt = (o1 - o + HUB_TILE - 1) / HUB_TILE;
            const unsigned long long slot = atomicAdd(nhub_tiles, (unsigned long long)nt);
            for (int64_t t = 0; t < nt; ++t) hub_tiles[slot + t] = make_int2((int)v, (int)t);
        }
        const int64_t xs = __shfl(o, 0, 64), xe = __shfl(o1, 63, 64);
        if (__ballot(kind != 0) == 0) {  // 64 unchanged rows: one shift
            const int64_t shift = __shfl(nn, 0, 64) - xs;
            for (int64_t x = xs + lane; x < xe; x += 64) ncol[x + shift] = ocol[x];
            continue;
        }
        so[w][lane] = o;
        if (lane == 63) so[w][64] = o1;
        sn[w][lane] = nn;
        kd[w][lane] = kind;
        if (kind == 1) {
            int64_t a, b, c, d;
            pair_segment(qv, nq, (uint32_t)v, a, b);
            pair_segment(pv, np, (uint32_t)v, c, d);
            sg[w][lane][0] = a; sg[w][lane][1] = b; sg[w][lane][2] = c; sg[w][lane][3] = d;
        }
        wave_sync();
        // the entries between the long rows (which the tile pass takes)
        uint64_t longs = __ballot(kind == 3);
        int64_t from = xs;
        while (true) {
            int64_t to = xe, next = xe;
            if (longs) {
                const int h = __ffsll((unsigned long long)longs) - 1;
                to = so[w][h];
                next = so[w][h + 1];
                longs &= longs - 1;
            }
            for (int64_t x = from + lane; x < to; x += 64) {
                const uint32_t e = (uint32_t)ocol[x];
                int lo = 0, hi = 63;  // the last row with so[row] <= x
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (so[w][mid] <= x) lo = mid; else hi = mid - 1;
                }
                const int kk = kd[w][lo];
                if (kk >= 2) continue;
                const int64_t dst = new_place(x, e, so[w][lo], sn[w][lo], kk, sg[w][lo][0], sg[w][lo][1],
                                              sg[w][lo][2], sg[w][lo][3], qu, pu);
                if (dst >= 0) ncol[dst] = (int32_t)e;
            }
            if (to == xe) break;
            from = next;
        }
        wave_sync();  // the next group rewrites this wave's LDS
    }
}

// Step 5: the long rows, HUB_TILE entries a workgroup (tiles listed by the
// rows pass); a changed row's losses and gains are staged in LDS when they
// fit.
constexpr int HUB_SEG = 2048;

__global__ void __launch_bounds__(256) dyn_rewrite_hubs_kernel(
    const int64_t *__restrict__ orp, const int32_t *__restrict__ ocol, const int64_t *__restrict__ nrp,
    const int32_t *__restrict__ touched, const uint32_t *__restrict__ qv, const uint32_t *__restrict__ qu,
    int64_t nq, const uint32_t *__restrict__ pv, const uint32_t *__restrict__ pu, int64_t np,
    int32_t *__restrict__ ncol, const int2 *__restrict__ hub_tiles, const unsigned long long *nhub_tiles)
{
    __shared__ uint32_t sq[HUB_SEG], sp[HUB_SEG];
    const int64_t nt = (int64_t)*nhub_tiles;
    for (int64_t t = blockIdx.x; t < nt; t += gridDim.x) {
        const int2 tile = hub_tiles[t];
        const int64_t v = tile.x;
        const int64_t o = orp[v], o1 = orp[v + 1], nn = nrp[v];
        const int changed = touched[v] ? 1 : 0;
        int64_t a = 0, b = 0, c = 0, d = 0;
        if (changed) {
            pair_segment(qv, nq, (uint32_t)v, a, b);
            pair_segment(pv, np, (uint32_t)v, c, d);
        }
        const bool staged = changed && b - a <= HUB_SEG && d - c <= HUB_SEG;
        __syncthreads();  // the previous tile's reads of the staged lists are done
        if (staged) {
            for (int64_t i = threadIdx.x; i < b - a; i += 256) sq[i] = qu[a + i];
            for (int64_t i = threadIdx.x; i < d - c; i += 256) sp[i] = pu[c + i];
        }
        __syncthreads();
        const int64_t xs = o + (int64_t)tile.y * HUB_TILE, xe = min(o1, xs + HUB_TILE);
        for (int64_t x = xs + threadIdx.x; x < xe; x += 256) {
            const uint32_t e = (uint32_t)ocol[x];
            int64_t dst;
            if (staged) {
                const int64_t lost = count_below_u32(sq, b - a, e);
                if (lost < b - a && sq[lost] == e) continue;
                dst = nn + (x - o) + count_below_u32(sp, d - c, e) - lost;
            } else {
                dst = new_place(x, e, o, nn, changed, a, b, c, d, qu, pu);
                if (dst < 0) continue;
            }
            ncol[dst] = (int32_t)e;
        }
    }
}

// Large batches: the new coordinates only (the state is then regenerated).
__global__ void __launch_bounds__(256) dyn_apply_kernel(const int32_t *__restrict__ mid, const double *__restrict__ mr,
                                                        const double *__restrict__ mt, int64_t k,
                                                        double *__restrict__ r, double *__restrict__ theta,
                                                        int32_t *__restrict__ moved)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= k) return;
    const int32_t id = mid[i];
    r[id] = mr[i];
    theta[id] = mt[i];
    moved[id] = 0;
}

// Step 5: the gains.  Pair j = (v, u) of the sorted gains goes to v's new
// start + its rank among v's gains + v's old entries below u - v's losses
// below u.
__global__ void __launch_bounds__(256) dyn_gain_place_kernel(const int64_t *__restrict__ orp,
                                                             const int32_t *__restrict__ ocol,
                                                             const int64_t *__restrict__ nrp,
                                                             const uint32_t *__restrict__ qv,
                                                             const uint32_t *__restrict__ qu, int64_t nq,
                                                             const uint32_t *__restrict__ pv,
                                                             const uint32_t *__restrict__ pu, int64_t np,
                                                             int32_t *__restrict__ ncol)
{
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= np) return;
    const uint32_t v = pv[j], u = pu[j];
    int64_t a, b;
    pair_segment(pv, np, v, a, b);
    int64_t qa, qb;
    pair_segment(qv, nq, v, qa, qb);
    // old entries of row v below u (the old row ascends)
    int64_t lo = orp[v], hi = orp[v + 1];
    const int64_t s0 = lo;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((uint32_t)ocol[mid] < u) lo = mid + 1; else hi = mid;
    }
    const int64_t old_below = lo - s0;
    const int64_t lost_below = count_below_u32(qu + qa, qb - qa, u);
    ncol[nrp[v] + (j - a) + old_below - lost_below] = (int32_t)u;
}

// Step 5: the moved vertices' rows (sorted) into place, a wavefront each.
__global__ void __launch_bounds__(256) dyn_moved_place_kernel(const uint32_t *__restrict__ nid_s, int64_t k,
                                                              const int64_t *__restrict__ nrp,
                                                              const int64_t *__restrict__ mrp,
                                                              const int32_t *__restrict__ mcol,
                                                              int32_t *__restrict__ ncol)
{
    const int lane = threadIdx.x & 63;
    const int64_t waves = (int64_t)gridDim.x * 4;
    for (int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); i < k; i += waves) {
        const int64_t d = nrp[nid_s[i]], s = mrp[i], e = mrp[i + 1];
        for (int64_t x = s + lane; x < e; x += 64) ncol[d + (x - s)] = mcol[x];
    }
}

// After a step: the per-id marks of the changed rows and moved vertices.
__global__ void __launch_bounds__(256) dyn_clear_kernel(const int32_t *__restrict__ changed, int64_t nch,
                                                        const uint32_t *__restrict__ nid_s, int64_t k,
                                                        int32_t *__restrict__ touched, int32_t *__restrict__ rem,
                                                        int32_t *__restrict__ add, int32_t *__restrict__ moved)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < nch) {
        const int32_t v = changed[i];
        touched[v] = 0;
        rem[v] = 0;
        add[v] = 0;
    } else if (i < nch + k) {
        moved[nid_s[i - nch]] = 0;
    }
}

unsigned grid(int64_t n, int64_t cap = 65536)
{
    int64_t b = (n + 255) / 256;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, cap));
}

}  // namespace
}  // namespace rhg

using namespace rhg;

// A device buffer the state grows on demand.
struct DynBuf {
    void *p = nullptr;
    size_t bytes = 0;
    hipError_t need(size_t b)
    {
        if (b <= bytes) return hipSuccess;
        if (p) {
            hipError_t e = hipFree(p);
            if (e != hipSuccess) return e;
            p = nullptr;
            bytes = 0;
        }
        b = std::max<size_t>(b + b / 2, 4096);
        hipError_t e = hipMalloc(&p, b);
        if (e == hipSuccess) bytes = b;
        return e;
    }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
};

struct rhg_dyn {
    rhg_params p;
    int64_t n = 0;
    void *ws = nullptr;
    rhg_index *idx = nullptr;
    // the index's sorted arrays, double-buffered: the step merges into the
    // other set and swaps
    uint32_t *keys[2] = {nullptr, nullptr}, *ids[2] = {nullptr, nullptr};
    double *sr[2] = {nullptr, nullptr}, *st[2] = {nullptr, nullptr};
    float4 *rec[2] = {nullptr, nullptr};
    int cur_idx = 0;
    void *idx_alt = nullptr;           // allocation of the second set
    double *r = nullptr, *theta = nullptr;
    int32_t *moved = nullptr, *touched = nullptr, *rem = nullptr, *add = nullptr, *mrow = nullptr;
    int32_t *changed = nullptr;
    void *per_id = nullptr;            // allocation of the per-id arrays
    int64_t *row_ptr[2] = {nullptr, nullptr};
    DynBuf col[2];
    int cur = 0;
    int64_t nnz = 0;
    DynBuf step;                       // per-step scratch
    DynBuf mcolb, pairs, sortb, tiles;
    unsigned long long *counters = nullptr;  // [0] changed rows, [1] pairs, [2] error flag
    unsigned long long *host = nullptr;      // pinned copy of 4 values
    int64_t last_changed = 0, last_moved_entries = 0;
    double regen_share = 0.125;  // regenerate when k (1 + mean degree) exceeds this share of n
};

static DynArgs dyn_args(const rhg_dyn *d)
{
    DynArgs A;
    memset(&A, 0, sizeof(A));
    const Layout &L = d->idx->L;
    for (int j = 0; j <= L.B; ++j) A.E[j] = L.E[j];
    A.B = L.B;
    A.band_bits = L.band_bits;
    A.R = d->p.R;
    A.inv = 1.0 / sqrt(2.0 * d->p.cosh_R);
    A.sc = sqrt(2.0 / d->p.cosh_R);
    A.n = d->n;
    return A;
}

static void dyn_point_index(rhg_dyn *d)
{
    const int c = d->cur_idx;
    d->idx->keys = d->keys[c];
    d->idx->ids = d->ids[c];
    d->idx->sr = d->sr[c];
    d->idx->st = d->st[c];
    d->idx->rec = d->rec[c];
}

static rhg_status dyn_sync_read(rhg_dyn *d, const void *src, size_t bytes, hipStream_t s)
{
    RHG_HIP(hipMemcpyAsync(d->host, src, bytes, hipMemcpyDeviceToHost, s));
    RHG_HIP(hipStreamSynchronize(s));
    return RHG_OK;
}

extern "C" {

void rhg_dyn_free(rhg_dyn *d)
{
    if (!d) return;
    if (d->idx) rhg_index_free(d->idx);
    if (d->ws) (void)hipFree(d->ws);
    if (d->idx_alt) (void)hipFree(d->idx_alt);
    if (d->per_id) (void)hipFree(d->per_id);
    for (int b = 0; b < 2; ++b) {
        if (d->row_ptr[b]) (void)hipFree(d->row_ptr[b]);
        d->col[b].release();
    }
    d->step.release();
    d->mcolb.release();
    d->pairs.release();
    d->sortb.release();
    d->tiles.release();
    if (d->counters) (void)hipFree(d->counters);
    if (d->host) (void)hipHostFree(d->host);
    delete d;
}

rhg_status rhg_dyn_create(const rhg_params *p, const rhg_tuning *t, const double *r, const double *theta,
                          rhg_dyn **out, void *stream)
{
    if (!p || !out) return fail(RHG_EINVAL, "rhg_dyn_create: NULL argument");
    *out = nullptr;
    if (p->n < 1 || p->n > (int64_t)INT32_MAX) return fail(RHG_EINVAL, "rhg_dyn_create: n must lie in [1, 2^31 - 1]");
    if (!r || !theta) return fail(RHG_EINVAL, "rhg_dyn_create: NULL points");
    hipStream_t s = (hipStream_t)stream;
    rhg_dyn *d = new (std::nothrow) rhg_dyn;
    if (!d) return fail(RHG_ENOMEM, "rhg_dyn_create: host allocation failed");
    d->p = *p;
    const int64_t n = p->n;
    d->n = n;
    auto bail = [&](rhg_status st) {
        rhg_dyn_free(d);
        return st;
    };
    auto dev = [&](hipError_t e, const char *what) -> rhg_status {
        return e == hipSuccess ? RHG_OK : check_hip(e, what);
    };
    rhg_status st;
    // points, per-id arrays (moved, touched, rem, add, mrow, changed)
    const size_t pb = align_up((size_t)n * 8, 256);
    const size_t ib = align_up((size_t)n * 4, 256);
    if ((st = dev(hipMalloc(&d->per_id, 2 * pb + 6 * ib), "rhg_dyn_create (points)")) != RHG_OK) return bail(st);
    char *b = (char *)d->per_id;
    d->r = (double *)b; b += pb;
    d->theta = (double *)b; b += pb;
    int32_t **arrs[6] = {&d->moved, &d->touched, &d->rem, &d->add, &d->mrow, &d->changed};
    for (int a = 0; a < 6; ++a) { *arrs[a] = (int32_t *)b; b += ib; }
    if ((st = dev(hipMemcpyAsync(d->r, r, (size_t)n * 8, hipMemcpyDeviceToDevice, s), "rhg_dyn_create (copy)")) != RHG_OK)
        return bail(st);
    if ((st = dev(hipMemcpyAsync(d->theta, theta, (size_t)n * 8, hipMemcpyDeviceToDevice, s), "rhg_dyn_create (copy)")) !=
        RHG_OK)
        return bail(st);
    for (int a = 0; a < 5; ++a) hipLaunchKernelGGL(dyn_fill_i32, dim3(grid(n)), dim3(256), 0, s, *arrs[a], n, 0);
    // the index, validated once
    const size_t wsb = rhg_index_workspace_bytes(p, t);
    if (!wsb) return bail(fail(RHG_EINVAL, "rhg_dyn_create: invalid parameters"));
    if ((st = dev(hipMalloc(&d->ws, wsb), "rhg_dyn_create (index workspace)")) != RHG_OK) return bail(st);
    if ((st = rhg_build_index(p, d->r, d->theta, t, d->ws, wsb, 1, &d->idx, stream)) != RHG_OK) return bail(st);
    d->keys[0] = d->idx->keys;
    d->ids[0] = d->idx->ids;
    d->sr[0] = d->idx->sr;
    d->st[0] = d->idx->st;
    d->rec[0] = d->idx->rec;
    {
        const size_t kb = align_up((size_t)n * 4, 256), fb = align_up((size_t)n * 16, 256);
        if ((st = dev(hipMalloc(&d->idx_alt, 2 * kb + 2 * pb + fb), "rhg_dyn_create (index buffers)")) != RHG_OK)
            return bail(st);
        char *c = (char *)d->idx_alt;
        d->keys[1] = (uint32_t *)c; c += kb;
        d->ids[1] = (uint32_t *)c; c += kb;
        d->sr[1] = (double *)c; c += pb;
        d->st[1] = (double *)c; c += pb;
        d->rec[1] = (float4 *)c;
    }
    // the initial graph, rows ascending
    for (int c = 0; c < 2; ++c)
        if ((st = dev(hipMalloc(&d->row_ptr[c], (size_t)(n + 1) * 8), "rhg_dyn_create (row offsets)")) != RHG_OK)
            return bail(st);
    if ((st = rhg_count_edges(d->idx, d->row_ptr[0], stream)) != RHG_OK) return bail(st);
    if ((st = dev(hipHostMalloc((void **)&d->host, 64, hipHostMallocDefault), "rhg_dyn_create (pinned)")) != RHG_OK)
        return bail(st);
    if ((st = dev(hipMalloc((void **)&d->counters, 64), "rhg_dyn_create (counters)")) != RHG_OK) return bail(st);
    if ((st = dyn_sync_read(d, d->row_ptr[0] + n, 8, s)) != RHG_OK) return bail(st);
    const int64_t nnz = (int64_t)d->host[0];
    for (int c = 0; c < 2; ++c)
        if ((st = dev(d->col[c].need((size_t)std::max<int64_t>(nnz, 1) * 4), "rhg_dyn_create (columns)")) != RHG_OK)
            return bail(st);
    if ((st = rhg_emit_edges(d->idx, d->row_ptr[0], (int32_t *)d->col[0].p, nnz, 0, stream)) != RHG_OK)
        return bail(st);
    const size_t sb = rhg_sort_rows_workspace_bytes(n, nnz);
    if ((st = dev(d->sortb.need(sb), "rhg_dyn_create (row sort)")) != RHG_OK) return bail(st);
    if ((st = rhg_sort_rows(n, d->row_ptr[0], (int32_t *)d->col[0].p, nnz, d->sortb.p, d->sortb.bytes, stream)) !=
        RHG_OK)
        return bail(st);
    d->nnz = nnz;
    rhg_stats diag;
    if ((st = rhg_index_stats(d->idx, &diag, stream)) != RHG_OK) return bail(st);
    *out = d;
    return RHG_OK;
}

rhg_status rhg_dyn_graph(rhg_dyn *d, rhg_csr *out)
{
    if (!d || !out) return fail(RHG_EINVAL, "rhg_dyn_graph: NULL argument");
    memset(out, 0, sizeof(*out));
    out->n = d->n;
    out->nnz = d->nnz;
    out->row_ptr = d->row_ptr[d->cur];
    out->col_idx = (int32_t *)d->col[d->cur].p;
    out->r = d->r;
    out->theta = d->theta;
    out->params = d->p;
    return RHG_OK;
}

rhg_status rhg_dyn_set_regenerate_share(rhg_dyn *d, double share)
{
    if (!d) return fail(RHG_EINVAL, "rhg_dyn_set_regenerate_share: NULL state");
    if (!(share >= 0.0)) return fail(RHG_EINVAL, "rhg_dyn_set_regenerate_share: share must be >= 0");
    d->regen_share = share;
    return RHG_OK;
}

rhg_status rhg_dyn_last_step(rhg_dyn *d, int64_t *changed_rows, int64_t *moved_entries)
{
    if (!d) return fail(RHG_EINVAL, "rhg_dyn_last_step: NULL argument");
    if (changed_rows) *changed_rows = d->last_changed;
    if (moved_entries) *moved_entries = d->last_moved_entries;
    return RHG_OK;
}

rhg_status rhg_dyn_move(rhg_dyn *d, int64_t k, const int32_t *ids, const double *r, const double *theta,
                        void *stream)
{
    if (!d) return fail(RHG_EINVAL, "rhg_dyn_move: NULL state");
    if (k < 0 || k > d->n) return fail(RHG_EINVAL, "rhg_dyn_move: k must lie in [0, n]");
    if (k == 0) {
        d->last_changed = d->last_moved_entries = 0;
        return RHG_OK;
    }
    if (!ids || !r || !theta) return fail(RHG_EINVAL, "rhg_dyn_move: NULL moves");
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = d->n;
    const DynArgs A = dyn_args(d);
    rhg_status st;
    // per-step scratch: gone positions, new keys and ids (two sorted
    // copies), sort buffers, the moved rows' offsets and counts
    const size_t kb = align_up((size_t)k * 4, 256), k8 = align_up((size_t)(k + 1) * 8, 256);
    const size_t rst = align_up(radix_sort_tmp_bytes(k), 256);
    const size_t sct = align_up(scan_tmp_bytes(k + 1), 256);
    RHG_HIP(d->step.need(8 * kb + 2 * k8 + std::max(rst, sct)));
    char *b = (char *)d->step.p;
    uint32_t *gone = (uint32_t *)b; b += kb;
    uint32_t *gval = (uint32_t *)b; b += kb;
    uint32_t *nkey = (uint32_t *)b; b += kb;
    uint32_t *nid = (uint32_t *)b; b += kb;
    uint32_t *t1 = (uint32_t *)b; b += kb;
    uint32_t *t2 = (uint32_t *)b; b += kb;
    int32_t *qpos = (int32_t *)b; b += kb;
    b += kb;  // spare
    int64_t *mcnt = (int64_t *)b; b += 2 * k8;  // moved rows' lengths, then offsets (k + 1)
    void *tmp = b;
    // 1. checks and marks
    RHG_HIP(hipMemsetAsync(d->counters, 0, 64, s));
    hipLaunchKernelGGL(dyn_check_kernel, dim3(grid(k, 1 << 30)), dim3(256), 0, s, A, ids, r, theta, k, d->moved,
                       (int32_t *)&d->counters[2]);
    RHG_HIP(hipGetLastError());
    if ((st = dyn_sync_read(d, d->counters, 32, s)) != RHG_OK) return st;
    if (d->host[2]) {
        hipLaunchKernelGGL(dyn_unmark_kernel, dim3(grid(k, 1 << 30)), dim3(256), 0, s, A, ids, k, d->moved);
        RHG_HIP(hipGetLastError());
        RHG_HIP(hipStreamSynchronize(s));
        return fail(RHG_EINVAL, (d->host[2] & 2) ? "rhg_dyn_move: a vertex is listed twice"
                                                 : "rhg_dyn_move: an id or a coordinate is out of range");
    }
    // A batch that would touch a large share of the rows (k (1 + mean
    // degree) above regen_share n, 1/8 by default) is cheaper to regenerate:
    // new coordinates, index rebuilt, both passes, rows sorted.
    if ((double)k * (1.0 + (double)d->nnz / (double)n) > (double)n * d->regen_share) {
        hipLaunchKernelGGL(dyn_apply_kernel, dim3(grid(k, 1 << 30)), dim3(256), 0, s, ids, r, theta, k, d->r, d->theta,
                           d->moved);
        RHG_HIP(hipGetLastError());
        const int c = d->cur_idx;
        dyn_point_index(d);
        uint32_t *k1 = (uint32_t *)d->rec[c], *v1 = k1 + n;  // sort buffers in the record array, as the build does
        RHG_HIP(launch_build_index(d->idx, d->r, d->theta, k1, d->ids[c], v1, 0, s));
        int64_t *nrp = d->row_ptr[1 - d->cur];
        if ((st = rhg_count_edges(d->idx, nrp, stream)) != RHG_OK) return st;
        if ((st = dyn_sync_read(d, nrp + n, 8, s)) != RHG_OK) return st;
        const int64_t nnz = (int64_t)d->host[0];
        RHG_HIP(d->col[1 - d->cur].need((size_t)std::max<int64_t>(nnz, 1) * 4));
        int32_t *ncol = (int32_t *)d->col[1 - d->cur].p;
        if ((st = rhg_emit_edges(d->idx, nrp, ncol, nnz, 0, stream)) != RHG_OK) return st;
        RHG_HIP(d->sortb.need(rhg_sort_rows_workspace_bytes(n, nnz)));
        if ((st = rhg_sort_rows(n, nrp, ncol, nnz, d->sortb.p, d->sortb.bytes, stream)) != RHG_OK) return st;
        d->cur = 1 - d->cur;
        d->nnz = nnz;
        d->last_changed = n;
        d->last_moved_entries = nnz;
        return RHG_OK;
    }
    // 2. the index merge
    {
        const int c = d->cur_idx, o = 1 - c;
        hipLaunchKernelGGL(dyn_prepare_kernel, dim3(grid(k, 1 << 30)), dim3(256), 0, s, A, ids, r, theta, k, d->r,
                           d->theta, d->keys[c], d->ids[c], gone, nkey, nid, gval, (int32_t *)&d->counters[2]);
        RHG_HIP(hipGetLastError());
        RHG_HIP(radix_sort_pairs(gone, gval, t1, t2, k, 32, tmp, s));
        // (key, id) order: by id, then stably by key
        RHG_HIP(radix_sort_pairs(nid, nkey, t1, t2, k, 32, tmp, s));
        RHG_HIP(radix_sort_pairs(nkey, nid, t1, t2, k, 32, tmp, s));
        hipLaunchKernelGGL(dyn_merge_old_kernel, dim3(grid(n)), dim3(256), 0, s, n, k, d->keys[c], d->ids[c], d->sr[c],
                           d->st[c], d->rec[c], gone, nkey, nid, d->keys[o], d->ids[o], d->sr[o], d->st[o], d->rec[o],
                           (int32_t *)&d->counters[2]);
        hipLaunchKernelGGL(dyn_merge_new_kernel, dim3(grid(k, 1 << 30)), dim3(256), 0, s, A, k, d->keys[c], d->ids[c],
                           gone, nkey, nid, d->r, d->theta, d->keys[o], d->ids[o], d->sr[o], d->st[o], d->rec[o], qpos,
                           (int32_t *)&d->counters[2]);
        RHG_HIP(hipGetLastError());
        d->cur_idx = o;
        dyn_point_index(d);
        RHG_HIP(launch_index_directory(d->idx, s));
    }
    // 3. the moved vertices' rows on the updated index, and the sum of their
    // old degrees (which bounds their losses)
    const int64_t *orp = d->row_ptr[d->cur];
    const int32_t *ocol = (const int32_t *)d->col[d->cur].p;
    const int64_t onnz = d->nnz;
    RHG_HIP(launch_query_rows(d->idx, qpos, k, mcnt + 1, nullptr, nullptr, 0, s));
    RHG_HIP(hipMemsetAsync(mcnt, 0, 8, s));
    RHG_HIP(inclusive_scan_i64(mcnt + 1, k, tmp, s));
    RHG_HIP(hipMemcpyAsync(&d->counters[3], mcnt + k, 8, hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(dyn_olddeg_kernel, dim3(grid(k, 1 << 30)), dim3(256), 0, s, nid, k, orp, &d->counters[6]);
    RHG_HIP(hipGetLastError());
    if ((st = dyn_sync_read(d, d->counters, 56, s)) != RHG_OK) return st;
    if (d->host[2]) return fail(RHG_EINTERNAL, "rhg_dyn_move: the index merge found an inconsistent state");
    const int64_t mnnz = (int64_t)d->host[3], oldsum = (int64_t)d->host[6];
    RHG_HIP(d->mcolb.need((size_t)std::max<int64_t>(mnnz, 1) * 4));
    int32_t *mcol = (int32_t *)d->mcolb.p;
    RHG_HIP(launch_query_rows(d->idx, qpos, k, nullptr, mcnt, mcol, 1, s));
    // the moved rows ascending
    {
        const size_t sb = rhg_sort_rows_workspace_bytes(k, mnnz);
        RHG_HIP(d->sortb.need(sb));
        if ((st = rhg_sort_rows(k, mcnt, mcol, mnnz, d->sortb.p, d->sortb.bytes, stream)) != RHG_OK) return st;
    }
    // 4. losses (pairs (w, u), at most oldsum) and gains (pairs (v, u), at
    // most mnnz), each sorted by vertex, then moved neighbour
    const int64_t pmax = std::max<int64_t>(std::max(oldsum, mnnz), 1);
    const size_t qb = align_up((size_t)std::max<int64_t>(oldsum, 1) * 4, 256);
    const size_t pb = align_up((size_t)std::max<int64_t>(mnnz, 1) * 4, 256);
    const size_t xb = align_up((size_t)pmax * 4, 256);
    const size_t prst = align_up(radix_sort_tmp_bytes(pmax), 256);
    RHG_HIP(d->pairs.need(2 * qb + 2 * pb + 2 * xb + prst));
    char *pp = (char *)d->pairs.p;
    uint32_t *qv = (uint32_t *)pp; pp += qb;
    uint32_t *qu = (uint32_t *)pp; pp += qb;
    uint32_t *pv = (uint32_t *)pp; pp += pb;
    uint32_t *pu = (uint32_t *)pp; pp += pb;
    uint32_t *x1 = (uint32_t *)pp; pp += xb;
    uint32_t *x2 = (uint32_t *)pp; pp += xb;
    void *ptmp = pp;
    const unsigned gw = (unsigned)std::min<int64_t>((k + 3) / 4, 16384);
    hipLaunchKernelGGL(dyn_losses_kernel, dim3(gw), dim3(256), 0, s, nid, k, orp, ocol, d->moved, d->rem, d->touched,
                       d->changed, d->counters, qv, qu);
    hipLaunchKernelGGL(dyn_gains_kernel, dim3(gw), dim3(256), 0, s, nid, k, mcnt, mcol, d->moved, d->add, d->touched,
                       d->changed, d->counters, pv, pu);
    hipLaunchKernelGGL(dyn_mrow_kernel, dim3(grid(k, 1 << 30)), dim3(256), 0, s, nid, k, d->mrow);
    // 5. new offsets
    int64_t *nrp = d->row_ptr[1 - d->cur];
    hipLaunchKernelGGL(dyn_degree_kernel, dim3(grid(n)), dim3(256), 0, s, n, orp, d->moved, d->mrow, mcnt, d->rem,
                       d->add, nrp);
    RHG_HIP(hipGetLastError());
    RHG_HIP(inclusive_scan_i64(nrp + 1, n, d->idx->tmp, s));
    RHG_HIP(hipMemcpyAsync(&d->counters[4], nrp + n, 8, hipMemcpyDeviceToDevice, s));
    if ((st = dyn_sync_read(d, d->counters, 48, s)) != RHG_OK) return st;
    const int64_t nch = (int64_t)d->host[0], npairs = (int64_t)d->host[1], nnz = (int64_t)d->host[4];
    const int64_t nloss = (int64_t)d->host[5];
    RHG_HIP(d->col[1 - d->cur].need((size_t)std::max<int64_t>(nnz, 1) * 4));
    int32_t *ncol = (int32_t *)d->col[1 - d->cur].p;
    // (vertex, moved neighbour) order: by neighbour, then stably by vertex
    RHG_HIP(radix_sort_pairs(qu, qv, x1, x2, nloss, 32, ptmp, s));
    RHG_HIP(radix_sort_pairs(qv, qu, x1, x2, nloss, 32, ptmp, s));
    RHG_HIP(radix_sort_pairs(pu, pv, x1, x2, npairs, 32, ptmp, s));
    RHG_HIP(radix_sort_pairs(pv, pu, x1, x2, npairs, 32, ptmp, s));
    // every old entry but the moved rows', the gains, the moved rows
    if (onnz > 0) {
        RHG_HIP(d->tiles.need((size_t)(onnz / HUB_TILE + onnz / HUB_DEG + 2) * 8));
        int2 *hub_tiles = (int2 *)d->tiles.p;
        hipLaunchKernelGGL(dyn_rewrite_rows_kernel, dim3(grid((n + 63) / 64 * 64, 65536)), dim3(256), 0, s, n, orp,
                           ocol, nrp, d->moved, d->touched, qv, qu, nloss, pv, pu, npairs, ncol, hub_tiles,
                           &d->counters[7]);
        hipLaunchKernelGGL(dyn_rewrite_hubs_kernel, dim3(2048), dim3(256), 0, s, orp, ocol, nrp, d->touched, qv, qu,
                           nloss, pv, pu, npairs, ncol, (const int2 *)hub_tiles, (const unsigned long long *)&d->counters[7]);
        RHG_HIP(hipGetLastError());
    }
    if (npairs > 0)
        hipLaunchKernelGGL(dyn_gain_place_kernel, dim3((unsigned)((npairs + 255) / 256)), dim3(256), 0, s, orp, ocol,
                           nrp, qv, qu, nloss, pv, pu, npairs, ncol);
    hipLaunchKernelGGL(dyn_moved_place_kernel, dim3(gw), dim3(256), 0, s, nid, k, nrp, mcnt, mcol, ncol);
    hipLaunchKernelGGL(dyn_clear_kernel, dim3(grid(nch + k, 1 << 30)), dim3(256), 0, s, d->changed, nch, nid, k,
                       d->touched, d->rem, d->add, d->moved);
    RHG_HIP(hipGetLastError());
    d->cur = 1 - d->cur;
    d->nnz = nnz;
    d->last_changed = nch + k;
    d->last_moved_entries = mnnz;
    return RHG_OK;
}

}  // extern "C"
