// Device BVH build for a triangle scene (Sec. III-B scenes; the paper rasterises,
// this path ray casts, so the scene needs an acceleration structure).
//
// Pipeline (all on the caller's stream, one scene at a time):
//   1. tri_prep      per-triangle bounds and centroid, block partial bounds
//   2. reduce        centroid and scene bounds
//   3. morton        30-bit Morton code of the centroid quantised in the cube around
//                    all centroids (one scale for the three axes), value = index
//   4. radix sort    stable LSD, 8-bit digits, 4 passes (histogram / scan / scatter)
//   5. radix tree    binary radix tree over the sorted codes (Karras, HPG 2012),
//                    duplicate codes split by index; parent links, then the binary
//                    boxes bottom-up (one climb per leaf, the second arrival goes on)
//   6. collapse      level by level: each wide node takes the two children of its
//                    binary node and opens the child of largest surface area among
//                    those too big for a leaf until it has kWidth; free slots are then
//                    filled by splitting leaf-sized subtrees; children with <= leaf_max
//                    triangles become leaves (a contiguous sorted range)
//   7. bounds        bottom-up per level (deepest first), leaf boxes padded by a
//                    few ulps, plus per-octant near-to-far child orders
//   8. triangles     (v0, e1, e2, caller id) in sorted order, id -> position map
// Node indices are assigned by prefix sums, so a rebuild of the same input is
// bitwise identical.
#include <float.h>

#include "vf_internal.h"

namespace vf {

namespace {

constexpr int kScanThreads = 1024;
constexpr int kSortThreads = 256;
constexpr int kSortItems = 8;
constexpr int kSortTile = kSortThreads * kSortItems;   // 2048 keys per block
constexpr int kPrepThreads = 256;

__device__ __forceinline__ uint32_t expand_bits10(uint32_t v) {
    v = (v * 0x00010001u) & 0xFF0000FFu;
    v = (v * 0x00000101u) & 0x0F00F00Fu;
    v = (v * 0x00000011u) & 0xC30C30C3u;
    v = (v * 0x00000005u) & 0x49249249u;
    return v;
}

__global__ void k_tri_prep(const float* __restrict__ verts, int64_t nv, const int32_t* __restrict__ tris, int32_t nt,
                           float4* __restrict__ tlo, float4* __restrict__ thi, float4* __restrict__ cen,
                           float* __restrict__ partial, uint32_t* __restrict__ err) {
    __shared__ float red[6][kPrepThreads];
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    float clo[3] = {FLT_MAX, FLT_MAX, FLT_MAX}, chi[3] = {-FLT_MAX, -FLT_MAX, -FLT_MAX};
    if (t < nt) {
        int32_t ia = tris[3 * t], ib = tris[3 * t + 1], ic = tris[3 * t + 2];
        bool ok = ia >= 0 && ib >= 0 && ic >= 0 && ia < nv && ib < nv && ic < nv;
        if (!ok) {
            atomicOr(err, kErrTriIndex);
            ia = ib = ic = 0;
        }
        float a[3], b[3], c[3], lo[3], hi[3], ce[3];
        for (int k = 0; k < 3; ++k) {
            a[k] = verts[3 * (int64_t)ia + k];
            b[k] = verts[3 * (int64_t)ib + k];
            c[k] = verts[3 * (int64_t)ic + k];
            if (!(isfinite(a[k]) && isfinite(b[k]) && isfinite(c[k]))) {
                atomicOr(err, kErrVertex);
                a[k] = b[k] = c[k] = 0.f;   // keep the rest of the build finite until it is rejected
            }
            lo[k] = fminf(a[k], fminf(b[k], c[k]));
            hi[k] = fmaxf(a[k], fmaxf(b[k], c[k]));
            ce[k] = 0.5f * lo[k] + 0.5f * hi[k];   // box centre: robust for degenerate triangles
            clo[k] = ce[k];
            chi[k] = ce[k];
        }
        tlo[t] = make_float4(lo[0], lo[1], lo[2], 0.f);
        thi[t] = make_float4(hi[0], hi[1], hi[2], 0.f);
        cen[t] = make_float4(ce[0], ce[1], ce[2], 0.f);
    }
    for (int k = 0; k < 3; ++k) {
        red[k][threadIdx.x] = clo[k];
        red[3 + k][threadIdx.x] = chi[k];
    }
    __syncthreads();
    for (int s = kPrepThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            for (int k = 0; k < 3; ++k) {
                red[k][threadIdx.x] = fminf(red[k][threadIdx.x], red[k][threadIdx.x + s]);
                red[3 + k][threadIdx.x] = fmaxf(red[3 + k][threadIdx.x], red[3 + k][threadIdx.x + s]);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < 6) partial[blockIdx.x * 6 + threadIdx.x] = red[threadIdx.x][0];
}

// Single block: reduce block partials (centroid bounds) and the triangle boxes (scene bounds).
__global__ void k_reduce_bounds(const float* __restrict__ partial, int nblocks, const float4* __restrict__ tlo,
                                const float4* __restrict__ thi, int32_t nt, float* __restrict__ out /*12*/) {
    __shared__ float red[12][kScanThreads];
    float v[12];
    for (int k = 0; k < 3; ++k) { v[k] = FLT_MAX; v[3 + k] = -FLT_MAX; v[6 + k] = FLT_MAX; v[9 + k] = -FLT_MAX; }
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x)
        for (int k = 0; k < 3; ++k) {
            v[k] = fminf(v[k], partial[6 * b + k]);
            v[3 + k] = fmaxf(v[3 + k], partial[6 * b + 3 + k]);
        }
    for (int t = threadIdx.x; t < nt; t += blockDim.x) {
        float4 lo = tlo[t], hi = thi[t];
        v[6] = fminf(v[6], lo.x); v[7] = fminf(v[7], lo.y); v[8] = fminf(v[8], lo.z);
        v[9] = fmaxf(v[9], hi.x); v[10] = fmaxf(v[10], hi.y); v[11] = fmaxf(v[11], hi.z);
    }
    for (int k = 0; k < 12; ++k) red[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int s = kScanThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int k = 0; k < 12; ++k) {
                bool is_min = (k < 3) || (k >= 6 && k < 9);
                float a = red[k][threadIdx.x], b = red[k][threadIdx.x + s];
                red[k][threadIdx.x] = is_min ? fminf(a, b) : fmaxf(a, b);
            }
        __syncthreads();
    }
    if (threadIdx.x < 12) out[threadIdx.x] = red[threadIdx.x][0];
}

__global__ void k_morton(const float4* __restrict__ cen, int32_t nt, const float* __restrict__ bounds,
                         uint32_t* __restrict__ keys, uint32_t* __restrict__ vals) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt) return;
    float4 c = cen[t];
    float lo[3] = {bounds[0], bounds[1], bounds[2]};
    float ext[3] = {bounds[3] - lo[0], bounds[4] - lo[1], bounds[5] - lo[2]};
    // one scale for all axes (the cube around the centroids): a flat scene is then split along its
    // long axes first, not the same number of times along each axis
    const float e = fmaxf(ext[0], fmaxf(ext[1], ext[2]));
    ext[0] = ext[1] = ext[2] = e;
    float cc[3] = {c.x, c.y, c.z};
    uint32_t q[3];
    for (int k = 0; k < 3; ++k) {
        float u = ext[k] > 0.f ? (cc[k] - lo[k]) / ext[k] : 0.f;
        u = fminf(fmaxf(u * 1024.0f, 0.0f), 1023.0f);
        q[k] = (uint32_t)u;
    }
    keys[t] = (expand_bits10(q[0]) << 2) | (expand_bits10(q[1]) << 1) | expand_bits10(q[2]);
    vals[t] = (uint32_t)t;
}

// ---------------------------------------------------------------------------
// exclusive scan (single workgroup; used for the sort histograms and the collapse)
// ---------------------------------------------------------------------------
template <class T>
__global__ void k_scan_exclusive(const T* __restrict__ in, T* __restrict__ out, int64_t n, T* __restrict__ total) {
    __shared__ T sums[kScanThreads];
    int64_t chunk = (n + kScanThreads - 1) / kScanThreads;
    int64_t b = threadIdx.x * chunk, e = b + chunk < n ? b + chunk : n;
    T s = 0;
    for (int64_t i = b; i < e; ++i) s += in[i];
    sums[threadIdx.x] = s;
    __syncthreads();
    // Hillis-Steele inclusive scan of the chunk sums
    for (int off = 1; off < kScanThreads; off <<= 1) {
        T v = (int)threadIdx.x >= off ? sums[threadIdx.x - off] : (T)0;
        __syncthreads();
        sums[threadIdx.x] += v;
        __syncthreads();
    }
    T run = threadIdx.x > 0 ? sums[threadIdx.x - 1] : (T)0;
    for (int64_t i = b; i < e; ++i) {
        T v = in[i];
        out[i] = run;
        run += v;
    }
    if (threadIdx.x == kScanThreads - 1 && total) *total = sums[kScanThreads - 1];
}

// Multi-workgroup exclusive scan for long arrays: the sum of each tile of kScanTile elements, an
// exclusive scan of the tile sums (one workgroup), then each tile scanned with its offset.
constexpr int kScanTile = 4 * kScanThreads;

template <class T>
__global__ void __launch_bounds__(kScanThreads) k_tile_sums(const T* __restrict__ in, int64_t n, T* __restrict__ sums) {
    __shared__ T red[kScanThreads];
    const int64_t i0 = (int64_t)blockIdx.x * kScanTile + 4 * (int64_t)threadIdx.x;
    T v = 0;
    for (int j = 0; j < 4; ++j)
        if (i0 + j < n) v += in[i0 + j];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = kScanThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) sums[blockIdx.x] = red[0];
}

template <class T>
__global__ void __launch_bounds__(kScanThreads) k_tile_scan(const T* __restrict__ in, int64_t n,
                                                             const T* __restrict__ tile_off, T* __restrict__ out) {
    __shared__ T sums[kScanThreads];
    const int64_t i0 = (int64_t)blockIdx.x * kScanTile + 4 * (int64_t)threadIdx.x;
    T v[4];
    T s = 0;
    for (int j = 0; j < 4; ++j) {
        v[j] = i0 + j < n ? in[i0 + j] : (T)0;
        s += v[j];
    }
    sums[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {   // Hillis-Steele inclusive scan of the thread sums
        T u = (int)threadIdx.x >= off ? sums[threadIdx.x - off] : (T)0;
        __syncthreads();
        sums[threadIdx.x] += u;
        __syncthreads();
    }
    T run = tile_off[blockIdx.x] + (threadIdx.x > 0 ? sums[threadIdx.x - 1] : (T)0);
    for (int j = 0; j < 4; ++j) {
        if (i0 + j < n) out[i0 + j] = run;
        run += v[j];
    }
}

// ---------------------------------------------------------------------------
// stable LSD radix sort of (key, value) pairs, 8-bit digits
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kSortThreads) k_sort_hist(const uint32_t* __restrict__ keys, int32_t n, int shift,
                                                            uint32_t* __restrict__ hist, int nblocks) {
    __shared__ uint32_t cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int j = 0; j < kSortItems; ++j) {
        int64_t e = base + j * kSortThreads + threadIdx.x;
        if (e < n) atomicAdd(&cnt[(keys[e] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = cnt[threadIdx.x];
}

// Each wave owns 512 consecutive keys of the block's tile (8 rows of 64) so the
// in-tile order is (wave, row, lane); ranks among equal digits follow that order.
__global__ void __launch_bounds__(kSortThreads) k_sort_scatter(const uint32_t* __restrict__ kin,
                                                               const uint32_t* __restrict__ vin,
                                                               uint32_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                                               int32_t n, int shift,
                                                               const uint32_t* __restrict__ offsets, int nblocks) {
    __shared__ uint32_t wrun[kSortThreads / kWave][256];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int d = lane; d < 256; d += 64) wrun[wave][d] = 0;
    __syncthreads();
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int64_t wbase = (int64_t)blockIdx.x * kSortTile + wave * (kSortItems * kWave);
    uint32_t key[kSortItems], val[kSortItems], rank[kSortItems];
    for (int j = 0; j < kSortItems; ++j) {
        int64_t e = wbase + j * kWave + lane;
        bool valid = e < n;
        key[j] = valid ? kin[e] : 0u;
        val[j] = valid ? vin[e] : 0u;
        uint32_t dig = (key[j] >> shift) & 255u;
        uint64_t peers = __ballot(valid);
        for (int b = 0; b < 8; ++b) {
            bool bit = (dig >> b) & 1u;
            uint64_t m = __ballot(valid && bit);
            peers &= bit ? m : ~m;
        }
        uint32_t before = wrun[wave][dig];
        rank[j] = before + (uint32_t)__popcll(peers & lt);
        // the highest lane of each peer group advances the running count
        bool leader = valid && ((peers >> lane) >> 1) == 0ull;
        __builtin_amdgcn_wave_barrier();
        if (leader) wrun[wave][dig] = before + (uint32_t)__popcll(peers);
        __builtin_amdgcn_wave_barrier();
        if (!valid) rank[j] = 0xFFFFFFFFu;
    }
    __syncthreads();
    // exclusive prefix over waves, per digit
    {
        int d = threadIdx.x;
        uint32_t s = 0;
        for (int w = 0; w < kSortThreads / kWave; ++w) {
            uint32_t c = wrun[w][d];
            wrun[w][d] = s;
            s += c;
        }
    }
    __syncthreads();
    for (int j = 0; j < kSortItems; ++j) {
        if (rank[j] == 0xFFFFFFFFu) continue;
        uint32_t dig = (key[j] >> shift) & 255u;
        uint32_t pos = offsets[(int64_t)dig * nblocks + blockIdx.x] + wrun[wave][dig] + rank[j];
        kout[pos] = key[j];
        vout[pos] = val[j];
    }
}

// ---------------------------------------------------------------------------
// binary radix tree (Karras 2012): internal node i covers [first, last]
// ---------------------------------------------------------------------------
__device__ __forceinline__ int common_prefix(const uint32_t* __restrict__ k, int n, int i, int j) {
    if (j < 0 || j >= n) return -1;
    uint32_t a = k[i], b = k[j];
    if (a == b) return 32 + __clz((uint32_t)(i ^ j));
    return __clz(a ^ b);
}

__global__ void k_radix_tree(const uint32_t* __restrict__ k, int32_t n, int32_t* __restrict__ left,
                             int32_t* __restrict__ right, int32_t* __restrict__ first, int32_t* __restrict__ last) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n - 1) return;
    int d = (common_prefix(k, n, i, i + 1) - common_prefix(k, n, i, i - 1)) >= 0 ? 1 : -1;
    int dmin = common_prefix(k, n, i, i - d);
    int lmax = 2;
    while (common_prefix(k, n, i, i + lmax * d) > dmin) lmax <<= 1;
    int l = 0;
    for (int t = lmax >> 1; t >= 1; t >>= 1)
        if (common_prefix(k, n, i, i + (l + t) * d) > dmin) l += t;
    int j = i + l * d;
    int dnode = common_prefix(k, n, i, j);
    int s = 0, t = l;
    do {
        t = (t + 1) >> 1;
        if (common_prefix(k, n, i, i + (s + t) * d) > dnode) s += t;
    } while (t > 1);
    int gamma = i + s * d + (d < 0 ? -1 : 0);
    int lo = i < j ? i : j, hi = i < j ? j : i;
    left[i] = (lo == gamma) ? -(gamma + 1) : gamma;
    right[i] = (hi == gamma + 1) ? -(gamma + 2) : gamma + 1;
    first[i] = lo;
    last[i] = hi;
}

// Parent links of the binary radix tree (-1 above the root).
__global__ void k_parents(const int32_t* __restrict__ left, const int32_t* __restrict__ right, int32_t n,
                          int32_t* __restrict__ par_int, int32_t* __restrict__ par_leaf) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n - 1) return;
    if (i == 0) par_int[0] = -1;
    int32_t l = left[i], r = right[i];
    if (l >= 0) par_int[l] = i; else par_leaf[-l - 1] = i;
    if (r >= 0) par_int[r] = i; else par_leaf[-r - 1] = i;
}

// Boxes of the binary tree's inner nodes, bottom-up: one thread per leaf climbs while it is the
// second of the two children to arrive at a node (an atomic counter per node), so every node is
// written once, after both children.  Unions of min/max are exact: the result does not depend on
// the arrival order.
__global__ void k_binary_bounds(const int32_t* __restrict__ left, const int32_t* __restrict__ right, int32_t n,
                                const uint32_t* __restrict__ sorted_vals, const float4* __restrict__ tlo,
                                const float4* __restrict__ thi, const int32_t* __restrict__ par_int,
                                const int32_t* __restrict__ par_leaf, uint32_t* __restrict__ flags, float4* nlo,
                                float4* nhi) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    int32_t p = par_leaf[j];
    while (p >= 0) {
        __threadfence();
        if (atomicAdd(&flags[p], 1u) == 0u) return;
        __threadfence();
        float l[3] = {FLT_MAX, FLT_MAX, FLT_MAX}, h[3] = {-FLT_MAX, -FLT_MAX, -FLT_MAX};
        for (int side = 0; side < 2; ++side) {
            int32_t c = side == 0 ? left[p] : right[p];
            float a[3], b[3];
            if (c >= 0) {
                const volatile float* vl = (const volatile float*)(nlo + c);
                const volatile float* vh = (const volatile float*)(nhi + c);
                for (int k = 0; k < 3; ++k) { a[k] = vl[k]; b[k] = vh[k]; }
            } else {
                uint32_t t = sorted_vals[-c - 1];
                float4 x = tlo[t], y = thi[t];
                a[0] = x.x; a[1] = x.y; a[2] = x.z;
                b[0] = y.x; b[1] = y.y; b[2] = y.z;
            }
            for (int k = 0; k < 3; ++k) { l[k] = fminf(l[k], a[k]); h[k] = fmaxf(h[k], b[k]); }
        }
        nlo[p] = make_float4(l[0], l[1], l[2], 0.f);
        nhi[p] = make_float4(h[0], h[1], h[2], 0.f);
        p = par_int[p];
    }
}

// ---------------------------------------------------------------------------
// binary tree by locally-ordered clustering (PLOC: Meister and Bittner, IEEE TVCG 2018).
// Clusters start as the leaves in Morton order.  Each pass, every cluster finds the
// neighbour within kPlocRadius positions whose merged box has the smallest surface
// area; mutual pairs merge into a new inner node placed at the lower position, and
// the cluster array is compacted.  Pairs are ordered by area, then by a symmetric
// tie order (see tie_before), so the globally best pair is always mutual and every
// pass merges at least once.  Inner nodes are numbered by pass and prefix sum (deterministic); a node's
// children are always from earlier passes, which the top-down range pass relies on.
// Child references: inner node k >= 0, leaf -(i + 1) for Morton position i; after
// the range pass leaves are renumbered to depth-first order, so every subtree is a
// contiguous range of the leaf array (what the collapse and the leaf encoding need).
// ---------------------------------------------------------------------------
#ifndef VF_PLOC_RADIUS
#define VF_PLOC_RADIUS 6
#endif
constexpr int kPlocRadius = VF_PLOC_RADIUS;

__device__ __forceinline__ float merged_area(float4 alo, float4 ahi, float4 blo, float4 bhi) {
    const float dx = fmaxf(ahi.x, bhi.x) - fminf(alo.x, blo.x);
    const float dy = fmaxf(ahi.y, bhi.y) - fminf(alo.y, blo.y);
    const float dz = fmaxf(ahi.z, bhi.z) - fminf(alo.z, blo.z);
    return dx * dy + dy * dz + dz * dx;
}

__global__ void k_ploc_init(const uint32_t* __restrict__ sorted_vals, int32_t nt, const float4* __restrict__ tlo,
                            const float4* __restrict__ thi, int32_t* __restrict__ cid, float4* __restrict__ clo,
                            float4* __restrict__ chi) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nt) return;
    const uint32_t t = sorted_vals[i];
    cid[i] = -(i + 1);
    clo[i] = tlo[t];
    chi[i] = thi[t];
}

// Order of the pairs (i, j) and (i, k) of equal merged area.  Normally the lower other index first
// (the pair order (area, lower index, higher index)).  That merges a run of identical boxes one pair
// per pass, so after a pass that merged under 1/32 of the clusters the next pass orders ties by index
// distance, then the fixed buddy i ^ 1, then the lower index: identical boxes pair off as buddies.
// Either order is symmetric in the pair and total with the area first, so the least pair is chosen by
// both its members and every pass merges.
__device__ __forceinline__ bool tie_before(int i, int j, int k) {
    const int dj = j > i ? j - i : i - j, dk = k > i ? k - i : i - k;
    if (dj != dk) return dj < dk;
    const bool bj = j == (i ^ 1), bk = k == (i ^ 1);
    if (bj != bk) return bj;
    return j < k;
}

// nearest neighbour of each of the m >= 2 clusters: least merged surface area; equal areas by the lower
// index, or by tie_before when spread_ties is set
__global__ void k_ploc_nn(int32_t m, const float4* __restrict__ clo, const float4* __restrict__ chi,
                          int32_t spread_ties, int32_t* __restrict__ nn) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const float4 l = clo[i], h = chi[i];
    const int j0 = i - kPlocRadius > 0 ? i - kPlocRadius : 0;
    const int j1 = i + kPlocRadius < m - 1 ? i + kPlocRadius : m - 1;
    int bj = -1;
    float ba = 0.f;
    for (int j = j0; j <= j1; ++j) {
        if (j == i) continue;
        const float a = merged_area(l, h, clo[j], chi[j]);
        if (bj < 0 || a < ba || (spread_ties && a == ba && tie_before(i, j, bj))) { ba = a; bj = j; }
    }
    nn[i] = bj;   // m >= 2: some j exists
}

// per cluster: bit 32 = it survives the pass, bit 0 = it is the lower member of a mutual pair
__global__ void k_ploc_flags(int32_t m, const int32_t* __restrict__ nn, uint64_t* __restrict__ fl) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const int32_t j = nn[i];
    const bool mutual = nn[j] == i;
    const uint64_t keep = (mutual && j < i) ? 0u : 1u;
    const uint64_t merge = (mutual && i < j) ? 1u : 0u;
    fl[i] = (keep << 32) | merge;
}

__global__ void k_ploc_merge(int32_t m, const int32_t* __restrict__ nn, const uint64_t* __restrict__ fl,
                             const uint64_t* __restrict__ pre, int32_t node_base, const int32_t* __restrict__ cid,
                             const float4* __restrict__ clo, const float4* __restrict__ chi,
                             int32_t* __restrict__ cid2, float4* __restrict__ clo2, float4* __restrict__ chi2,
                             int32_t* __restrict__ left, int32_t* __restrict__ right, int32_t* __restrict__ cnt,
                             float4* __restrict__ nlo, float4* __restrict__ nhi) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const uint64_t f = fl[i];
    if (!(f >> 32)) return;
    const int32_t pos = (int32_t)(pre[i] >> 32);
    if (f & 1u) {
        const int32_t j = nn[i];
        const int32_t k = node_base + (int32_t)(pre[i] & 0xffffffffu);
        const int32_t a = cid[i], b = cid[j];
        const float4 al = clo[i], ah = chi[i], bl = clo[j], bh = chi[j];
        const float4 lo = make_float4(fminf(al.x, bl.x), fminf(al.y, bl.y), fminf(al.z, bl.z), 0.f);
        const float4 hi = make_float4(fmaxf(ah.x, bh.x), fmaxf(ah.y, bh.y), fmaxf(ah.z, bh.z), 0.f);
        left[k] = a;
        right[k] = b;
        cnt[k] = (a >= 0 ? cnt[a] : 1) + (b >= 0 ? cnt[b] : 1);
        nlo[k] = lo;
        nhi[k] = hi;
        cid2[pos] = k;
        clo2[pos] = lo;
        chi2[pos] = hi;
    } else {
        cid2[pos] = cid[i];
        clo2[pos] = clo[i];
        chi2[pos] = chi[i];
    }
}

// top-down: the inner nodes of one pass [k0, k1) hand their depth-first leaf offsets to their children
__global__ void k_ploc_offsets(int32_t k0, int32_t k1, const int32_t* __restrict__ left,
                               const int32_t* __restrict__ right, const int32_t* __restrict__ cnt,
                               int32_t* __restrict__ off, int32_t* __restrict__ newpos) {
    int k = k0 + blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= k1) return;
    const int32_t o = off[k], a = left[k], b = right[k];
    const int32_t ob = o + (a >= 0 ? cnt[a] : 1);
    if (a >= 0) off[a] = o; else newpos[-a - 1] = o;
    if (b >= 0) off[b] = ob; else newpos[-b - 1] = ob;
}

// leaf ranges of the inner nodes, leaves renumbered to depth-first order, triangle order to match
__global__ void k_ploc_finish(int32_t nt, int32_t* __restrict__ left, int32_t* __restrict__ right,
                              const int32_t* __restrict__ cnt, const int32_t* __restrict__ off,
                              const int32_t* __restrict__ newpos, int32_t* __restrict__ first,
                              int32_t* __restrict__ last, const uint32_t* __restrict__ sorted_vals,
                              uint32_t* __restrict__ dfs_vals) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nt) return;
    dfs_vals[newpos[i]] = sorted_vals[i];
    if (i >= nt - 1) return;
    first[i] = off[i];
    last[i] = off[i] + cnt[i] - 1;
    const int32_t a = left[i], b = right[i];
    if (a < 0) left[i] = -(newpos[-a - 1] + 1);
    if (b < 0) right[i] = -(newpos[-b - 1] + 1);
}

// ---------------------------------------------------------------------------
// collapse to 4-wide nodes, one level per launch
// ---------------------------------------------------------------------------
struct TreeView {
    const int32_t* left;
    const int32_t* right;
    const int32_t* first;
    const int32_t* last;
    const float4* nlo;   // inner-node boxes
    const float4* nhi;
    int leaf_max;        // subtrees of at most this many triangles become leaves (1..kLeafMax)
    __device__ int count(int32_t r) const { return r >= 0 ? last[r] - first[r] + 1 : 1; }
    __device__ int start(int32_t r) const { return r >= 0 ? first[r] : -r - 1; }
    __device__ float area(int32_t r) const {
        float4 a = nlo[r], b = nhi[r];
        float dx = b.x - a.x, dy = b.y - a.y, dz = b.z - a.z;
        return dx * dy + dy * dz + dz * dx;
    }
};

constexpr int32_t kEmpty = INT32_MIN;

__global__ void k_collapse_count(TreeView tv, const int32_t* __restrict__ entries, int32_t level_base, int32_t n_level,
                                 int32_t* __restrict__ kids, uint32_t* __restrict__ n_inner) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_level) return;
    int32_t r = entries[level_base + e];
    int32_t c[kWidth];
    for (int k = 0; k < kWidth; ++k) c[k] = kEmpty;
    int nk;
    if (r == kEmpty) {  // whole scene in one leaf (handled by the host; kept for safety)
        nk = 0;
    } else {
        c[0] = tv.left[r];
        c[1] = tv.right[r];
        nk = 2;
        // open the child with the largest surface area among those too big for a leaf, until there
        // are kWidth (the greedy collapse of a binary tree into a wide one)
        while (nk < kWidth) {
            int best = -1;
            float besta = -1.0f;
            for (int k = 0; k < nk; ++k) {
                if (c[k] >= 0 && tv.count(c[k]) > tv.leaf_max) {
                    float ar = tv.area(c[k]);
                    if (ar > besta) { besta = ar; best = k; }
                }
            }
            if (best < 0) break;
            int32_t rr = c[best];
            c[best] = tv.left[rr];
            c[nk++] = tv.right[rr];
        }
        // slots still free: split leaf-sized subtrees too (largest area first).  A node tests all its
        // boxes anyway, so smaller leaves cost no extra box tests and save triangle tests.
        while (nk < kWidth) {
            int best = -1;
            float besta = -1.0f;
            for (int k = 0; k < nk; ++k) {
                if (c[k] >= 0) {
                    float ar = tv.area(c[k]);
                    if (ar > besta) { besta = ar; best = k; }
                }
            }
            if (best < 0) break;
            int32_t rr = c[best];
            c[best] = tv.left[rr];
            c[nk++] = tv.right[rr];
        }
    }
    uint32_t ni = 0;
    for (int k = 0; k < kWidth; ++k) {
        kids[kWidth * (int64_t)e + k] = c[k];
        if (c[k] != kEmpty && c[k] >= 0 && tv.count(c[k]) > tv.leaf_max) ++ni;
    }
    n_inner[e] = ni;
}

__global__ void k_collapse_emit(TreeView tv, int32_t* __restrict__ entries, int32_t level_base, int32_t n_level,
                                const int32_t* __restrict__ kids, const uint32_t* __restrict__ prefix,
                                int32_t next_base, Node* __restrict__ nodes) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_level) return;
    Node& nd = nodes[level_base + e];
    uint32_t at = prefix[e];
    for (int k = 0; k < kWidth; ++k) {
        int32_t c = kids[kWidth * (int64_t)e + k];
        int32_t entry;
        if (c == kEmpty) {
            entry = kEmptyChild;
        } else if (c >= 0 && tv.count(c) > tv.leaf_max) {
            entry = next_base + (int32_t)at;
            entries[entry] = c;
            ++at;
        } else {
            // a leaf's slot holds the traversal's stack entry: -((first << 3 | (count - 1)) + 1)
            entry = -(((tv.start(c) << 3) | (tv.count(c) - 1)) + 1);
        }
        nd.child[k] = entry;
        set_leaf_count(nd, k, leaf_count(entry));
    }
}

__device__ __forceinline__ float pad_down(float x) { return x - (fabsf(x) + 1.0f) * 1.9073486e-6f; }  // 2^-19
__device__ __forceinline__ float pad_up(float x) { return x + (fabsf(x) + 1.0f) * 1.9073486e-6f; }

__global__ void k_bounds(Node* __restrict__ nodes, int32_t level_base, int32_t n_level,
                         const uint32_t* __restrict__ sorted_vals, const float4* __restrict__ tlo,
                         const float4* __restrict__ thi) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_level) return;
    Node& nd = nodes[level_base + e];
    float lo[kWidth][3], hi[kWidth][3];
    bool valid[kWidth];
    for (int k = 0; k < kWidth; ++k) {
        int32_t c = nd.child[k];
        int cnt = leaf_count(c);
        float l[3] = {FLT_MAX, FLT_MAX, FLT_MAX}, h[3] = {-FLT_MAX, -FLT_MAX, -FLT_MAX};
        valid[k] = c != kEmptyChild;
        if (c >= 0) {
            const Node& ch = nodes[c];
            for (int j = 0; j < kWidth; ++j) {
                if (ch.child[j] == kEmptyChild) continue;
                l[0] = fminf(l[0], ch.lo_x[j]); h[0] = fmaxf(h[0], ch.hi_x[j]);
                l[1] = fminf(l[1], ch.lo_y[j]); h[1] = fmaxf(h[1], ch.hi_y[j]);
                l[2] = fminf(l[2], ch.lo_z[j]); h[2] = fmaxf(h[2], ch.hi_z[j]);
            }
        } else if (cnt > 0) {
            int f = leaf_first(c);
            for (int j = 0; j < cnt; ++j) {
                uint32_t t = sorted_vals[f + j];
                float4 a = tlo[t], b = thi[t];
                l[0] = fminf(l[0], a.x); l[1] = fminf(l[1], a.y); l[2] = fminf(l[2], a.z);
                h[0] = fmaxf(h[0], b.x); h[1] = fmaxf(h[1], b.y); h[2] = fmaxf(h[2], b.z);
            }
            for (int a = 0; a < 3; ++a) { l[a] = pad_down(l[a]); h[a] = pad_up(h[a]); }
        }
        for (int a = 0; a < 3; ++a) { lo[k][a] = l[a]; hi[k][a] = h[a]; }
    }
    for (int k = 0; k < kWidth; ++k) {
        // an empty slot gets the box [FLT_MAX, FLT_MAX]^3, which no ray enters
        if (!valid[k])
            for (int a = 0; a < 3; ++a) lo[k][a] = hi[k][a] = FLT_MAX;
        nd.lo_x[k] = lo[k][0]; nd.hi_x[k] = hi[k][0];
        nd.lo_y[k] = lo[k][1]; nd.hi_y[k] = hi[k][1];
        nd.lo_z[k] = lo[k][2]; nd.hi_z[k] = hi[k][2];
    }
    // near-to-far child order for each ray-direction octant: sort slots by the
    // projection of the box centre on the octant's diagonal; empty slots last
    uint64_t orders4 = 0;
    for (int o = 0; o < 8; ++o) {
        float sx = (o & 1) ? -1.f : 1.f, sy = (o & 2) ? -1.f : 1.f, sz = (o & 4) ? -1.f : 1.f;
        float key[kWidth];
        int idx[kWidth];
        for (int k = 0; k < kWidth; ++k) {
            idx[k] = k;
            key[k] = valid[k] ? sx * (lo[k][0] + hi[k][0]) + sy * (lo[k][1] + hi[k][1]) + sz * (lo[k][2] + hi[k][2])
                              : FLT_MAX;
        }
        for (int a = 1; a < kWidth; ++a)
            for (int b = a; b > 0 && key[idx[b]] < key[idx[b - 1]]; --b) {
                int tmp = idx[b]; idx[b] = idx[b - 1]; idx[b - 1] = tmp;
            }
        uint32_t slots = 0;
        for (int a = 0; a < kWidth; ++a) slots |= (uint32_t)idx[a] << (kWidthBits * a);
        if constexpr (kWidth == 4)
            orders4 |= (uint64_t)slots << (8 * o);
        else
            nd.order[o] = slots;
    }
    if constexpr (kWidth == 4) {
        nd.order[0] = (uint32_t)orders4;
        nd.order[1] = (uint32_t)(orders4 >> 32);
        nd.order[2] = 0;
    }
}

__global__ void k_single_leaf_root(Node* __restrict__ nodes, int32_t nt, const float4* __restrict__ tlo,
                                   const float4* __restrict__ thi) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    Node& nd = nodes[0];
    float l[3] = {FLT_MAX, FLT_MAX, FLT_MAX}, h[3] = {-FLT_MAX, -FLT_MAX, -FLT_MAX};
    for (int t = 0; t < nt; ++t) {
        float4 a = tlo[t], b = thi[t];
        l[0] = fminf(l[0], a.x); l[1] = fminf(l[1], a.y); l[2] = fminf(l[2], a.z);
        h[0] = fmaxf(h[0], b.x); h[1] = fmaxf(h[1], b.y); h[2] = fmaxf(h[2], b.z);
    }
    for (int k = 0; k < kWidth; ++k) {
        bool v = k == 0;
        nd.lo_x[k] = v ? pad_down(l[0]) : FLT_MAX; nd.hi_x[k] = v ? pad_up(h[0]) : FLT_MAX;
        nd.lo_y[k] = v ? pad_down(l[1]) : FLT_MAX; nd.hi_y[k] = v ? pad_up(h[1]) : FLT_MAX;
        nd.lo_z[k] = v ? pad_down(l[2]) : FLT_MAX; nd.hi_z[k] = v ? pad_up(h[2]) : FLT_MAX;
        nd.child[k] = v ? -(((0 << 3) | (nt - 1)) + 1) : kEmptyChild;
        set_leaf_count(nd, k, v ? nt : 0);
    }
    // identity order for every octant
    uint32_t slots = 0;
    for (int a = 0; a < kWidth; ++a) slots |= (uint32_t)a << (kWidthBits * a);
    if constexpr (kWidth == 4) {
        nd.order[0] = nd.order[1] = slots * 0x01010101u;
        nd.order[2] = 0;
    } else {
        for (int o = 0; o < 8; ++o) nd.order[o] = slots;
    }
}

__global__ void k_tri_write(const float* __restrict__ verts, const int32_t* __restrict__ tris,
                            const uint32_t* __restrict__ sorted_vals, int32_t nt, int64_t nv, Tri* __restrict__ out,
                            int32_t* __restrict__ sorted_of) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nt) return;
    uint32_t t = sorted_vals[j];
    int32_t ia = tris[3 * (int64_t)t], ib = tris[3 * (int64_t)t + 1], ic = tris[3 * (int64_t)t + 2];
    if (ia < 0 || ib < 0 || ic < 0 || ia >= nv || ib >= nv || ic >= nv) ia = ib = ic = 0;
    float a[3], b[3], c[3];
    for (int k = 0; k < 3; ++k) {
        a[k] = verts[3 * (int64_t)ia + k];
        b[k] = verts[3 * (int64_t)ib + k];
        c[k] = verts[3 * (int64_t)ic + k];
    }
    Tri r;
    r.v0x = a[0]; r.v0y = a[1]; r.v0z = a[2]; r.id = (int32_t)t;
    r.e1x = b[0] - a[0]; r.e1y = b[1] - a[1]; r.e1z = b[2] - a[2]; r.pad1 = 0.f;
    r.e2x = c[0] - a[0]; r.e2y = c[1] - a[1]; r.e2z = c[2] - a[2]; r.pad2 = 0.f;
    out[j] = r;
    sorted_of[t] = j;
}

__global__ void k_fill_u8(uint8_t* __restrict__ p, int64_t n, uint8_t v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

inline int blocks_for(int64_t n, int t) { return (int)((n + t - 1) / t); }

// Exclusive scan of n >= 1 elements of `in` into `out` (distinct arrays); *total (nullable) gets the
// sum.  tile holds at least 2 ceil(n / kScanTile) elements: the tile sums, then their scan.
template <class T>
void scan_exclusive(const T* in, T* out, int64_t n, T* total, T* tile, hipStream_t st) {
    if (n <= kScanTile) {
        hipLaunchKernelGGL(k_scan_exclusive<T>, dim3(1), dim3(kScanThreads), 0, st, in, out, n, total);
        return;
    }
    const int nb = blocks_for(n, kScanTile);
    hipLaunchKernelGGL(k_tile_sums<T>, dim3(nb), dim3(kScanThreads), 0, st, in, n, tile);
    hipLaunchKernelGGL(k_scan_exclusive<T>, dim3(1), dim3(kScanThreads), 0, st, tile, tile + nb, (int64_t)nb, total);
    hipLaunchKernelGGL(k_tile_scan<T>, dim3(nb), dim3(kScanThreads), 0, st, in, n, tile + nb, out);
}

}  // namespace

// Scratch of one build; freed when the build returns.
struct BuildScratch {
    vf_ctx* ctx;
    std::vector<std::pair<void*, int64_t>> held;
    explicit BuildScratch(vf_ctx* c) : ctx(c) {}
    ~BuildScratch() {
        for (auto& h : held) ctx_free(ctx, h.first, h.second);
    }
    template <class T>
    vf_status get(T** p, int64_t count) {
        void* q = nullptr;
        int64_t bytes = count * (int64_t)sizeof(T);
        if (bytes <= 0) bytes = 16;
        vf_status st = ctx_alloc(ctx, &q, bytes);
        if (st != VF_OK) return st;
        held.emplace_back(q, bytes);
        *p = (T*)q;
        return VF_OK;
    }
};

vf_status build_scene(vf_ctx* ctx, const float* verts, int64_t nv, const int32_t* tris, int32_t nt,
                      const uint8_t* rgb, hipStream_t st, SceneHost* out) {
    BuildScratch sc(ctx);
    float4 *tlo, *thi, *cen;
    float *partial, *bounds;
    uint32_t *keys, *vals, *keys2, *vals2, *hist, *offs, *total;
    int32_t *left, *right, *first, *last, *entries, *kids;
    uint32_t *n_inner, *prefix;
    const int nb_prep = blocks_for(nt, kPrepThreads);
    const int nb_sort = blocks_for(nt, kSortTile);
    vf_status s;
#define GET(p, n) if ((s = sc.get(&p, n)) != VF_OK) return s
    GET(tlo, nt); GET(thi, nt); GET(cen, nt); GET(partial, 6 * (int64_t)nb_prep); GET(bounds, 12);
    GET(keys, nt); GET(vals, nt); GET(keys2, nt); GET(vals2, nt);
    GET(hist, 256 * (int64_t)nb_sort); GET(offs, 256 * (int64_t)nb_sort); GET(total, 4);
    GET(left, nt); GET(right, nt); GET(first, nt); GET(last, nt);
    GET(entries, nt + 1); GET(kids, kWidth * (int64_t)(nt + 1)); GET(n_inner, nt + 1); GET(prefix, nt + 1);
    // tile sums of the multi-workgroup scans (longest scan: the sort histograms or nt + 1 elements)
    const int64_t scan_max = std::max<int64_t>(256 * (int64_t)nb_sort, (int64_t)nt + 1);
    uint32_t* tsum32;
    uint64_t* tsum64;
    GET(tsum32, 2 * (scan_max / kScanTile + 2)); GET(tsum64, 2 * (scan_max / kScanTile + 2));
    int32_t *par_int, *par_leaf;
    uint32_t* flags;
    float4 *nlo, *nhi;
    GET(par_int, nt); GET(par_leaf, nt); GET(flags, nt); GET(nlo, nt); GET(nhi, nt);
#undef GET

    hipEvent_t ev0, ev1;
    VF_HIP(hipEventCreate(&ev0));
    VF_HIP(hipEventCreate(&ev1));
    VF_HIP(hipEventRecord(ev0, st));

    hipLaunchKernelGGL(k_tri_prep, dim3(nb_prep), dim3(kPrepThreads), 0, st, verts, nv, tris, nt, tlo, thi, cen,
                       partial, ctx->d_build_err);
    hipLaunchKernelGGL(k_reduce_bounds, dim3(1), dim3(kScanThreads), 0, st, partial, nb_prep, tlo, thi, nt, bounds);
    {
        // reject bad input before the passes that would work on it
        uint32_t bad = 0;
        VF_HIP(hipMemcpyAsync(&bad, ctx->d_build_err, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
        VF_HIP(hipStreamSynchronize(st));
        if (bad & (kErrTriIndex | kErrVertex)) {
            return fail(VF_EINVAL, (bad & kErrTriIndex) ? "vf_scene_build: triangle vertex index out of range"
                                                        : "vf_scene_build: vertex coordinates must be finite");
        }
    }
    hipLaunchKernelGGL(k_morton, dim3(blocks_for(nt, 256)), dim3(256), 0, st, cen, nt, bounds, keys, vals);
    uint32_t *ka = keys, *va = vals, *kb = keys2, *vb = vals2;
    for (int shift = 0; shift < 32; shift += 8) {
        hipLaunchKernelGGL(k_sort_hist, dim3(nb_sort), dim3(kSortThreads), 0, st, ka, nt, shift, hist, nb_sort);
        scan_exclusive<uint32_t>(hist, offs, 256 * (int64_t)nb_sort, nullptr, tsum32, st);
        hipLaunchKernelGGL(k_sort_scatter, dim3(nb_sort), dim3(kSortThreads), 0, st, ka, va, kb, vb, nt, shift, offs,
                           nb_sort);
        uint32_t* t;
        t = ka; ka = kb; kb = t;
        t = va; va = vb; vb = t;
    }
    // after 4 passes the sorted pairs are back in (keys, vals)

    // scene block: nodes | tris | sorted_of | rgb
    const int64_t max_nodes = nt > 1 ? nt : 1;
    int64_t node_bytes = max_nodes * (int64_t)sizeof(Node);
    // padded by kLeafMax records: a leaf's triangles are fetched as one fixed-size burst
    int64_t tri_bytes = ((int64_t)nt + kLeafMax) * (int64_t)sizeof(Tri);
    int64_t map_bytes = ((int64_t)nt * 4 + 255) / 256 * 256;
    int64_t rgb_bytes = ((int64_t)nt * 3 + 255) / 256 * 256;
    Node* nodes = nullptr;
    // allocate the final block after the topology is known (node count); use a
    // temporary node array of the upper-bound size first
    Node* tmp_nodes;
    if ((s = sc.get(&tmp_nodes, max_nodes)) != VF_OK) return s;

    std::vector<int32_t> level_base, level_n;
    int depth = 0;
    // triangle of each leaf position: Morton order, or depth-first order of the clustered tree
    const uint32_t* leaf_vals = vals;
    uint32_t* dfs_vals = nullptr;
    int32_t builder_used = ctx->bvh_builder;
    int32_t n_nodes = 0;
    bool single_leaf = nt <= kLeafMax;
    if (single_leaf) {
        hipLaunchKernelGGL(k_single_leaf_root, dim3(1), dim3(64), 0, st, tmp_nodes, nt, tlo, thi);
        n_nodes = 1;
        depth = 1;
    } else {
        TreeView tv{left, right, first, last, nlo, nhi, ctx->bvh_leaf};
        // collapse the binary tree below `root` level by level; *too_deep when the wide tree would
        // exceed the traversal's depth bound
        auto collapse = [&](int32_t root, const uint32_t* leaf_vals, bool* too_deep) -> vf_status {
            *too_deep = false;
            level_base.clear();
            level_n.clear();
            depth = 0;
            VF_HIP(hipMemcpyAsync(entries, &root, sizeof(int32_t), hipMemcpyHostToDevice, st));
            int32_t base = 0, n_level = 1;
            while (n_level > 0) {
                if (depth >= kMaxBvhDepth) {
                    *too_deep = true;
                    return VF_OK;
                }
                level_base.push_back(base);
                level_n.push_back(n_level);
                ++depth;
                hipLaunchKernelGGL(k_collapse_count, dim3(blocks_for(n_level, 256)), dim3(256), 0, st, tv, entries,
                                   base, n_level, kids, n_inner);
                scan_exclusive<uint32_t>(n_inner, prefix, (int64_t)n_level, total, tsum32, st);
                int32_t next_base = base + n_level;
                hipLaunchKernelGGL(k_collapse_emit, dim3(blocks_for(n_level, 256)), dim3(256), 0, st, tv, entries,
                                   base, n_level, kids, prefix, next_base, tmp_nodes);
                uint32_t nnext = 0;
                VF_HIP(hipMemcpyAsync(&nnext, total, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
                VF_HIP(hipStreamSynchronize(st));
                base = next_base;
                n_level = (int32_t)nnext;
            }
            n_nodes = base;
            for (int L = depth - 1; L >= 0; --L)
                hipLaunchKernelGGL(k_bounds, dim3(blocks_for(level_n[L], 128)), dim3(128), 0, st, tmp_nodes,
                                   level_base[L], level_n[L], leaf_vals, tlo, thi);
            return VF_OK;
        };
        bool too_deep = true;
        if (ctx->bvh_builder == VF_BVH_CLUSTER) {
            int32_t *cid, *cid2, *nn, *cnt, *off, *newpos;
            float4 *clo, *chi, *clo2, *chi2;
            uint64_t *fl, *pre, *tot64;
#define GET(p, n) if ((s = sc.get(&p, n)) != VF_OK) return s
            GET(cid, nt); GET(cid2, nt); GET(nn, nt); GET(cnt, nt); GET(off, nt); GET(newpos, nt);
            GET(clo, nt); GET(chi, nt); GET(clo2, nt); GET(chi2, nt); GET(fl, nt); GET(pre, nt); GET(tot64, 1);
            GET(dfs_vals, nt);
#undef GET
            hipLaunchKernelGGL(k_ploc_init, dim3(blocks_for(nt, 256)), dim3(256), 0, st, vals, nt, tlo, thi, cid, clo,
                               chi);
            std::vector<int32_t> pass_base;
            int32_t m = nt, node_base = 0;
            int32_t spread_ties = 0;
            while (m > 1) {
                hipLaunchKernelGGL(k_ploc_nn, dim3(blocks_for(m, 256)), dim3(256), 0, st, m, clo, chi,
                                   spread_ties, nn);
                hipLaunchKernelGGL(k_ploc_flags, dim3(blocks_for(m, 256)), dim3(256), 0, st, m, nn, fl);
                scan_exclusive<uint64_t>(fl, pre, (int64_t)m, tot64, tsum64, st);
                hipLaunchKernelGGL(k_ploc_merge, dim3(blocks_for(m, 256)), dim3(256), 0, st, m, nn, fl, pre,
                                   node_base, cid, clo, chi, cid2, clo2, chi2, left, right, cnt, nlo, nhi);
                uint64_t t = 0;
                VF_HIP(hipMemcpyAsync(&t, tot64, sizeof(uint64_t), hipMemcpyDeviceToHost, st));
                VF_HIP(hipStreamSynchronize(st));
                const int32_t merges = (int32_t)(t & 0xffffffffu), kept = (int32_t)(t >> 32);
                // the best pair is always mutual; anything else means corrupted input
                if (merges <= 0 || kept != m - merges || node_base + merges > nt - 1)
                    return fail(VF_EHIP, "scene build: clustering pass made no progress");
                pass_base.push_back(node_base);
                node_base += merges;
                spread_ties = (int64_t)merges * 32 < (int64_t)m ? 1 : 0;
                m = kept;
                std::swap(cid, cid2);
                std::swap(clo, clo2);
                std::swap(chi, chi2);
            }
            pass_base.push_back(node_base);   // == nt - 1
            const int32_t root = nt - 2;
            VF_HIP(hipMemsetAsync(off + root, 0, sizeof(int32_t), st));
            for (int p = (int)pass_base.size() - 2; p >= 0; --p) {
                const int32_t k0 = pass_base[p], k1 = pass_base[p + 1];
                hipLaunchKernelGGL(k_ploc_offsets, dim3(blocks_for(k1 - k0, 256)), dim3(256), 0, st, k0, k1, left,
                                   right, cnt, off, newpos);
            }
            hipLaunchKernelGGL(k_ploc_finish, dim3(blocks_for(nt, 256)), dim3(256), 0, st, nt, left, right, cnt, off,
                               newpos, first, last, vals, dfs_vals);
            leaf_vals = dfs_vals;
            if ((s = collapse(root, leaf_vals, &too_deep)) != VF_OK) return s;
        }
        if (too_deep) {
            builder_used = VF_BVH_RADIX;
            // the Morton radix tree (its depth is bounded by the key bits plus log2 of duplicates)
            hipLaunchKernelGGL(k_radix_tree, dim3(blocks_for(nt - 1, 256)), dim3(256), 0, st, ka, nt, left, right,
                               first, last);
            hipLaunchKernelGGL(k_parents, dim3(blocks_for(nt - 1, 256)), dim3(256), 0, st, left, right, nt, par_int,
                               par_leaf);
            VF_HIP(hipMemsetAsync(flags, 0, (size_t)nt * 4, st));
            hipLaunchKernelGGL(k_binary_bounds, dim3(blocks_for(nt, 256)), dim3(256), 0, st, left, right, nt, vals,
                               tlo, thi, par_int, par_leaf, flags, nlo, nhi);
            leaf_vals = vals;
            if ((s = collapse(0, leaf_vals, &too_deep)) != VF_OK) return s;
            if (too_deep) return fail(VF_EINVAL, "scene BVH deeper than the traversal stack allows");
        }
    }
    node_bytes = (int64_t)n_nodes * (int64_t)sizeof(Node);
    int64_t total_bytes = node_bytes + tri_bytes + map_bytes + rgb_bytes;
    void* block = nullptr;
    if ((s = ctx_alloc(ctx, &block, total_bytes)) != VF_OK) return s;
    nodes = (Node*)block;
    Tri* tri_out = (Tri*)((char*)block + node_bytes);
    int32_t* sorted_of = (int32_t*)((char*)block + node_bytes + tri_bytes);
    uint8_t* rgb_out = (uint8_t*)((char*)block + node_bytes + tri_bytes + map_bytes);
    hipError_t e = hipMemcpyAsync(nodes, tmp_nodes, node_bytes, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess)
        e = hipMemsetAsync((char*)tri_out + (int64_t)nt * sizeof(Tri), 0, kLeafMax * sizeof(Tri), st);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_tri_write, dim3(blocks_for(nt, 256)), dim3(256), 0, st, verts, tris, leaf_vals, nt, nv, tri_out,
                           sorted_of);
        if (rgb)
            e = hipMemcpyAsync(rgb_out, rgb, (size_t)nt * 3, hipMemcpyDeviceToDevice, st);
        else
            hipLaunchKernelGGL(k_fill_u8, dim3(blocks_for((int64_t)nt * 3, 256)), dim3(256), 0, st, rgb_out,
                               (int64_t)nt * 3, (uint8_t)128);
    }
    if (e == hipSuccess) e = hipEventRecord(ev1, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) {
        ctx_free(ctx, block, total_bytes);
        (void)hipEventDestroy(ev0);
        (void)hipEventDestroy(ev1);
        return hip_fail(e, "scene build");
    }
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, ev0, ev1);
    (void)hipEventDestroy(ev0);
    (void)hipEventDestroy(ev1);
    float bnd[12];
    VF_HIP(hipMemcpy(bnd, bounds, sizeof(bnd), hipMemcpyDeviceToHost));

    out->block = block;
    out->bytes = total_bytes;
    out->info.n_tris = nt;
    out->info.n_nodes = n_nodes;
    out->info.n_leaves = 0;
    out->info.bytes = total_bytes;
    out->info.depth = depth;
    out->info.leaf_max = ctx->bvh_leaf;
    for (int k = 0; k < 3; ++k) {
        out->info.bounds_lo[k] = bnd[6 + k];
        out->info.bounds_hi[k] = bnd[9 + k];
    }
    out->info.build_ms = ms;
    out->info.width = kWidth;
    out->info.builder = builder_used;
    out->info.reserved = 0;
    out->desc.nodes = nodes;
    out->desc.tris = tri_out;
    out->desc.rgb = rgb_out;
    out->desc.sorted_of = sorted_of;
    out->desc.n_tris = nt;
    out->desc.root_leaf = single_leaf ? 1 : 0;
    out->desc.n_nodes = (int32_t)n_nodes;
    out->desc.valid = 1;
    return VF_OK;
}

}  // namespace vf
