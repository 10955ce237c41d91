// Top-level trees over swarm members (the swarm example of Sec. IV), rebuilt from the states before every
// render that shows swarms.  One workgroup per swarm:
//   1. bounds of the members' positions, a 30-bit Morton code of each (10 bits per axis over the bounds);
//   2. a bitonic sort of (code, index) in LDS;
//   3. member records in sorted order: R(q / |q|) in float32 (the render's member test reads it), the
//      position, the index in the swarm's list and the state slot;
//   4. an implicit 4-wide tree over groups of four consecutive members, level by level from the bottom:
//      child boxes are the world-axis boxes of the members' oriented boxes (centre +- |R| half), padded
//      outward by 2^-19 (|x| + 1) like the mesh BVH, with each octant's near-to-far child order.
// Bad slots set kErrSlot and place the member at the origin (its state is not read).
#include <float.h>

#include "dynamics.h"
#include "swarm.h"
#include "vf_internal.h"

namespace vf {

namespace {

constexpr int kTreeThreads = 256;

__device__ __forceinline__ float pad_lo(float x) { return x - (fabsf(x) + 1.0f) * 1.9073486328125e-6f; }
__device__ __forceinline__ float pad_hi(float x) { return x + (fabsf(x) + 1.0f) * 1.9073486328125e-6f; }

struct TreeArgs {
    SwarmTable sw;
    const float* state;
    int64_t n_slots;
    uint32_t* err;
};

// world-axis box of member record k
__device__ __forceinline__ void member_box(const SwarmMember* mem, int k, const float half[3], float lo[3],
                                           float hi[3]) {
    const SwarmMember& mb = mem[k];
    for (int a = 0; a < 3; ++a) {
        const float ext = fabsf(mb.r[3 * a]) * half[0] + fabsf(mb.r[3 * a + 1]) * half[1] +
                          fabsf(mb.r[3 * a + 2]) * half[2];
        lo[a] = mb.c[a] - ext;
        hi[a] = mb.c[a] + ext;
    }
}

__global__ void __launch_bounds__(kTreeThreads) k_swarm_tree(TreeArgs a) {
    __shared__ unsigned long long keys[kSwarmMaxMembers];
    __shared__ float red[6][kTreeThreads / 64];
    __shared__ float bounds[6];
    const int s = blockIdx.x, t = threadIdx.x;
    const int32_t first = a.sw.off[s];
    const int32_t m = a.sw.off[s + 1] - first;
    if (m <= 0 || m > kSwarmMaxMembers) return;
    const int32_t* slots = a.sw.slots + first;
    auto position = [&](int j, float p[3]) {
        const int64_t slot = slots[j];
        if (slot < 0 || slot >= a.n_slots) {
            p[0] = p[1] = p[2] = 0.0f;
            return false;
        }
        for (int k = 0; k < 3; ++k) p[k] = a.state[slot * 17 + k];
        return true;
    };
    // 1. bounds of the positions
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int j = t; j < m; j += kTreeThreads) {
        float p[3];
        if (!position(j, p)) atomicOr(a.err, kErrSlot);
        for (int k = 0; k < 3; ++k) {
            lo[k] = fminf(lo[k], p[k]);
            hi[k] = fmaxf(hi[k], p[k]);
        }
    }
    for (int off = 32; off > 0; off >>= 1)
        for (int k = 0; k < 3; ++k) {
            lo[k] = fminf(lo[k], __shfl_xor(lo[k], off));
            hi[k] = fmaxf(hi[k], __shfl_xor(hi[k], off));
        }
    if ((t & 63) == 0)
        for (int k = 0; k < 3; ++k) {
            red[k][t >> 6] = lo[k];
            red[3 + k][t >> 6] = hi[k];
        }
    __syncthreads();
    if (t == 0) {
        for (int k = 0; k < 3; ++k) {
            float l = red[k][0], h = red[3 + k][0];
            for (int w = 1; w < kTreeThreads / 64; ++w) {
                l = fminf(l, red[k][w]);
                h = fmaxf(h, red[3 + k][w]);
            }
            bounds[k] = l;
            bounds[3 + k] = h;
        }
    }
    __syncthreads();
    // 2. Morton keys, padded to a power of two with keys that sort last
    int32_t pow2 = 1;
    while (pow2 < m) pow2 <<= 1;
    for (int j = t; j < pow2; j += kTreeThreads) {
        unsigned long long key = ~0ull;
        if (j < m) {
            float p[3];
            position(j, p);
            uint32_t q[3];
            for (int k = 0; k < 3; ++k) {
                const float ext = bounds[3 + k] - bounds[k];
                const float x = ext > 0.0f ? (p[k] - bounds[k]) / ext * 1023.0f : 0.0f;
                q[k] = (uint32_t)fminf(fmaxf(x, 0.0f), 1023.0f);
            }
            key = ((unsigned long long)morton3_10(q[0], q[1], q[2]) << 32) | (uint32_t)j;
        }
        keys[j] = key;
    }
    __syncthreads();
    for (int32_t k = 2; k <= pow2; k <<= 1)
        for (int32_t jj = k >> 1; jj > 0; jj >>= 1) {
            for (int32_t i = t; i < pow2; i += kTreeThreads) {
                const int32_t l = i ^ jj;
                if (l > i) {
                    const unsigned long long x = keys[i], y = keys[l];
                    const bool up = (i & k) == 0;
                    if ((x > y) == up) {
                        keys[i] = y;
                        keys[l] = x;
                    }
                }
            }
            __syncthreads();
        }
    // 3. member records in tree order
    SwarmMember* mem = a.sw.members + first;
    for (int k = t; k < m; k += kTreeThreads) {
        const int32_t j = (int32_t)(keys[k] & 0xFFFFFFFFu);
        SwarmMember rec;
        float p[3];
        const bool ok = position(j, p);
        if (ok) {
            quat_rot(a.state + (int64_t)slots[j] * 17 + 3, rec.r);
        } else {
            for (int i = 0; i < 9; ++i) rec.r[i] = (i % 4 == 0) ? 1.0f : 0.0f;
        }
        for (int i = 0; i < 3; ++i) rec.c[i] = p[i];
        rec.j = j;
        rec.slot = slots[j];
        rec.pad[0] = rec.pad[1] = 0;
        mem[k] = rec;
    }
    __syncthreads();
    // 4. the tree, bottom level first
    Node4* nodes = a.sw.nodes + a.sw.node_off[s];
    const int32_t levels = swarm_tree_levels(m);
    const int32_t groups = (m + 3) / 4;
    int32_t level_first[8];
    {
        int32_t acc = 0;
        for (int32_t d = 0; d < levels; ++d) {
            level_first[d] = acc;
            acc += swarm_level_nodes(m, levels, d);
        }
    }
    for (int32_t d = levels - 1; d >= 0; --d) {
        const int32_t n_d = swarm_level_nodes(m, levels, d);
        const int32_t n_below = d + 1 < levels ? swarm_level_nodes(m, levels, d + 1) : groups;
        for (int32_t i = t; i < n_d; i += kTreeThreads) {
            Node4 nd;
            float clo[4][3], chi[4][3];
            bool valid[4];
            for (int c = 0; c < 4; ++c) {
                const int32_t ci = i * 4 + c;
                valid[c] = ci < n_below;
                float l[3] = {FLT_MAX, FLT_MAX, FLT_MAX}, h[3] = {-FLT_MAX, -FLT_MAX, -FLT_MAX};
                int32_t entry = kEmptyChild;
                if (valid[c] && d + 1 == levels) {
                    // a leaf: members [4 ci, min(4 ci + 4, m))
                    const int32_t f = 4 * ci, cnt = (m - f) < 4 ? (m - f) : 4;
                    for (int k = 0; k < cnt; ++k) {
                        float bl[3], bh[3];
                        member_box(mem, f + k, a.sw.half, bl, bh);
                        for (int q = 0; q < 3; ++q) {
                            l[q] = fminf(l[q], bl[q]);
                            h[q] = fmaxf(h[q], bh[q]);
                        }
                    }
                    for (int q = 0; q < 3; ++q) {
                        l[q] = pad_lo(l[q]);
                        h[q] = pad_hi(h[q]);
                    }
                    entry = -((f << 3 | (cnt - 1)) + 1);
                } else if (valid[c]) {
                    const int32_t child = level_first[d + 1] + ci;
                    const Node4& ch = nodes[child];
                    for (int k = 0; k < 4; ++k) {
                        if (ch.child[k] == kEmptyChild) continue;
                        l[0] = fminf(l[0], ch.lo_x[k]); h[0] = fmaxf(h[0], ch.hi_x[k]);
                        l[1] = fminf(l[1], ch.lo_y[k]); h[1] = fmaxf(h[1], ch.hi_y[k]);
                        l[2] = fminf(l[2], ch.lo_z[k]); h[2] = fmaxf(h[2], ch.hi_z[k]);
                    }
                    entry = child;
                }
                if (!valid[c])
                    for (int q = 0; q < 3; ++q) l[q] = h[q] = FLT_MAX;   // a box no ray enters
                for (int q = 0; q < 3; ++q) {
                    clo[c][q] = l[q];
                    chi[c][q] = h[q];
                }
                nd.child[c] = entry;
                nd.count[c] = (uint8_t)(entry < 0 && entry != kEmptyChild ? ((-entry - 1) & 7) + 1 : 0);
                nd.lo_x[c] = l[0]; nd.hi_x[c] = h[0];
                nd.lo_y[c] = l[1]; nd.hi_y[c] = h[1];
                nd.lo_z[c] = l[2]; nd.hi_z[c] = h[2];
            }
            // near-to-far order of the children for each ray-direction octant (empty slots last)
            uint64_t orders = 0;
            for (int o = 0; o < 8; ++o) {
                const float sx = (o & 1) ? -1.f : 1.f, sy = (o & 2) ? -1.f : 1.f, sz = (o & 4) ? -1.f : 1.f;
                float key[4];
                int idx[4];
                for (int c = 0; c < 4; ++c) {
                    idx[c] = c;
                    key[c] = valid[c] ? sx * (clo[c][0] + chi[c][0]) + sy * (clo[c][1] + chi[c][1]) +
                                            sz * (clo[c][2] + chi[c][2])
                                      : FLT_MAX;
                }
                for (int x = 1; x < 4; ++x)
                    for (int y = x; y > 0 && key[idx[y]] < key[idx[y - 1]]; --y) {
                        const int tmp = idx[y];
                        idx[y] = idx[y - 1];
                        idx[y - 1] = tmp;
                    }
                uint32_t sl = 0;
                for (int c = 0; c < 4; ++c) sl |= (uint32_t)idx[c] << (2 * c);
                orders |= (uint64_t)sl << (8 * o);
            }
            nd.order[0] = (uint32_t)orders;
            nd.order[1] = (uint32_t)(orders >> 32);
            nd.order[2] = 0;
            nodes[level_first[d] + i] = nd;
        }
        __syncthreads();
    }
}

}  // namespace

hipError_t launch_swarm_tree(const SwarmTable& sw, const float* state, int64_t n_slots, uint32_t* err,
                             hipStream_t st) {
    if (sw.n <= 0) return hipSuccess;
    TreeArgs a{sw, state, n_slots, err};
    hipLaunchKernelGGL(k_swarm_tree, dim3((unsigned)sw.n), dim3(kTreeThreads), 0, st, a);
    return hipGetLastError();
}

}  // namespace vf
