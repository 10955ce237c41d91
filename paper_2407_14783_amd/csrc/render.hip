// Batched step + ray-cast render kernels (Sec. III-A dynamics, Sec. III-B views).
//
// One wavefront traces one 8 x 8 pixel packet of one agent.  The packet walks
// the 4-wide BVH together: every node and leaf triangle is fetched once per
// wavefront through the scalar data path (wave-uniform address), each lane
// tests its own ray, and ballots decide which children the packet visits.  The
// traversal stack is wave-uniform and lives in two VGPRs, one entry per lane
// (a lane-select write and v_readlane, the stack pointer in an SGPR).  Children are
// pushed far-to-near using the node's precomputed order for the packet's
// direction octant, so the nearest child is popped first and lanes that have
// found a closer hit cull the rest by their per-lane t.
//
// Launch: one workgroup = 4 wavefronts = 4 tiles of one agent; the grid covers
// n agents x ceil(tiles(max_h, max_w) / 4) groups.  Workgroups are remapped so
// each XCD (workgroup id mod 8) processes a contiguous range of agents, keeping
// one agent's (and, with agents grouped by scene, one scene's) traffic in one L2.
//
// The fused kernel (vf_step with views) first advances the agent's dynamics in
// one lane per workgroup (every workgroup of the agent computes the same bits),
// then renders at the new pose; the last workgroup of the agent to arrive on the
// agent's counter writes the new state, so the state can be updated in place.
#include "dynamics.h"
#include "vf_internal.h"

namespace vf {

#define CONST_AS __attribute__((address_space(4)))

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

__device__ __forceinline__ int uniform_i(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Logical group of this workgroup after the XCD-aware remap.
__device__ __forceinline__ int logical_group(int total) {
    int b = blockIdx.x;
    int q = total >> 3, r = total & 7;
    int x = b & 7, k = b >> 3;
    return x * q + (x < r ? x : r) + k;
}

// Camera ray of pixel (r, c): d = R (1, -u, v); R from the normalised quaternion.
__device__ __forceinline__ void pixel_ray(const float rot[9], float tan_h, int H, int W, int r, int c, float d[3]) {
    float u = (2.0f * ((float)c + 0.5f) / (float)W - 1.0f) * tan_h;
    float v = (1.0f - 2.0f * ((float)r + 0.5f) / (float)H) * tan_h * ((float)H / (float)W);
    d[0] = rot[0] - rot[1] * u + rot[2] * v;
    d[1] = rot[3] - rot[4] * u + rot[5] * v;
    d[2] = rot[6] - rot[7] * u + rot[8] * v;
}

__device__ __forceinline__ float safe_inv(float x) {
    const float eps = 1e-20f;
    return 1.0f / (fabsf(x) < eps ? copysignf(eps, x) : x);
}

struct TraceStats {
    unsigned long long node_lane, box_lane, tri_lane, node_wave, tri_wave, hits;
};

template <bool STATS>
__device__ __forceinline__ void trace_packet(const SceneDesc& sc, bool valid, const float o[3], const float d[3],
                                             float t_near, float t_far, float& t_best, int32_t& id_best,
                                             uint32_t* err, TraceStats& ts) {
    const Node4 CONST_AS* nodes = (const Node4 CONST_AS*)sc.nodes;
    const Tri CONST_AS* tris = (const Tri CONST_AS*)sc.tris;
    const float inv[3] = {safe_inv(d[0]), safe_inv(d[1]), safe_inv(d[2])};
    // 1 + 2 gamma_3 (Ize 2013) keeps the slab test conservative in float32
    const float grow = 1.0000004f;
    int oct = (d[0] < 0.f ? 1 : 0) | (d[1] < 0.f ? 2 : 0) | (d[2] < 0.f ? 4 : 0);
    oct = uniform_i(oct);
    t_best = t_far;
    id_best = -1;
    const uint64_t lanes = __ballot(valid);
    if (lanes == 0ull) return;

    int stk0 = 0, stk1 = 0;
    int sp = 0;
    int32_t entry = 0;          // root: inner node 0
    bool overflow = false;
    while (true) {
        if (entry >= 0) {
            // the whole 128-byte node in one burst of wave-uniform (scalar) loads
            const uint32_t CONST_AS* np = (const uint32_t CONST_AS*)(nodes + entry);
            uint32_t w[32];
#pragma unroll
            for (int i = 0; i < 32; ++i) w[i] = np[i];
            if (STATS) {
                ts.node_wave += 1;
                ts.node_lane += valid ? 1 : 0;
            }
            const uint32_t counts = w[28];
            uint64_t hitmask[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const float lox = __uint_as_float(w[k]), hix = __uint_as_float(w[4 + k]);
                const float loy = __uint_as_float(w[8 + k]), hiy = __uint_as_float(w[12 + k]);
                const float loz = __uint_as_float(w[16 + k]), hiz = __uint_as_float(w[20 + k]);
                const int32_t ch = (int32_t)w[24 + k];
                const uint32_t cnt = (counts >> (8 * k)) & 255u;
                float tx0 = (lox - o[0]) * inv[0], tx1 = (hix - o[0]) * inv[0];
                float ty0 = (loy - o[1]) * inv[1], ty1 = (hiy - o[1]) * inv[1];
                float tz0 = (loz - o[2]) * inv[2], tz1 = (hiz - o[2]) * inv[2];
                float t0 = fmaxf(fmaxf(fminf(tx0, tx1), fminf(ty0, ty1)), fmaxf(fminf(tz0, tz1), t_near));
                float t1 = fminf(fminf(fmaxf(tx0, tx1), fmaxf(ty0, ty1)), fmaxf(tz0, tz1)) * grow;
                bool slot = ch >= 0 || cnt > 0u;
                bool h = valid && slot && t0 <= fminf(t1, t_best);
                hitmask[k] = __ballot(h);
            }
            if (STATS) ts.box_lane += 4 * (unsigned long long)(valid ? 1 : 0);
            const uint64_t ord = ((uint64_t)w[30] << 32) | w[29];
            const uint32_t byte = (uint32_t)(ord >> (8 * oct)) & 255u;
            // push hit children far-to-near so the nearest is on top
#pragma unroll
            for (int i = 3; i >= 0; --i) {
                int k = (byte >> (2 * i)) & 3;
                uint64_t hm = k == 0 ? hitmask[0] : k == 1 ? hitmask[1] : k == 2 ? hitmask[2] : hitmask[3];
                if (hm != 0ull) {
                    int32_t c = (int32_t)(k == 0 ? w[24] : k == 1 ? w[25] : k == 2 ? w[26] : w[27]);
                    int32_t cnt = (int32_t)((counts >> (8 * k)) & 255u);
                    int32_t e = c >= 0 ? c : -((((-c - 1) << 3) | (cnt - 1)) + 1);
                    if (sp < kStackCap) {
                        // write lane sp of the two stack registers (a lane compare + select)
                        if (sp < 64)
                            stk0 = lane_id() == sp ? e : stk0;
                        else
                            stk1 = lane_id() == sp - 64 ? e : stk1;
                        ++sp;
                    } else {
                        overflow = true;
                    }
                }
            }
        } else {
            // leaf: entry = -((first << 3 | (count - 1)) + 1).  All kLeafMax records are fetched in
            // one burst of scalar loads (the triangle array is padded by kLeafMax records), then the
            // leaf's own triangles are tested from registers.
            int32_t code = -entry - 1;
            int32_t first = code >> 3, cnt = (code & 7) + 1;
            const uint32_t CONST_AS* tp = (const uint32_t CONST_AS*)(tris + first);
            uint32_t tw[12 * kLeafMax];
#pragma unroll
            for (int i = 0; i < 12 * kLeafMax; ++i) tw[i] = tp[i];
            if (STATS) {
                ts.tri_wave += cnt;
                ts.tri_lane += valid ? cnt : 0;
            }
#pragma unroll
            for (int j = 0; j < kLeafMax; ++j) {
                if (j >= cnt) break;
                const uint32_t* w3 = tw + 12 * j;
                const float v0x = __uint_as_float(w3[0]), v0y = __uint_as_float(w3[1]), v0z = __uint_as_float(w3[2]);
                const int32_t id = (int32_t)w3[3];
                const float e1x = __uint_as_float(w3[4]), e1y = __uint_as_float(w3[5]), e1z = __uint_as_float(w3[6]);
                const float e2x = __uint_as_float(w3[8]), e2y = __uint_as_float(w3[9]), e2z = __uint_as_float(w3[10]);
                float px = d[1] * e2z - d[2] * e2y;
                float py = d[2] * e2x - d[0] * e2z;
                float pz = d[0] * e2y - d[1] * e2x;
                float det = e1x * px + e1y * py + e1z * pz;
                float sx = o[0] - v0x, sy = o[1] - v0y, sz = o[2] - v0z;
                float qx = sy * e1z - sz * e1y;
                float qy = sz * e1x - sx * e1z;
                float qz = sx * e1y - sy * e1x;
                float inv_det = __builtin_amdgcn_rcpf(det);
                float u = (sx * px + sy * py + sz * pz) * inv_det;
                float v = (d[0] * qx + d[1] * qy + d[2] * qz) * inv_det;
                float t = (e2x * qx + e2y * qy + e2z * qz) * inv_det;
                bool h = valid && det != 0.0f && u >= 0.0f && v >= 0.0f && u + v <= 1.0f && t >= t_near;
                bool take = h && (t < t_best || (t == t_best && (id_best < 0 || id < id_best)));
                t_best = take ? t : t_best;
                id_best = take ? id : id_best;
            }
        }
        if (sp == 0) break;
        --sp;
        entry = sp < 64 ? __builtin_amdgcn_readlane(stk0, sp) : __builtin_amdgcn_readlane(stk1, sp - 64);
    }
    if (overflow && lane_id() == 0) atomicOr(err, kErrStack);
    if (STATS) ts.hits += (id_best >= 0) ? 1 : 0;
}

// Validate an agent's view; returns false (and flags the error) if it cannot be rendered.
__device__ __forceinline__ bool view_ok(const RenderArgs& a, const vf_view& vw) {
    uint32_t bits = 0;
    if (vw.scene_id < 0 || vw.scene_id >= a.n_scenes) bits |= kErrScene;
    if (vw.H < 1 || vw.W < 1 || vw.H > a.max_h || vw.W > a.max_w || !(vw.hfov > 0.f && vw.hfov < 3.1415926f))
        bits |= kErrView;
    if (vw.out_offset < 0 || vw.out_offset + (int64_t)vw.H * vw.W > a.out_pixels) bits |= kErrPixels;
    if (bits == 0 && !a.scenes[vw.scene_id].valid) bits |= kErrScene;
    if (bits) {
        if (threadIdx.x == 0) atomicOr(a.err, bits);
        return false;
    }
    return true;
}

template <bool FUSED, bool STATS>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8)))
k_render(RenderArgs a) {
    __shared__ float pose[17];
    __shared__ int ok_shared;
    const int g = logical_group(a.total_groups);
    const int agent = g / a.groups_per_agent;
    const int group = g - agent * a.groups_per_agent;
    const int wave = threadIdx.x >> 6;
    const int lane = lane_id();

    int64_t slot = a.env_idx ? (int64_t)a.env_idx[agent] : (int64_t)agent;
    if (slot < 0 || slot >= a.n_slots) {
        if (threadIdx.x == 0 && group == 0) atomicOr(a.err, kErrSlot);
        return;
    }
    if (FUSED) {
        if (threadIdx.x == 0) {
            float s[17], act[4], o[17];
            for (int i = 0; i < 17; ++i) s[i] = a.state[slot * 17 + i];
            for (int i = 0; i < 4; ++i) act[i] = a.action[(int64_t)agent * 4 + i];
            dyn_step(a.dyn, s, act, o);
            for (int i = 0; i < 17; ++i) pose[i] = o[i];
            // every workgroup of the agent read the old state before its arrival;
            // the last to arrive writes the new one
            __threadfence();
            int prev = atomicAdd(&a.counters[slot], 1);
            if (prev == a.groups_per_agent - 1) {
                for (int i = 0; i < 17; ++i) a.state[slot * 17 + i] = o[i];
                atomicExch(&a.counters[slot], 0);
            }
        }
    } else {
        if (threadIdx.x < 17) pose[threadIdx.x] = a.state[slot * 17 + threadIdx.x];
    }
    vf_view vw = a.views[agent];
    if (threadIdx.x == 0) ok_shared = view_ok(a, vw) ? 1 : 0;
    __syncthreads();
    if (!ok_shared) return;

    const int tiles_x = (vw.W + kTile - 1) / kTile;
    const int tiles_y = (vw.H + kTile - 1) / kTile;
    const int tile = group * kWavesPerBlock + wave;
    if (tile >= tiles_x * tiles_y) return;
    const int ty = tile / tiles_x, tx = tile - ty * tiles_x;
    const int r = ty * kTile + (lane >> 3), c = tx * kTile + (lane & 7);
    const bool valid = r < vw.H && c < vw.W;

    float rot[9];
    quat_rot(pose + 3, rot);
    float o[3] = {pose[0], pose[1], pose[2]};
    float d[3];
    pixel_ray(rot, tanf(0.5f * vw.hfov), vw.H, vw.W, r, c, d);
    const SceneDesc sc = a.scenes[vw.scene_id];
    float t_best;
    int32_t id_best;
    TraceStats ts = {0, 0, 0, 0, 0, 0};
    trace_packet<STATS>(sc, valid, o, d, vw.near_clip, vw.far_clip, t_best, id_best, a.err, ts);
    if (valid) {
        int64_t pix = vw.out_offset + (int64_t)r * vw.W + c;
        if (a.depth) a.depth[pix] = id_best >= 0 ? t_best : vw.miss_depth;
        if (a.tri_id) a.tri_id[pix] = id_best;
        if (a.rgb) {
            int64_t plane = (int64_t)vw.H * vw.W;
            uint8_t* dst = a.rgb + 3 * vw.out_offset + (int64_t)r * vw.W + c;
            if (id_best >= 0 && sc.rgb) {
                const uint8_t* src = sc.rgb + 3 * (int64_t)id_best;
                dst[0] = src[0];
                dst[plane] = src[1];
                dst[2 * plane] = src[2];
            } else {
                dst[0] = 0;
                dst[plane] = 0;
                dst[2 * plane] = 0;
            }
        }
    }
    if (STATS) {
        // wave reduction of the per-lane counters, one atomic per counter per wave
        unsigned long long v[6] = {ts.node_lane, ts.box_lane, ts.tri_lane, ts.node_wave, ts.tri_wave, ts.hits};
        unsigned long long rays = valid ? 1 : 0;
        for (int off = 32; off > 0; off >>= 1) {
            for (int i = 0; i < 6; ++i) v[i] += __shfl_xor(v[i], off);
            rays += __shfl_xor(rays, off);
        }
        if (lane == 0) {
            atomicAdd(&a.stats[0], rays);
            atomicAdd(&a.stats[1], v[0]);
            atomicAdd(&a.stats[2], v[1]);
            atomicAdd(&a.stats[3], v[2]);
            atomicAdd(&a.stats[4], v[3] / 64);   // wave-level counts were added by every lane
            atomicAdd(&a.stats[5], v[4] / 64);
            atomicAdd(&a.stats[6], v[1]);
            atomicAdd(&a.stats[7], v[5]);
        }
    }
}

__global__ void __launch_bounds__(256) k_step(StepArgs a) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    int64_t slot = a.env_idx ? (int64_t)a.env_idx[i] : (int64_t)i;
    if (slot < 0 || slot >= a.n_slots) {
        atomicOr(a.err, kErrSlot);
        return;
    }
    float s[17], act[4], o[17];
    for (int k = 0; k < 17; ++k) s[k] = a.state[slot * 17 + k];
    for (int k = 0; k < 4; ++k) act[k] = a.action[(int64_t)i * 4 + k];
    dyn_step(a.dyn, s, act, o);
    for (int k = 0; k < 17; ++k) a.state[slot * 17 + k] = o[k];
}

// Copy state rows idx[i] -> out[i] (one thread per value).
__global__ void k_gather_rows(const float* __restrict__ state, const int32_t* __restrict__ idx, int32_t n,
                              float* __restrict__ out) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * 17) return;
    int a = i / 17, k = i - a * 17;
    out[i] = state[(int64_t)idx[a] * 17 + k];
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
hipError_t launch_step(const StepArgs& a, hipStream_t st) {
    if (a.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_step, dim3((a.n + 255) / 256), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_gather_rows(const float* state, const int32_t* idx, int32_t n, float* out, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_rows, dim3((n * 17 + 255) / 256), dim3(256), 0, st, state, idx, n, out);
    return hipGetLastError();
}

hipError_t launch_render(RenderArgs a, bool fused, bool stats, hipStream_t st) {
    if (a.n <= 0) return hipSuccess;
    int tiles = ((a.max_h + kTile - 1) / kTile) * ((a.max_w + kTile - 1) / kTile);
    a.groups_per_agent = (tiles + kWavesPerBlock - 1) / kWavesPerBlock;
    int64_t total = (int64_t)a.n * a.groups_per_agent;
    if (total > 0x7fffffff) return hipErrorInvalidValue;
    a.total_groups = (int32_t)total;
    dim3 grid((unsigned)total), block(256);
    if (fused) {
        if (stats)
            hipLaunchKernelGGL((k_render<true, true>), grid, block, 0, st, a);
        else
            hipLaunchKernelGGL((k_render<true, false>), grid, block, 0, st, a);
    } else {
        if (stats)
            hipLaunchKernelGGL((k_render<false, true>), grid, block, 0, st, a);
        else
            hipLaunchKernelGGL((k_render<false, false>), grid, block, 0, st, a);
    }
    return hipGetLastError();
}

}  // namespace vf
