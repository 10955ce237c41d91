// Batched step + ray-cast render kernels (Sec. III-A dynamics, Sec. III-B views).
//
// One wavefront traces one 16 x 4 pixel packet (kTileH x kTileW) of one agent.  The packet walks
// the 4-wide BVH together: every node and leaf triangle is fetched once per
// wavefront through the scalar data path (wave-uniform address), each lane
// tests its own ray, and ballots decide which children the packet visits.  The
// traversal stack is wave-uniform and lives in VGPR lanes, one entry per lane (a
// lane-select write and v_readlane, the stack pointer in an SGPR): one VGPR while every
// resident BVH is at most kShallowDepth levels deep, two otherwise.  Children are
// pushed far-to-near using the node's precomputed order for the packet's
// direction octant, so the nearest child is popped first and lanes that have
// found a closer hit cull the rest by their per-lane t.  The traversal is
// compiled for each combination of fixed ray-direction signs a packet can have
// (one octant: 8; one mixed axis: 12; the general case): where every ray of the
// packet has the same sign on an axis, the near and far slab planes of that axis
// are known at compile time and the box test drops its per-axis min/max.
//
// Launch: one workgroup = kWavesPerBlock wavefronts (one by default) = that many
// tiles of one agent; the grid covers n agents x ceil(tiles(max_h, max_w) /
// kWavesPerBlock) groups.  Workgroups are remapped so
// each XCD (workgroup id mod 8) processes a contiguous range of agents, keeping
// one agent's (and, with agents grouped by scene, one scene's) traffic in one L2.  Within its range an
// XCD may take the workgroups in an order given by k_group_order, or by k_step_order together with a
// split step's dynamics (longest packets first); every wavefront reports its traversal work for the next
// launch's order.
//
// The fused kernel (vf_step with views) first advances the agent's dynamics in
// one lane per workgroup (every workgroup of the agent computes the same bits),
// then renders at the new pose; the last workgroup of the agent to arrive on the
// agent's counter writes the new state, so the state can be updated in place.
#include "dynamics.h"
#include "noise.h"
#include "swarm.h"
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

// Counters of the counting variant.  *_lane: work issued per lane (every valid lane at every node and
// leaf its packet visits); need_*: the part a lane's own ray asked for -- visits of nodes and leaves
// whose box that ray entered (with its best depth at the time), the work a traversal of that ray alone
// in the packet's order would do (with several rays per lane, a lane counts when any of them entered).
struct TraceStats {
    unsigned long long node_lane, box_lane, tri_lane, node_wave, tri_wave, hits, box_ops, need_node, need_box,
        need_tri, member_lane;
};

// VALU operations of one ray-box test by the axes whose direction sign is fixed for the packet
__host__ __device__ constexpr int box_test_ops(int fix) {
    return fix == 7 ? 11 : fix == 0 ? 18 : 14;   // one axis mixed: 14
}

// One slab of the box test.  A fixed axis (every ray of the packet has the sign SGNA there, by the
// sign bit, as the reciprocal takes it) knows its near and far plane at compile time and takes the
// exit growth from the grown reciprocal; a mixed axis orders the two plane distances per lane.
template <bool FIXA, bool SGNA>
__device__ __forceinline__ void slab(float lo, float hi, float inv, float oi, float ing, float oig, float grow2,
                                     float& tn, float& tf) {
    if constexpr (FIXA) {
        tn = fmaf(SGNA ? hi : lo, inv, oi);
        tf = fmaf(SGNA ? lo : hi, ing, oig);
    } else {
        const float t0 = fmaf(lo, inv, oi), t1 = fmaf(hi, inv, oi);
        tn = fminf(t0, t1);
        tf = fmaxf(t0, t1) * grow2;
    }
}

// FIX: bit a set = every ray of the packet has the direction sign of bit a of SGN on axis a (set =
// negative).  FIX = 7: one octant, all slab planes known at compile time; FIX = 0: the general test.
template <int NR, bool STATS, int FIX, int SGN, bool DEEP>
__device__ __forceinline__ void trace_packet(const SceneDesc& sc, const bool (&valid)[NR], const float o[3],
                                             const float (&d)[NR][3], float t_near, float t_far,
                                             float (&t_best)[NR], int32_t (&id_best)[NR], uint32_t* err,
                                             TraceStats& ts, int32_t& work) {
    const Node CONST_AS* nodes = (const Node CONST_AS*)sc.nodes;
    const Tri CONST_AS* tris = (const Tri CONST_AS*)sc.tris;
    float inv[NR][3], oi[NR][3];
    int n_valid = 0;
    bool any = false;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        for (int k = 0; k < 3; ++k) {
            inv[r][k] = safe_inv(d[r][k]);
            oi[r][k] = -o[k] * inv[r][k];
        }
        // a lane outside the image gets a best depth of -1: no box or triangle test passes for it
        t_best[r] = valid[r] ? t_far : -1.0f;
        id_best[r] = -1;
        any = any || valid[r];
        n_valid += valid[r] ? 1 : 0;
    }
    // 1 + 2 gamma_3 (Ize 2013) widens the slab exit.  The fused form lo * (1/d) - o * (1/d) adds an
    // error of about |o| 2^-24 in space; the child boxes' padding of 2^-19 (|x| + 1) plus the entry
    // shrunk by the same relative margin (distance x 4e-7) always exceed it, so no box a ray meets
    // is rejected.  The shrink is applied to the other side of the comparison: to the exit growth
    // and to a copy of the best depth refreshed after every leaf.
    const float grow2 = 1.000001f, unshrink = 1.0000005f;   // >= grow / shrink and 1 / shrink
    float tb_box[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) tb_box[r] = t_best[r] * unshrink;
    // far-plane distances of a known-octant packet come out grown: (x - o) (1/d) grow2 as one fused
    // multiply-add of the products rounded once more (a relative 2^-24 each, far inside the padding)
    float ing[NR][3], oig[NR][3];
#pragma unroll
    for (int r = 0; r < NR; ++r)
        for (int k = 0; k < 3; ++k) {
            ing[r][k] = inv[r][k] * grow2;
            oig[r][k] = oi[r][k] * grow2;
        }
    int oct = SGN;
    if constexpr (FIX != 7) {
        oct = (d[0][0] < 0.f ? 1 : 0) | (d[0][1] < 0.f ? 2 : 0) | (d[0][2] < 0.f ? 4 : 0);
        oct = uniform_i(oct);
    }
    if (__ballot(any) == 0ull) return;

    // the stack: entry i in lane i of stk0, and for deep BVHs lane i - 64 of stk1
    int stk0 = 0, stk1 = 0;
    int sp = 0;
    int32_t entry = 0;          // root: inner node 0
    // counting variant (one ray per lane): the lanes whose ray entered the entry being visited, kept
    // beside the stack as two 32-bit halves per stack position
    uint64_t act = __ballot(any);
    uint32_t mlo0 = 0, mhi0 = 0, mlo1 = 0, mhi1 = 0;
    uint64_t child_m[kWidth];
    while (true) {
        if (entry >= 0) {
            // the whole 128-byte node in one burst of wave-uniform (scalar) loads
            const uint32_t CONST_AS* np = (const uint32_t CONST_AS*)(nodes + entry);
            uint32_t w[kNodeWords];
#pragma unroll
            for (int i = 0; i < kNodeWords; ++i) w[i] = np[i];
            // words the traversal may not read (leaf counts, padding, other octants' orders): naming
            // them keeps the node one run of 16-dword loads
            if constexpr (kWidth == 4) {
                asm volatile("" ::"s"(w[28]), "s"(w[31]));
                if constexpr (FIX == 7) asm volatile("" ::"s"(w[29]), "s"(w[30]));
            } else {
#pragma unroll
                for (int i = kOrderWord; i < kNodeWords; ++i) asm volatile("" ::"s"(w[i]));
            }
            work += 3;      // four box tests and the pushes: about three triangle tests' worth
            if (STATS) {
                ts.node_wave += 1;
                ts.node_lane += n_valid;
                ts.box_lane += kWidth * n_valid;
                ts.box_ops += (unsigned long long)box_test_ops(FIX) * kWidth * n_valid;
                const unsigned mine = (unsigned)((act >> lane_id()) & 1ull) * (unsigned)n_valid;
                ts.need_node += mine;
                ts.need_box += kWidth * mine;
            }
            // bit k: some ray of the packet enters child k's box (empty slots hold a box no ray enters)
            uint32_t hb = 0;
#pragma unroll
            for (int k = 0; k < kWidth; ++k) {
                const float lox = __uint_as_float(w[k]), hix = __uint_as_float(w[kWidth + k]);
                const float loy = __uint_as_float(w[2 * kWidth + k]), hiy = __uint_as_float(w[3 * kWidth + k]);
                const float loz = __uint_as_float(w[4 * kWidth + k]), hiz = __uint_as_float(w[5 * kWidth + k]);
                uint64_t m = 0;   // lanes with a ray entering the box (the union over the lane's rays)
                if constexpr (FIX != 0) {
#pragma unroll
                    for (int r = 0; r < NR; ++r) {
                        float tnx, tfx, tny, tfy, tnz, tfz;
                        slab<(FIX & 1) != 0, (SGN & 1) != 0>(lox, hix, inv[r][0], oi[r][0], ing[r][0], oig[r][0],
                                                             grow2, tnx, tfx);
                        slab<(FIX & 2) != 0, (SGN & 2) != 0>(loy, hiy, inv[r][1], oi[r][1], ing[r][1], oig[r][1],
                                                             grow2, tny, tfy);
                        slab<(FIX & 4) != 0, (SGN & 4) != 0>(loz, hiz, inv[r][2], oi[r][2], ing[r][2], oig[r][2],
                                                             grow2, tnz, tfz);
                        const float t0 = fmaxf(fmaxf(tnx, tny), fmaxf(tnz, t_near));
                        const float t1 = fminf(fminf(tfx, tfy), fminf(tfz, tb_box[r]));
                        m |= __ballot(t0 <= t1);
                    }
                } else
#pragma unroll
                for (int r = 0; r < NR; ++r) {
                    // (lo - o) / d as one fused multiply-add: lo * (1/d) - o * (1/d)
                    float tx0 = fmaf(lox, inv[r][0], oi[r][0]), tx1 = fmaf(hix, inv[r][0], oi[r][0]);
                    float ty0 = fmaf(loy, inv[r][1], oi[r][1]), ty1 = fmaf(hiy, inv[r][1], oi[r][1]);
                    float tz0 = fmaf(loz, inv[r][2], oi[r][2]), tz1 = fmaf(hiz, inv[r][2], oi[r][2]);
                    // entry * shrink <= min(exit * grow, best)  <=>  entry <= min(exit * grow / shrink, best / shrink)
                    float t0 = fmaxf(fmaxf(fminf(tx0, tx1), fminf(ty0, ty1)), fmaxf(fminf(tz0, tz1), t_near));
                    float t1 = fminf(fminf(fmaxf(tx0, tx1), fmaxf(ty0, ty1)), fmaxf(tz0, tz1)) * grow2;
                    m |= __ballot(t0 <= fminf(t1, tb_box[r]));
                }
                hb |= (m != 0ull ? 1u : 0u) << k;
                if (STATS) child_m[k] = m;
            }
            // the octant's child slots, near to far
            uint32_t slots;
            if constexpr (kWidth == 4) {
                const uint64_t ord = ((uint64_t)w[kOrderWord + 1] << 32) | w[kOrderWord];
                slots = (uint32_t)(ord >> (8 * oct)) & 255u;
            } else {
                const uint32_t o01 = (oct & 1) ? w[kOrderWord + 1] : w[kOrderWord];
                const uint32_t o23 = (oct & 1) ? w[kOrderWord + 3] : w[kOrderWord + 2];
                const uint32_t o45 = (oct & 1) ? w[kOrderWord + 5] : w[kOrderWord + 4];
                const uint32_t o67 = (oct & 1) ? w[kOrderWord + 7] : w[kOrderWord + 6];
                const uint32_t o03 = (oct & 2) ? o23 : o01, o47 = (oct & 2) ? o67 : o45;
                slots = (oct & 4) ? o47 : o03;
            }
            // push hit children far-to-near so the nearest is on top
#pragma unroll
            for (int i = kWidth - 1; i >= 0; --i) {
                const uint32_t k = (slots >> (kWidthBits * i)) & (uint32_t)(kWidth - 1);
                if ((hb >> k) & 1u) {
                    // the slot word is the stack entry: a node index, or the leaf's encoded range
                    const int32_t e01 = (int32_t)((k & 1u) ? w[kChildWord + 1] : w[kChildWord]);
                    const int32_t e23 = (int32_t)((k & 1u) ? w[kChildWord + 3] : w[kChildWord + 2]);
                    int32_t e = (k & 2u) ? e23 : e01;
                    if constexpr (kWidth == 8) {
                        const int32_t e45 = (int32_t)((k & 1u) ? w[kChildWord + 5] : w[kChildWord + 4]);
                        const int32_t e67 = (int32_t)((k & 1u) ? w[kChildWord + 7] : w[kChildWord + 6]);
                        e = (k & 4u) ? ((k & 2u) ? e67 : e45) : e;
                    }
                    // write lane sp of the stack registers (lane compares + selects, no branch); the
                    // depth limit of the build bounds sp below kStackCap, and the launch takes the
                    // one-register form only when every resident BVH is at most kShallowDepth deep
                    stk0 = lane_id() == sp ? e : stk0;
                    if constexpr (DEEP) stk1 = lane_id() == sp - 64 ? e : stk1;
                    if (STATS) {
                        const uint64_t cm = child_m[k];
                        mlo0 = lane_id() == sp ? (uint32_t)cm : mlo0;
                        mhi0 = lane_id() == sp ? (uint32_t)(cm >> 32) : mhi0;
                        if constexpr (DEEP) {
                            mlo1 = lane_id() == sp - 64 ? (uint32_t)cm : mlo1;
                            mhi1 = lane_id() == sp - 64 ? (uint32_t)(cm >> 32) : mhi1;
                        }
                    }
                    ++sp;
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
            // the padding words are never used; naming them keeps the leaf one run of 16-dword loads
            // instead of many small ones
#pragma unroll
            for (int j = 0; j < kLeafMax; ++j) asm volatile("" ::"s"(tw[12 * j + 7]), "s"(tw[12 * j + 11]));
            work += cnt;
            if (STATS) {
                ts.tri_wave += cnt;
                ts.tri_lane += cnt * n_valid;
                ts.need_tri += (unsigned)cnt * (unsigned)((act >> lane_id()) & 1ull) * (unsigned)n_valid;
            }
#pragma unroll
            for (int j = 0; j < kLeafMax; ++j) {
                if (j >= cnt) break;
                const uint32_t* w3 = tw + 12 * j;
                const float v0x = __uint_as_float(w3[0]), v0y = __uint_as_float(w3[1]), v0z = __uint_as_float(w3[2]);
                const int32_t id = (int32_t)w3[3];
                const float e1x = __uint_as_float(w3[4]), e1y = __uint_as_float(w3[5]), e1z = __uint_as_float(w3[6]);
                const float e2x = __uint_as_float(w3[8]), e2y = __uint_as_float(w3[9]), e2z = __uint_as_float(w3[10]);
                // S = o - v0 and Q = S x e1 do not depend on the ray direction: shared by the lane's rays
                const float sx = o[0] - v0x, sy = o[1] - v0y, sz = o[2] - v0z;
                const float qx = sy * e1z - sz * e1y;
                const float qy = sz * e1x - sx * e1z;
                const float qz = sx * e1y - sy * e1x;
                const float tq = e2x * qx + e2y * qy + e2z * qz;
#pragma unroll
                for (int r = 0; r < NR; ++r) {
                    const float* dr = d[r];
                    float px = dr[1] * e2z - dr[2] * e2y;
                    float py = dr[2] * e2x - dr[0] * e2z;
                    float pz = dr[0] * e2y - dr[1] * e2x;
                    float det = e1x * px + e1y * py + e1z * pz;
                    float inv_det = __builtin_amdgcn_rcpf(det);
                    float u = (sx * px + sy * py + sz * pz) * inv_det;
                    float v = (dr[0] * qx + dr[1] * qy + dr[2] * qz) * inv_det;
                    float t = tq * inv_det;
                    // bitwise, not short-circuit: no divergent branches.  An empty best (id -1) compares
                    // as the largest unsigned id, so any hit at the same depth replaces it.
                    // det == 0 needs no test of its own: 1/det is infinite, so u and v are infinite or
                    // NaN and one of the comparisons fails
                    const bool h = (u >= 0.0f) & (v >= 0.0f) & (u + v <= 1.0f) & (t >= t_near);
                    // nearer, or as near with a lower id, as one unsigned compare of (depth bits, id): a
                    // depth >= t_near > 0 (the view check rejects other clip ranges) orders by its bits; lanes
                    // outside the image (best depth -1) are kept out by their flag
                    const uint64_t key = ((uint64_t)__float_as_uint(t) << 32) | (uint32_t)id;
                    const uint64_t bk = ((uint64_t)__float_as_uint(t_best[r]) << 32) | (uint32_t)id_best[r];
                    const bool take = h & valid[r] & (key < bk);
                    t_best[r] = take ? t : t_best[r];
                    id_best[r] = take ? id : id_best[r];
                }
            }
#pragma unroll
            for (int r = 0; r < NR; ++r) tb_box[r] = t_best[r] * unshrink;
        }
        if (sp == 0) break;
        --sp;
        if constexpr (DEEP) {
            const int32_t a0 = __builtin_amdgcn_readlane(stk0, sp & 63);
            const int32_t a1 = __builtin_amdgcn_readlane(stk1, sp & 63);
            entry = sp < 64 ? a0 : a1;
            if (STATS) {
                const uint32_t l0 = __builtin_amdgcn_readlane(mlo0, sp & 63), h0 = __builtin_amdgcn_readlane(mhi0, sp & 63);
                const uint32_t l1 = __builtin_amdgcn_readlane(mlo1, sp & 63), h1 = __builtin_amdgcn_readlane(mhi1, sp & 63);
                act = sp < 64 ? ((uint64_t)h0 << 32 | l0) : ((uint64_t)h1 << 32 | l1);
            }
        } else {
            entry = __builtin_amdgcn_readlane(stk0, sp);
            if (STATS) {
                const uint32_t l0 = __builtin_amdgcn_readlane(mlo0, sp), h0 = __builtin_amdgcn_readlane(mhi0, sp);
                act = (uint64_t)h0 << 32 | l0;
            }
        }
    }
    if (STATS)
        for (int r = 0; r < NR; ++r) ts.hits += (valid[r] && id_best[r] >= 0) ? 1 : 0;
}

// Validate an agent's view; returns false (and flags the error) if it cannot be rendered.
__device__ __forceinline__ bool view_ok(const RenderArgs& a, const vf_view& vw) {
    uint32_t bits = 0;
    if (vw.scene_id < 0 || vw.scene_id >= a.n_scenes) bits |= kErrScene;
    if (vw.H < 1 || vw.W < 1 || vw.H > a.max_h || vw.W > a.max_w || !(vw.hfov > 0.f && vw.hfov < 3.1415926f) ||
        !(vw.near_clip > 0.f && vw.far_clip > vw.near_clip))
        bits |= kErrView;
    if (vw.out_offset < 0 || vw.out_offset + (int64_t)vw.H * vw.W > a.out_pixels) bits |= kErrPixels;
    if (bits == 0 && !a.scenes[vw.scene_id].valid) bits |= kErrScene;
    if (bits) {
        if (threadIdx.x == 0) atomicOr(a.err, bits);
        return false;
    }
    return true;
}

template <bool FUSED, bool STATS, bool NOISE, bool SWARM, bool DEEP>
__device__ __forceinline__ void render_body(const RenderArgs& a) {
    __shared__ float pose[17];
    __shared__ int ok_shared;
    int g = logical_group(a.total_groups);
    if (a.group_order) g = a.group_order[g];
    const int la = g / a.groups_per_agent;
    const int group = g - la * a.groups_per_agent;
    const int agent = a.order ? a.order[la] : la;
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
    // the view and scene records stay in vector registers: the traversal needs the scalar ones
    const vf_view vw = a.views[agent];
    if (threadIdx.x == 0) ok_shared = view_ok(a, vw) ? 1 : 0;
    __syncthreads();
    if (!ok_shared) return;
    const SceneDesc sc = a.scenes[vw.scene_id];


    // the wavefront's packet: kPacketRows x kPacketCols tiles of kTileH x kTileW, one ray of each per lane
    constexpr int NR = kPacketRows * kPacketCols;
    const int th = kTileH * kPacketRows, tw_ = kTileW * kPacketCols;
    const int tiles_x = (vw.W + tw_ - 1) / tw_;
    const int tiles_y = (vw.H + th - 1) / th;
    const int tile = group * kWavesPerBlock + wave;
    if (tile >= tiles_x * tiles_y) return;
    const int ty = tile / tiles_x, tx = tile - ty * tiles_x;
    int row[NR], col[NR];
    bool valid[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        row[k] = ty * th + (k / kPacketCols) * kTileH + lane / kTileW;
        col[k] = tx * tw_ + (k % kPacketCols) * kTileW + lane % kTileW;
        valid[k] = row[k] < vw.H && col[k] < vw.W;
    }

    float rot[9], o[3];
    camera_pose(pose, vw, o, rot);
    float d[NR][3];
    const float tan_h = tanf(0.5f * vw.hfov);
#pragma unroll
    for (int k = 0; k < NR; ++k) pixel_ray(rot, tan_h, vw.H, vw.W, row[k], col[k], d[k]);
    float t_best[NR];
    int32_t id_best[NR];
    TraceStats ts = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    int32_t work = 0;
    // one octant for every ray of the packet (lanes outside the image do not count: their best depth
    // of -1 fails every test)?  Then the traversal with the slab planes fixed at compile time.
    uint64_t m_neg[3] = {0, 0, 0}, m_pos[3] = {0, 0, 0};
#pragma unroll
    for (int k = 0; k < NR; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            m_neg[c] |= __ballot(valid[k] && signbit(d[k][c]));
            m_pos[c] |= __ballot(valid[k] && !signbit(d[k][c]));
        }
    // axes on which every ray of the packet has one sign, and those signs
    int fix = 0, sgn = 0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        if (m_neg[c] == 0 || m_pos[c] == 0) fix |= 1 << c;
        if (m_neg[c] != 0) sgn |= 1 << c;
    }
    sgn &= fix;
    if (!VF_OCTANT_PACKETS) fix = 0;
    if (!VF_PARTIAL_OCTANT && fix != 7) fix = 0;
    if (__builtin_popcount(fix) < 2) fix = 0;       // two or three mixed axes: the general test
#define VF_TRACE(F, S) trace_packet<NR, STATS, F, S, DEEP>(sc, valid, o, d, vw.near_clip, vw.far_clip, t_best, id_best, a.err, ts, work)
    switch (fix == 0 ? 0 : (fix << 3) | sgn) {
        case (7 << 3) | 0: VF_TRACE(7, 0); break;
        case (7 << 3) | 1: VF_TRACE(7, 1); break;
        case (7 << 3) | 2: VF_TRACE(7, 2); break;
        case (7 << 3) | 3: VF_TRACE(7, 3); break;
        case (7 << 3) | 4: VF_TRACE(7, 4); break;
        case (7 << 3) | 5: VF_TRACE(7, 5); break;
        case (7 << 3) | 6: VF_TRACE(7, 6); break;
        case (7 << 3) | 7: VF_TRACE(7, 7); break;
        case (6 << 3) | 0: VF_TRACE(6, 0); break;       // x mixed
        case (6 << 3) | 2: VF_TRACE(6, 2); break;
        case (6 << 3) | 4: VF_TRACE(6, 4); break;
        case (6 << 3) | 6: VF_TRACE(6, 6); break;
        case (5 << 3) | 0: VF_TRACE(5, 0); break;       // y mixed
        case (5 << 3) | 1: VF_TRACE(5, 1); break;
        case (5 << 3) | 4: VF_TRACE(5, 4); break;
        case (5 << 3) | 5: VF_TRACE(5, 5); break;
        case (3 << 3) | 0: VF_TRACE(3, 0); break;       // z mixed
        case (3 << 3) | 1: VF_TRACE(3, 1); break;
        case (3 << 3) | 2: VF_TRACE(3, 2); break;
        case (3 << 3) | 3: VF_TRACE(3, 3); break;
        default: VF_TRACE(0, 0); break;
    }
#undef VF_TRACE
    if (vw.swarm != 0) {
        // the other members of the view's swarm, through the swarm's tree (rebuilt for this launch); the
        // kernels without swarms leave the tree walk out
        if (!SWARM || vw.swarm < 0 || vw.swarm > a.swarm.n || !a.swarm.nodes) {
            if (lane == 0) atomicOr(a.err, kErrView);
        } else if constexpr (SWARM) {
            trace_swarm<NR, STATS>(a.swarm, vw.swarm - 1, slot, sc.n_tris, valid, o, d, vw.near_clip, t_best,
                                   id_best, ts.box_lane, ts.member_lane);
        }
    }
    // depth goes to the view's own target when the caller gave a table of them, else at out_offset
    float* const dbase = a.depth_views ? a.depth_views[agent] : (a.depth ? a.depth + vw.out_offset : nullptr);
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        if (!valid[k]) continue;
        const int64_t in_view = (int64_t)row[k] * vw.W + col[k];
        const int64_t pix = vw.out_offset + in_view;
        if (dbase) {
            float dv = id_best[k] >= 0 ? t_best[k] : vw.miss_depth;
            // epilogue noise: the separate pass's function of the same pixel, so the same bits
            if (NOISE && id_best[k] >= 0)
                dv = noisy_depth_px(a.noise, (uint32_t)vw.flags, (uint32_t)in_view, dv, vw.near_clip, vw.far_clip);
            dbase[in_view] = dv;
        }
        if (a.tri_id) a.tri_id[pix] = id_best[k];
        if (a.rgb) {
            const int64_t plane = (int64_t)vw.H * vw.W;
            uint8_t* dst = a.rgb + 3 * vw.out_offset + in_view;
            uint8_t ch[3] = {0, 0, 0};
            if (id_best[k] >= sc.n_tris) {
                ch[0] = a.swarm.rgb[0];
                ch[1] = a.swarm.rgb[1];
                ch[2] = a.swarm.rgb[2];
            } else if (id_best[k] >= 0 && sc.rgb) {
                const uint8_t* src = sc.rgb + 3 * (int64_t)id_best[k];
                ch[0] = src[0];
                ch[1] = src[1];
                ch[2] = src[2];
            }
            if (NOISE) noisy_rgb_px(a.noise, (uint32_t)vw.flags, (uint32_t)in_view, ch);
            dst[0] = ch[0];
            dst[plane] = ch[1];
            dst[2 * plane] = ch[2];
        }
    }
    if (a.cost && lane == 0)
        a.cost[(int64_t)g * kWavesPerBlock + wave] = work;
    if (STATS) {
        // wave reduction of the per-lane counters, one atomic per counter per wave
        unsigned long long v[11] = {ts.node_lane, ts.box_lane, ts.tri_lane, ts.node_wave, ts.tri_wave, ts.hits,
                                    ts.box_ops, ts.need_node, ts.need_box, ts.need_tri, ts.member_lane};
        unsigned long long rays = 0;
        for (int k = 0; k < NR; ++k) rays += valid[k] ? 1 : 0;
        for (int off = 32; off > 0; off >>= 1) {
            for (int i = 0; i < 11; ++i) v[i] += __shfl_xor(v[i], off);
            rays += __shfl_xor(rays, off);
        }
        if (lane == 0) {
            atomicAdd(&a.stats[0], rays);
            atomicAdd(&a.stats[1], v[0]);
            atomicAdd(&a.stats[2], v[1]);
            atomicAdd(&a.stats[3], v[2]);
            atomicAdd(&a.stats[4], v[3] / 64);   // wave-level counts were added by every lane
            atomicAdd(&a.stats[5], v[4] / 64);
            atomicAdd(&a.stats[6], v[6]);
            atomicAdd(&a.stats[7], v[5]);
            atomicAdd(&a.stats[8], v[7]);
            atomicAdd(&a.stats[9], v[8]);
            atomicAdd(&a.stats[10], v[9]);
            atomicAdd(&a.stats[11], v[10]);
        }
    }
}

// The render kernel of split launches: occupancy of kRenderWavesPerEu waves per SIMD for the traversal.
// SWARM: the views may show swarm members (the tree walk is compiled in).  DEEP: a resident BVH is deeper
// than kShallowDepth, so the traversal stack takes two registers.
template <bool STATS, bool NOISE, bool SWARM, bool DEEP>
__global__ void __launch_bounds__(64 * kWavesPerBlock) __attribute__((amdgpu_waves_per_eu(kRenderWavesPerEu)))
k_render(RenderArgs a) {
    render_body<false, STATS, NOISE, SWARM, DEEP>(a);
}

// The fused kernel (small batches: few workgroups, so occupancy matters less than keeping the one-lane
// FP64 dynamics and the traversal in registers): compiled for kFusedWavesPerEu waves per SIMD.
template <bool STATS, bool NOISE>
__global__ void __launch_bounds__(64 * kWavesPerBlock) __attribute__((amdgpu_waves_per_eu(kFusedWavesPerEu)))
k_render_fused(RenderArgs a) {
    render_body<true, STATS, NOISE, false, true>(a);   // swarms always take split launches
}

// Agent i's control step on its state slot.
__device__ __forceinline__ void step_agent(const StepArgs& a, int i) {
    if (i >= a.n) return;
    int64_t slot = a.env_idx ? (int64_t)a.env_idx[i] : (int64_t)i;
    if (slot < 0 || slot >= a.n_slots) {
        atomicOr(a.err, kErrSlot);
        return;
    }
    float s[17], act[4], o[17];
    for (int k = 0; k < 17; ++k) s[k] = a.state[slot * 17 + k];
    if (a.before)
        for (int k = 0; k < 17; ++k) a.before[(int64_t)i * 17 + k] = s[k];
    for (int k = 0; k < 4; ++k) act[k] = a.action[(int64_t)i * 4 + k];
    dyn_step(a.dyn, s, act, o);
    for (int k = 0; k < 17; ++k) a.state[slot * 17 + k] = o[k];
}

__global__ void __launch_bounds__(256) k_step(StepArgs a) { step_agent(a, blockIdx.x * blockDim.x + threadIdx.x); }


// Copy state rows idx[i] -> out[i] (one thread per value).
__global__ void k_gather_rows(const float* __restrict__ state, const int32_t* __restrict__ idx, int32_t n,
                              float* __restrict__ out) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * 17) return;
    int a = i / 17, k = i - a * 17;
    out[i] = state[(int64_t)idx[a] * 17 + k];
}

// p[0, n) = value (a kernel, not a memset, so the fill can be captured in a graph).
__global__ void k_fill_i32(int32_t* __restrict__ p, int64_t n, int32_t value) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

// Copy rows[i] -> state row idx[i] (one thread per value): puts saved states back.
__global__ void k_scatter_rows(float* __restrict__ state, const int32_t* __restrict__ idx, int32_t n,
                               const float* __restrict__ rows) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * 17) return;
    int a = i / 17, k = i - a * 17;
    state[(int64_t)idx[a] * 17 + k] = rows[i];
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t value, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)(blocks < 1024 ? blocks : 1024)), dim3(256), 0, st, p, n, value);
    return hipGetLastError();
}

hipError_t launch_scatter_rows(float* state, const int32_t* idx, int32_t n, const float* rows, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter_rows, dim3((n * 17 + 255) / 256), dim3(256), 0, st, state, idx, n, rows);
    return hipGetLastError();
}
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

// Spatial order of a batch (one workgroup): key = scene id, then a 2-D Morton code of the position on a
// 1024 x 1024 grid over the batch's own bounds; each agent's rank counted over the keys in LDS.  Consecutive
// logical agents -- and so the agents one XCD renders -- then share a scene region, which keeps the
// part of the BVH each XCD touches small enough for its L2.  The order changes which workgroup renders
// an agent, never what it renders.
__device__ __forceinline__ uint32_t spread10(uint32_t v) {
    v &= 1023u;
    v = (v | (v << 8)) & 0x00FF00FFu;
    v = (v | (v << 4)) & 0x0F0F0F0Fu;
    v = (v | (v << 2)) & 0x33333333u;
    v = (v | (v << 1)) & 0x55555555u;
    return v;
}

__global__ void __launch_bounds__(1024) k_order(OrderArgs a) {
    __shared__ unsigned long long keys[kOrderMax];
    __shared__ float red[4][32];
    const int t = threadIdx.x;
    // bounds of the positions
    float lx = INFINITY, ly = INFINITY, hx = -INFINITY, hy = -INFINITY;
    for (int i = t; i < a.n; i += blockDim.x) {
        int64_t slot = a.env_idx ? (int64_t)a.env_idx[i] : (int64_t)i;
        if (slot < 0 || slot >= a.n_slots) continue;
        float x = a.state[slot * 17], y = a.state[slot * 17 + 1];
        lx = fminf(lx, x);
        ly = fminf(ly, y);
        hx = fmaxf(hx, x);
        hy = fmaxf(hy, y);
    }
    for (int off = 32; off > 0; off >>= 1) {
        lx = fminf(lx, __shfl_xor(lx, off));
        ly = fminf(ly, __shfl_xor(ly, off));
        hx = fmaxf(hx, __shfl_xor(hx, off));
        hy = fmaxf(hy, __shfl_xor(hy, off));
    }
    const int w = t >> 6, nw = blockDim.x >> 6;
    if ((t & 63) == 0) {
        red[0][w] = lx;
        red[1][w] = ly;
        red[2][w] = hx;
        red[3][w] = hy;
    }
    __syncthreads();
    lx = red[0][0];
    ly = red[1][0];
    hx = red[2][0];
    hy = red[3][0];
    for (int k = 1; k < nw; ++k) {
        lx = fminf(lx, red[0][k]);
        ly = fminf(ly, red[1][k]);
        hx = fmaxf(hx, red[2][k]);
        hy = fmaxf(hy, red[3][k]);
    }
    const float sx = hx > lx ? 1023.0f / (hx - lx) : 0.0f, sy = hy > ly ? 1023.0f / (hy - ly) : 0.0f;
    for (int i = t; i < a.n; i += blockDim.x) {
        int64_t slot = a.env_idx ? (int64_t)a.env_idx[i] : (int64_t)i;
        uint32_t code = 0xFFFFFFFFu;
        if (slot >= 0 && slot < a.n_slots) {
            float x = a.state[slot * 17], y = a.state[slot * 17 + 1];
            uint32_t cx = (uint32_t)fminf(fmaxf((x - lx) * sx, 0.0f), 1023.0f);
            uint32_t cy = (uint32_t)fminf(fmaxf((y - ly) * sy, 0.0f), 1023.0f);
            uint32_t sid = (uint32_t)a.views[i].scene_id & 1023u;
            code = (sid << 20) | spread10(cx) | (spread10(cy) << 1);
        }
        keys[i] = ((unsigned long long)code << 32) | (uint32_t)i;
    }
    __syncthreads();
    // each agent's rank is the number of smaller keys (keys are distinct: the index is in the low bits)
    for (int i = t; i < a.n; i += blockDim.x) {
        const unsigned long long mine = keys[i];
        int rank = 0;
        for (int j = 0; j < a.n; ++j) rank += keys[j] < mine ? 1 : 0;
        a.order[rank] = i;
    }
}

hipError_t launch_order(const OrderArgs& a, hipStream_t st) {
    if (a.n <= 0 || a.n > kOrderMax) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_order, dim3(1), dim3(1024), 0, st, a);
    return hipGetLastError();
}

// Cost order of a launch's workgroups: the render hands the hardware workgroup ids in turn to the eight
// XCDs, and each XCD takes its contiguous range of logical groups in order (the remap above).  Within each
// XCD's range the groups are put in decreasing order of the traversal work their wavefronts reported in
// the previous launch of the same shape (a counting sort over 32 buckets, two per octave, in chunks of
// kGroupOrderChunk groups: one workgroup per chunk), so long packets start first and short ones fill the
// end of the launch instead of a few long ones running alone.  Work is kept per logical group, so a change of the agents' spatial order
// between launches only makes the estimate staler.  Any cost values, stale or uninitialised, give a valid
// permutation of each range: the bucket of every group is computed once and kept in LDS for both passes.
// The order changes which workgroup renders a packet, never what it renders.
__device__ __forceinline__ int cost_bucket(uint32_t c) {
    // two buckets per octave of c + 1, largest first
    const uint32_t v = c < 0xFFFFFFFFu ? c + 1u : c;
    const int lg = 31 - __clz(v);
    const int half = lg > 0 ? (int)((v >> (lg - 1)) & 1u) : 0;
    const int b = 2 * lg + half;
    return kCostBuckets - 1 - (b < kCostBuckets - 1 ? b : kCostBuckets - 1);
}

// One workgroup of the cost order: XCD range (block & 7), chunk (block >> 3); any workgroup size of at
// least kCostBuckets threads.
constexpr int kOrderBatch = 8;
__device__ __forceinline__ void group_order_block(const GroupOrderArgs& a, int block) {
    __shared__ uint8_t bucket[kGroupOrderChunk];
    __shared__ int32_t off[kCostBuckets];
    const int t = threadIdx.x, x = block & 7, chunk = block >> 3;
    const int q = a.total >> 3, r = a.total & 7;
    const int range = q + (x < r ? 1 : 0);
    const int begin = x * q + (x < r ? x : r) + chunk * kGroupOrderChunk;
    const int left = range - chunk * kGroupOrderChunk;
    const int size = left < kGroupOrderChunk ? left : kGroupOrderChunk;      // <= 0: nothing to sort
    if (t < kCostBuckets) off[t] = 0;
    __syncthreads();
    // kOrderBatch groups' cost loads in flight per thread, then their buckets
    for (int i0 = t; i0 < size; i0 += kOrderBatch * (int)blockDim.x) {
        uint32_t c[kOrderBatch];
#pragma unroll
        for (int u = 0; u < kOrderBatch; ++u) {
            const int i = i0 + u * (int)blockDim.x;
            c[u] = 0;
            if (i < size)
                for (int w = 0; w < kWavesPerBlock; ++w) {
                    const uint32_t cw = (uint32_t)a.cost[(int64_t)(begin + i) * kWavesPerBlock + w];
                    c[u] = c[u] + cw < c[u] ? 0xFFFFFFFFu : c[u] + cw;
                }
        }
#pragma unroll
        for (int u = 0; u < kOrderBatch; ++u) {
            const int i = i0 + u * (int)blockDim.x;
            if (i < size) {
                const int b = cost_bucket(c[u]);
                bucket[i] = (uint8_t)b;
                atomicAdd(&off[b], 1);
            }
        }
    }
    __syncthreads();
    if (t == 0) {
        int run = begin;
        for (int b = 0; b < kCostBuckets; ++b) {
            const int c = off[b];
            off[b] = run;
            run += c;
        }
    }
    __syncthreads();
    for (int i0 = t; i0 < size; i0 += kOrderBatch * (int)blockDim.x) {
        int slot[kOrderBatch];
#pragma unroll
        for (int u = 0; u < kOrderBatch; ++u) {
            const int i = i0 + u * (int)blockDim.x;
            slot[u] = i < size ? atomicAdd(&off[bucket[i]], 1) : -1;
        }
#pragma unroll
        for (int u = 0; u < kOrderBatch; ++u)
            if (slot[u] >= 0) a.perm[slot[u]] = begin + i0 + u * (int)blockDim.x;
    }
}

__global__ void __launch_bounds__(1024) k_group_order(GroupOrderArgs a) { group_order_block(a, blockIdx.x); }

// A split step's dynamics and the next render's cost order in one launch (the two do not depend on each
// other): the first order_blocks workgroups sort, the rest step 256 agents each.
__global__ void __launch_bounds__(256) k_step_order(StepArgs s, GroupOrderArgs g, int order_blocks) {
    if ((int)blockIdx.x < order_blocks)
        group_order_block(g, blockIdx.x);
    else
        step_agent(s, ((int)blockIdx.x - order_blocks) * 256 + threadIdx.x);
}

static int group_order_blocks(int32_t total) {
    const int range = (total + 7) / 8;     // the largest XCD range
    return 8 * ((range + kGroupOrderChunk - 1) / kGroupOrderChunk);
}

hipError_t launch_group_order(const GroupOrderArgs& a, hipStream_t st) {
    if (a.total <= 0 || a.total > kGroupOrderMax) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_group_order, dim3(group_order_blocks(a.total)), dim3(1024), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_step_order(const StepArgs& s, const GroupOrderArgs& g, hipStream_t st) {
    if (g.total <= 0 || g.total > kGroupOrderMax) return hipErrorInvalidValue;
    const int ob = group_order_blocks(g.total);
    const int sb = s.n > 0 ? (s.n + 255) / 256 : 0;
    hipLaunchKernelGGL(k_step_order, dim3(ob + sb), dim3(256), 0, st, s, g, ob);
    return hipGetLastError();
}

int32_t render_groups_per_agent(int32_t max_h, int32_t max_w) {
    const int th = kTileH * kPacketRows, tw = kTileW * kPacketCols;
    int tiles = ((max_h + th - 1) / th) * ((max_w + tw - 1) / tw);
    return (tiles + kWavesPerBlock - 1) / kWavesPerBlock;
}

template <bool FUSED, bool STATS>
static void launch_render_noise(bool noise, dim3 grid, dim3 block, hipStream_t st, const RenderArgs& a) {
    const bool swarm = a.swarm.n > 0 && a.swarm.nodes;
    if (FUSED) {
        if (noise)
            hipLaunchKernelGGL((k_render_fused<STATS, true>), grid, block, 0, st, a);
        else
            hipLaunchKernelGGL((k_render_fused<STATS, false>), grid, block, 0, st, a);
    } else if (STATS || a.max_depth > kShallowDepth) {
        // the counting variants always take the two-register stack (they count the same walk)
        if (swarm) {
            if (noise)
                hipLaunchKernelGGL((k_render<STATS, true, true, true>), grid, block, 0, st, a);
            else
                hipLaunchKernelGGL((k_render<STATS, false, true, true>), grid, block, 0, st, a);
        } else {
            if (noise)
                hipLaunchKernelGGL((k_render<STATS, true, false, true>), grid, block, 0, st, a);
            else
                hipLaunchKernelGGL((k_render<STATS, false, false, true>), grid, block, 0, st, a);
        }
    } else {
        if (swarm) {
            if (noise)
                hipLaunchKernelGGL((k_render<false, true, true, false>), grid, block, 0, st, a);
            else
                hipLaunchKernelGGL((k_render<false, false, true, false>), grid, block, 0, st, a);
        } else {
            if (noise)
                hipLaunchKernelGGL((k_render<false, true, false, false>), grid, block, 0, st, a);
            else
                hipLaunchKernelGGL((k_render<false, false, false, false>), grid, block, 0, st, a);
        }
    }
}

hipError_t launch_render(RenderArgs a, bool fused, bool stats, bool noise, hipStream_t st) {
    if (a.n <= 0) return hipSuccess;
    a.groups_per_agent = render_groups_per_agent(a.max_h, a.max_w);
    int64_t total = (int64_t)a.n * a.groups_per_agent;
    if (total > 0x7fffffff) return hipErrorInvalidValue;
    a.total_groups = (int32_t)total;
    dim3 grid((unsigned)total), block(64 * kWavesPerBlock);
    if (fused) {
        if (stats)
            launch_render_noise<true, true>(noise, grid, block, st, a);
        else
            launch_render_noise<true, false>(noise, grid, block, st, a);
    } else {
        if (stats)
            launch_render_noise<false, true>(noise, grid, block, st, a);
        else
            launch_render_noise<false, false>(noise, grid, block, st, a);
    }
    return hipGetLastError();
}

}  // namespace vf
