// Swarm members as seen by the render (the swarm example of Sec. IV: agents see each other).
//
// Each swarm's members are boxes turned with their attitude.  A top-level tree over them is rebuilt from
// the states before every render that shows swarms (k_swarm_tree, swarm.hip): members sorted by the
// Morton code of their centres, grouped four to a leaf, and an implicit 4-wide tree of world-axis boxes
// over the groups, with the near-to-far child order of every ray-direction octant like the mesh BVH.
// A packet walks it after the mesh, pruned by the depth it has already found, and tests the members of
// the leaves it reaches in their own frame (slab test).  A member is hit where a ray enters its box at
// t in [near, far]; a camera inside a box does not see that box; the agent's own box is skipped.  At
// equal depth the mesh keeps its hit and a lower member index wins, whatever order the tree gives.
#pragma once

#include "vf_internal.h"

namespace vf {

#define SWARM_CONST_AS __attribute__((address_space(4)))

// quantised centre -> 30-bit Morton code (bit b of x, y, z at 3b, 3b + 1, 3b + 2)
__device__ __forceinline__ uint32_t morton3_10(uint32_t x, uint32_t y, uint32_t z) {
    uint32_t code = 0;
    for (int b = 0; b < 10; ++b)
        code |= (((x >> b) & 1u) << (3 * b)) | (((y >> b) & 1u) << (3 * b + 1)) | (((z >> b) & 1u) << (3 * b + 2));
    return code;
}

// Oriented member boxes of one swarm against a packet: the tree walk and the member tests.
// STATS adds the member tests a lane performs to ts_member (per lane) and the tree's box tests to
// box_lane (issued per lane, as the mesh's).
template <int NR, bool STATS>
__device__ __forceinline__ void trace_swarm(const SwarmTable& sw, int s, int64_t self, int32_t n_tris,
                                            const bool (&valid)[NR], const float o[3], const float (&d)[NR][3],
                                            float t_near, float (&t_best)[NR], int32_t (&id_best)[NR],
                                            unsigned long long& box_lane, unsigned long long& member_lane) {
    const int32_t first = sw.off[s];
    const int32_t m = sw.off[s + 1] - first;
    if (m <= 0) return;
    const Node4 SWARM_CONST_AS* nodes = (const Node4 SWARM_CONST_AS*)(sw.nodes + sw.node_off[s]);
    const SwarmMember SWARM_CONST_AS* mem = (const SwarmMember SWARM_CONST_AS*)(sw.members + first);
    float inv[NR][3], oi[NR][3];
    int n_valid = 0;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        for (int k = 0; k < 3; ++k) {
            const float dk = d[r][k];
            inv[r][k] = 1.0f / (fabsf(dk) < 1e-20f ? copysignf(1e-20f, dk) : dk);
            oi[r][k] = -o[k] * inv[r][k];
        }
        n_valid += valid[r] ? 1 : 0;
    }
    const float grow2 = 1.000001f, unshrink = 1.0000005f;
    int oct = (d[0][0] < 0.f ? 1 : 0) | (d[0][1] < 0.f ? 2 : 0) | (d[0][2] < 0.f ? 4 : 0);
    oct = __builtin_amdgcn_readfirstlane(oct);
    // a tree of at most 4,096 members is at most 6 levels deep: the pending entries fit one VGPR's lanes
    int stk = 0, sp = 0;
    int32_t entry = 0;
    while (true) {
        if (entry >= 0) {
            const uint32_t SWARM_CONST_AS* np = (const uint32_t SWARM_CONST_AS*)(nodes + entry);
            uint32_t w[32];
#pragma unroll
            for (int i = 0; i < 32; ++i) w[i] = np[i];
            asm volatile("" ::"s"(w[28]), "s"(w[31]));
            if (STATS) box_lane += 4 * n_valid;
            uint32_t hb = 0;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const float lox = __uint_as_float(w[k]), hix = __uint_as_float(w[4 + k]);
                const float loy = __uint_as_float(w[8 + k]), hiy = __uint_as_float(w[12 + k]);
                const float loz = __uint_as_float(w[16 + k]), hiz = __uint_as_float(w[20 + k]);
                uint64_t mk = 0;
#pragma unroll
                for (int r = 0; r < NR; ++r) {
                    const float tx0 = fmaf(lox, inv[r][0], oi[r][0]), tx1 = fmaf(hix, inv[r][0], oi[r][0]);
                    const float ty0 = fmaf(loy, inv[r][1], oi[r][1]), ty1 = fmaf(hiy, inv[r][1], oi[r][1]);
                    const float tz0 = fmaf(loz, inv[r][2], oi[r][2]), tz1 = fmaf(hiz, inv[r][2], oi[r][2]);
                    const float t0 = fmaxf(fmaxf(fminf(tx0, tx1), fminf(ty0, ty1)), fmaxf(fminf(tz0, tz1), t_near));
                    const float t1 = fminf(fminf(fmaxf(tx0, tx1), fmaxf(ty0, ty1)), fmaxf(tz0, tz1)) * grow2;
                    const float tb = valid[r] ? t_best[r] * unshrink : -1.0f;
                    mk |= __ballot(t0 <= fminf(t1, tb));
                }
                hb |= (mk != 0ull ? 1u : 0u) << k;
            }
            const uint64_t ord = ((uint64_t)w[30] << 32) | w[29];
            const uint32_t slots = (uint32_t)(ord >> (8 * oct)) & 255u;
#pragma unroll
            for (int i = 3; i >= 0; --i) {
                const uint32_t k = (slots >> (2 * i)) & 3u;
                if ((hb >> k) & 1u) {
                    const int32_t e01 = (int32_t)((k & 1u) ? w[25] : w[24]);
                    const int32_t e23 = (int32_t)((k & 1u) ? w[27] : w[26]);
                    const int32_t e = (k & 2u) ? e23 : e01;
                    stk = (int)(threadIdx.x & 63) == sp ? e : stk;
                    ++sp;
                }
            }
        } else {
            // a leaf: members [first, first + count) of the tree order
            const int32_t code = -entry - 1;
            const int32_t f = code >> 3, cnt = (code & 7) + 1;
            for (int j = 0; j < cnt; ++j) {
                const uint32_t SWARM_CONST_AS* mp = (const uint32_t SWARM_CONST_AS*)(mem + f + j);
                uint32_t u[16];
#pragma unroll
                for (int i = 0; i < 16; ++i) u[i] = mp[i];
                asm volatile("" ::"s"(u[14]), "s"(u[15]));
                if ((int64_t)(int32_t)u[13] == self) continue;
                float r[9];
#pragma unroll
                for (int i = 0; i < 9; ++i) r[i] = __uint_as_float(u[i]);
                const int32_t id = n_tris + (int32_t)u[12];
                // o' = R^T (o - c)
                const float dx = o[0] - __uint_as_float(u[9]), dy = o[1] - __uint_as_float(u[10]),
                            dz = o[2] - __uint_as_float(u[11]);
                float ob[3];
                for (int k = 0; k < 3; ++k) ob[k] = r[k] * dx + r[3 + k] * dy + r[6 + k] * dz;
                if (STATS) member_lane += n_valid;
#pragma unroll
                for (int q = 0; q < NR; ++q) {
                    float t_in = -INFINITY, t_out = INFINITY;
                    for (int ax = 0; ax < 3; ++ax) {
                        const float db = r[ax] * d[q][0] + r[3 + ax] * d[q][1] + r[6 + ax] * d[q][2];
                        const float iv = 1.0f / (fabsf(db) < 1e-20f ? copysignf(1e-20f, db) : db);
                        const float t1 = (-sw.half[ax] - ob[ax]) * iv, t2 = (sw.half[ax] - ob[ax]) * iv;
                        t_in = fmaxf(t_in, fminf(t1, t2));
                        t_out = fminf(t_out, fmaxf(t1, t2));
                    }
                    // nearer, or as near as an earlier member (the mesh keeps equal depths)
                    const bool tie_wins = id_best[q] < 0 || (id_best[q] >= n_tris && id < id_best[q]);
                    const bool take = valid[q] && t_in <= t_out && t_in >= t_near &&
                                      (t_in < t_best[q] || (t_in == t_best[q] && tie_wins));
                    t_best[q] = take ? t_in : t_best[q];
                    id_best[q] = take ? id : id_best[q];
                }
            }
        }
        if (sp == 0) break;
        --sp;
        entry = __builtin_amdgcn_readlane(stk, sp & 63);
    }
}

}  // namespace vf
