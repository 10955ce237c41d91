// Nearest-obstacle query on the device BVH (Sec. III-B: the spatial distance
// module that reports the nearest obstacle point without a collision having to
// happen).  One lane per query point; query points are unrelated to each other,
// so each lane walks the 4-wide BVH on its own: children are visited nearest
// box first and a subtree is skipped when its box is farther than the best
// distance found so far.  The closest point on a triangle is found by the
// Voronoi-region method (Ericson, Real-Time Collision Detection, 5.1.5):
// vertex, edge or face region from the signs of a few dot products (a point in the face region is
// projected onto the plane directly).
// Equal distances go to the lower caller triangle index.  In agent mode the query
// points are the agents' positions (state rows) and the flag dist <= radius is
// the collision test that ends an episode.
#include <float.h>

#include "vf_internal.h"

namespace vf {

constexpr int kQueryStack = 128;

__device__ __forceinline__ float box_dist2(float px, float py, float pz, float lx, float hx, float ly, float hy,
                                           float lz, float hz) {
    float dx = fmaxf(fmaxf(lx - px, px - hx), 0.0f);
    float dy = fmaxf(fmaxf(ly - py, py - hy), 0.0f);
    float dz = fmaxf(fmaxf(lz - pz, pz - hz), 0.0f);
    return dx * dx + dy * dy + dz * dz;
}

// Closest point to p on triangle (a, b = a + e1, c = a + e2).
__device__ __forceinline__ void closest_on_triangle(const float p[3], const float a[3], const float e1[3],
                                                    const float e2[3], float out[3]) {
    float ap[3] = {p[0] - a[0], p[1] - a[1], p[2] - a[2]};
    float d1 = e1[0] * ap[0] + e1[1] * ap[1] + e1[2] * ap[2];
    float d2 = e2[0] * ap[0] + e2[1] * ap[1] + e2[2] * ap[2];
    if (d1 <= 0.0f && d2 <= 0.0f) {   // vertex a
        for (int i = 0; i < 3; ++i) out[i] = a[i];
        return;
    }
    float bp[3] = {ap[0] - e1[0], ap[1] - e1[1], ap[2] - e1[2]};
    float d3 = e1[0] * bp[0] + e1[1] * bp[1] + e1[2] * bp[2];
    float d4 = e2[0] * bp[0] + e2[1] * bp[1] + e2[2] * bp[2];
    if (d3 >= 0.0f && d4 <= d3) {     // vertex b
        for (int i = 0; i < 3; ++i) out[i] = a[i] + e1[i];
        return;
    }
    float vc = d1 * d4 - d3 * d2;
    if (vc <= 0.0f && d1 >= 0.0f && d3 <= 0.0f) {   // edge ab
        float v = d1 / (d1 - d3);
        for (int i = 0; i < 3; ++i) out[i] = a[i] + v * e1[i];
        return;
    }
    float cp[3] = {ap[0] - e2[0], ap[1] - e2[1], ap[2] - e2[2]};
    float d5 = e1[0] * cp[0] + e1[1] * cp[1] + e1[2] * cp[2];
    float d6 = e2[0] * cp[0] + e2[1] * cp[1] + e2[2] * cp[2];
    if (d6 >= 0.0f && d5 <= d6) {     // vertex c
        for (int i = 0; i < 3; ++i) out[i] = a[i] + e2[i];
        return;
    }
    float vb = d5 * d2 - d1 * d6;
    if (vb <= 0.0f && d2 >= 0.0f && d6 <= 0.0f) {   // edge ac
        float w = d2 / (d2 - d6);
        for (int i = 0; i < 3; ++i) out[i] = a[i] + w * e2[i];
        return;
    }
    float va = d3 * d6 - d5 * d4;
    if (va <= 0.0f && (d4 - d3) >= 0.0f && (d5 - d6) >= 0.0f) {   // edge bc
        float w = (d4 - d3) / ((d4 - d3) + (d5 - d6));
        for (int i = 0; i < 3; ++i) out[i] = a[i] + e1[i] + w * (e2[i] - e1[i]);
        return;
    }
    // face interior: orthogonal projection onto the plane (no cancellation in barycentric weights)
    float n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
    float s = (ap[0] * n[0] + ap[1] * n[1] + ap[2] * n[2]) / (n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    for (int i = 0; i < 3; ++i) out[i] = p[i] - s * n[i];
}

__global__ void __launch_bounds__(128) k_closest_point(QueryArgs q) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= q.n) return;
    int32_t sid;
    float p[3];
    bool ok = true;
    if (q.state) {
        int64_t slot = q.env_idx ? (int64_t)q.env_idx[i] : (int64_t)i;
        if (slot < 0 || slot >= q.n_slots) {
            atomicOr(q.err, kErrSlot);
            ok = false;
            slot = 0;
        }
        for (int k = 0; k < 3; ++k) p[k] = q.state[slot * 17 + k];
        sid = q.views[i].scene_id;
    } else {
        sid = q.scene_ids ? q.scene_ids[i] : q.scene_id0;
        for (int k = 0; k < 3; ++k) p[k] = q.points[3 * (int64_t)i + k];
    }
    if (ok && (sid < 0 || sid >= q.n_scenes || !q.scenes[sid].valid)) {
        atomicOr(q.err, kErrScene);
        ok = false;
    }
    if (!ok) {
        q.dist[i] = INFINITY;
        if (q.tri_id) q.tri_id[i] = -1;
        if (q.collided) q.collided[i] = 0;
        if (q.rel)
            for (int k = 0; k < 3; ++k) q.rel[3 * (int64_t)i + k] = 0.0f;
        return;
    }
    const SceneDesc sc = q.scenes[sid];
    float best = q.max_dist * q.max_dist;
    int32_t best_id = -1;
    float best_pt[3] = {0.f, 0.f, 0.f};
    int32_t stack[kQueryStack];
    float sdist[kQueryStack];
    int sp = 0;
    stack[sp] = 0;
    sdist[sp] = 0.0f;
    ++sp;
    bool overflow = false;
    while (sp > 0) {
        --sp;
        int32_t e = stack[sp];
        if (sdist[sp] > best) continue;
        if (e >= 0) {
            const Node& nd = sc.nodes[e];
            float dk[kWidth];
            int32_t ek[kWidth];
            int nk = 0;
            for (int k = 0; k < kWidth; ++k) {
                const int32_t c = nd.child[k];   // node index, or the leaf's encoded range
                if (c == kEmptyChild) continue;
                float d2 = box_dist2(p[0], p[1], p[2], nd.lo_x[k], nd.hi_x[k], nd.lo_y[k], nd.hi_y[k], nd.lo_z[k],
                                     nd.hi_z[k]);
                if (d2 > best) continue;
                // insertion into the small list, farthest first
                int j = nk++;
                while (j > 0 && dk[j - 1] < d2) {
                    dk[j] = dk[j - 1];
                    ek[j] = ek[j - 1];
                    --j;
                }
                dk[j] = d2;
                ek[j] = c;
            }
            for (int j = 0; j < nk; ++j) {
                if (sp < kQueryStack) {
                    stack[sp] = ek[j];
                    sdist[sp] = dk[j];
                    ++sp;
                } else {
                    overflow = true;
                }
            }
        } else {
            int32_t code = -e - 1;
            int32_t first = code >> 3, cnt = (code & 7) + 1;
            for (int j = 0; j < cnt; ++j) {
                const Tri tr = sc.tris[first + j];
                const float a[3] = {tr.v0x, tr.v0y, tr.v0z};
                const float e1[3] = {tr.e1x, tr.e1y, tr.e1z};
                const float e2[3] = {tr.e2x, tr.e2y, tr.e2z};
                float c[3];
                closest_on_triangle(p, a, e1, e2, c);
                float dx = p[0] - c[0], dy = p[1] - c[1], dz = p[2] - c[2];
                float d2 = dx * dx + dy * dy + dz * dz;
                if (d2 < best || (d2 == best && best_id >= 0 && tr.id < best_id) || (d2 == best && best_id < 0)) {
                    best = d2;
                    best_id = tr.id;
                    best_pt[0] = c[0];
                    best_pt[1] = c[1];
                    best_pt[2] = c[2];
                }
            }
        }
    }
    if (overflow) atomicOr(q.err, kErrStack);
    float d = best_id >= 0 ? sqrtf(best) : INFINITY;
    if (q.state && q.views[i].swarm > 0) {
        // other members of the agent's swarm, as bounding spheres
        const int sw = q.views[i].swarm;
        if (sw > q.swarm.n) {
            atomicOr(q.err, kErrView);
        } else {
            const int64_t self = q.env_idx ? (int64_t)q.env_idx[i] : (int64_t)i;
            for (int j = q.swarm.off[sw - 1]; j < q.swarm.off[sw]; ++j) {
                const int64_t ms = q.swarm.slots[j];
                if (ms == self) continue;
                if (ms < 0 || ms >= q.n_slots) {
                    atomicOr(q.err, kErrSlot);
                    continue;
                }
                const float* mp = q.state + ms * 17;
                const float vx = mp[0] - p[0], vy = mp[1] - p[1], vz = mp[2] - p[2];
                const float c = sqrtf(vx * vx + vy * vy + vz * vz);
                const float dm = c - q.swarm.radius;
                if (dm < d) {
                    d = dm;
                    best_id = -2;
                    const float s = c > 0.0f ? dm / c : 0.0f;
                    best_pt[0] = p[0] + s * vx;
                    best_pt[1] = p[1] + s * vy;
                    best_pt[2] = p[2] + s * vz;
                }
            }
        }
    }
    q.dist[i] = d;
    if (q.collided) q.collided[i] = d <= q.radius ? 1 : 0;
    if (q.rel)
        for (int k = 0; k < 3; ++k) q.rel[3 * (int64_t)i + k] = best_id != -1 ? best_pt[k] - p[k] : 0.0f;
    if (q.tri_id) q.tri_id[i] = best_id;
    if (q.closest) {
        q.closest[3 * (int64_t)i] = best_pt[0];
        q.closest[3 * (int64_t)i + 1] = best_pt[1];
        q.closest[3 * (int64_t)i + 2] = best_pt[2];
    }
}

hipError_t launch_closest_point(const QueryArgs& q, hipStream_t st) {
    if (q.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_closest_point, dim3((q.n + 127) / 128), dim3(128), 0, st, q);
    return hipGetLastError();
}

}  // namespace vf
