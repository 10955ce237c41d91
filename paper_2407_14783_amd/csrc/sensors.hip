// Sensor extensions (Table I sensor set; Sec. III-D, Table II noise models).
//
// Noise draws come from Philox4x32-10 (Salmon et al., SC 2011), a counter-based
// generator: the four output words for a pixel are a pure function of
// (seed, agent key, pixel index, stream), so the noise of an agent's image does
// not depend on which other agents share the launch.  One 32-bit word gives a
// uniform (x >> 8) * 2^-24 in [0, 1); two give a Box-Muller normal.
//   depth  normal: D + sigma n; speckle: D (1 + sigma n); salt & pepper: u < p/2 -> far, u < p -> near
//   colour normal / speckle per channel (stream 1 + c), rounded to nearest and clamped to [0, 255];
//          salt & pepper (stream 4) sets the whole pixel to 255 / 0
// Missed pixels (tri id -1) keep their depth.
// Segmentation: label of the hit triangle from the scene's per-triangle labels (or the triangle index
// if the scene has none), -1 on a miss, -2 - j on swarm member j.
// IMU: specific force (F_b + d) / m in the body frame and the body rates, at the given state, with
// optional Normal noise (stream 7, one draw pair per axis).
#include "dynamics.h"
#include "vf_internal.h"

namespace vf {

struct Philox4 {
    uint32_t x[4];
};

__device__ __forceinline__ Philox4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                                 uint32_t k1) {
    for (int r = 0; r < 10; ++r) {
        uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
        uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
        uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    Philox4 o;
    o.x[0] = c0;
    o.x[1] = c1;
    o.x[2] = c2;
    o.x[3] = c3;
    return o;
}

__device__ __forceinline__ Philox4 draws(uint64_t seed, uint32_t key, uint32_t pixel, uint32_t stream) {
    return philox4x32_10(pixel, key, stream, 0u, (uint32_t)seed, (uint32_t)(seed >> 32));
}

__device__ __forceinline__ float uniform01(uint32_t w) { return (float)(w >> 8) * 5.9604644775390625e-8f; }

__device__ __forceinline__ float normal01(uint32_t w1, uint32_t w2) {
    float u1 = uniform01(w1), u2 = uniform01(w2);
    return sqrtf(-2.0f * logf(1.0f - u1)) * cosf(6.28318530717958647692f * u2);
}

__global__ void __launch_bounds__(256) k_noise(NoiseArgs a) {
    const int agent = blockIdx.x / a.blocks_per_agent;
    const int blk = blockIdx.x - agent * a.blocks_per_agent;
    vf_view vw = a.views[agent];
    if (vw.H < 1 || vw.W < 1 || vw.H > a.max_h || vw.W > a.max_w || vw.out_offset < 0 ||
        vw.out_offset + (int64_t)vw.H * vw.W > a.out_pixels) {
        if (threadIdx.x == 0 && blk == 0) atomicOr(a.err, kErrPixels);
        return;
    }
    const int npx = vw.H * vw.W;
    const uint32_t key = (uint32_t)vw.flags;
    for (int pix = blk * blockDim.x + threadIdx.x; pix < npx; pix += a.blocks_per_agent * blockDim.x) {
        int64_t at = vw.out_offset + pix;
        if (a.depth && a.cfg.depth_model != VF_NOISE_NONE) {
            bool hit = a.tri_id ? a.tri_id[at] >= 0 : true;
            if (hit) {
                Philox4 w = draws(a.cfg.seed, key, (uint32_t)pix, 0u);
                float dv = a.depth[at];
                if (a.cfg.depth_model == VF_NOISE_NORMAL) {
                    dv = dv + a.cfg.depth_sigma * normal01(w.x[0], w.x[1]);
                } else if (a.cfg.depth_model == VF_NOISE_SPECKLE) {
                    dv = dv * (1.0f + a.cfg.depth_sigma * normal01(w.x[0], w.x[1]));
                } else if (a.cfg.depth_model == VF_NOISE_SALT_PEPPER) {
                    float u = uniform01(w.x[2]);
                    dv = u < a.cfg.depth_p * 0.5f ? vw.far_clip : (u < a.cfg.depth_p ? vw.near_clip : dv);
                }
                a.depth[at] = dv;
            }
        }
        if (a.rgb && a.cfg.rgb_model != VF_NOISE_NONE) {
            int64_t plane = (int64_t)npx;
            uint8_t* px = a.rgb + 3 * vw.out_offset + pix;
            if (a.cfg.rgb_model == VF_NOISE_SALT_PEPPER) {
                Philox4 w = draws(a.cfg.seed, key, (uint32_t)pix, 4u);
                float u = uniform01(w.x[2]);
                if (u < a.cfg.rgb_p) {
                    uint8_t v = u < a.cfg.rgb_p * 0.5f ? 255 : 0;
                    px[0] = v;
                    px[plane] = v;
                    px[2 * plane] = v;
                }
            } else {
                for (int c = 0; c < 3; ++c) {
                    Philox4 w = draws(a.cfg.seed, key, (uint32_t)pix, 1u + (uint32_t)c);
                    float n = normal01(w.x[0], w.x[1]);
                    float val = (float)px[c * plane];
                    val = a.cfg.rgb_model == VF_NOISE_NORMAL ? val + a.cfg.rgb_sigma * n
                                                             : val * (1.0f + a.cfg.rgb_sigma * n);
                    val = fminf(fmaxf(floorf(val + 0.5f), 0.0f), 255.0f);
                    px[c * plane] = (uint8_t)val;
                }
            }
        }
    }
}

__global__ void __launch_bounds__(256) k_segment(SegArgs a) {
    const int agent = blockIdx.x / a.blocks_per_agent;
    const int blk = blockIdx.x - agent * a.blocks_per_agent;
    vf_view vw = a.views[agent];
    bool ok = vw.H >= 1 && vw.W >= 1 && vw.H <= a.max_h && vw.W <= a.max_w && vw.out_offset >= 0 &&
              vw.out_offset + (int64_t)vw.H * vw.W <= a.out_pixels && vw.scene_id >= 0 && vw.scene_id < a.n_scenes;
    if (ok) ok = a.scenes[vw.scene_id].valid != 0;
    if (!ok) {
        if (threadIdx.x == 0 && blk == 0) atomicOr(a.err, kErrView);
        return;
    }
    const SceneDesc sc = a.scenes[vw.scene_id];
    const int32_t* labels = a.labels[vw.scene_id];
    const int npx = vw.H * vw.W;
    for (int pix = blk * blockDim.x + threadIdx.x; pix < npx; pix += a.blocks_per_agent * blockDim.x) {
        int64_t at = vw.out_offset + pix;
        int32_t id = a.tri_id[at];
        int32_t lab = -1;
        if (id >= 0 && id < sc.n_tris)
            lab = labels ? labels[id] : id;
        else if (id >= sc.n_tris && vw.swarm > 0)
            lab = -2 - (id - sc.n_tris);   // swarm member j
        else if (id >= sc.n_tris)
            atomicOr(a.err, kErrTriId);
        a.seg[at] = lab;
    }
}

__global__ void __launch_bounds__(128) k_imu(ImuArgs a) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    int64_t slot = a.env_idx ? (int64_t)a.env_idx[i] : (int64_t)i;
    if (slot < 0 || slot >= a.n_slots) {
        atomicOr(a.err, kErrSlot);
        return;
    }
    const float* s = a.state + slot * 17;
    Vec13 y, dy;
    for (int k = 0; k < 3; ++k) { y.p[k] = s[k]; y.v[k] = s[7 + k]; y.w[k] = s[10 + k]; }
    for (int k = 0; k < 4; ++k) y.q[k] = s[3 + k];
    float w[4] = {s[13], s[14], s[15], s[16]};
    derivative(a.dyn, y, w, dy);
    float r[9];
    quat_rot(y.q, r);
    float fw[3] = {dy.v[0], dy.v[1], dy.v[2] + a.dyn.g};   // non-gravitational acceleration (world)
    float out[6];
    for (int k = 0; k < 3; ++k) out[k] = r[k] * fw[0] + r[3 + k] * fw[1] + r[6 + k] * fw[2];
    for (int k = 0; k < 3; ++k) out[3 + k] = y.w[k];
    if (a.sigma_acc > 0.0f || a.sigma_gyro > 0.0f) {
        uint32_t key = a.keys ? (uint32_t)a.keys[i] : (uint32_t)i;
        for (int k = 0; k < 6; ++k) {
            Philox4 d = draws(a.seed, key, (uint32_t)k, 7u);
            out[k] += (k < 3 ? a.sigma_acc : a.sigma_gyro) * normal01(d.x[0], d.x[1]);
        }
    }
    for (int k = 0; k < 6; ++k) a.out[(int64_t)i * 6 + k] = out[k];
}

hipError_t launch_noise(NoiseArgs a, hipStream_t st) {
    if (a.n <= 0) return hipSuccess;
    int per = (a.max_h * a.max_w + 255) / 256;
    a.blocks_per_agent = per < 16 ? per : 16;
    int64_t total = (int64_t)a.n * a.blocks_per_agent;
    if (total > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_noise, dim3((unsigned)total), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_segment(SegArgs a, hipStream_t st) {
    if (a.n <= 0) return hipSuccess;
    int per = (a.max_h * a.max_w + 255) / 256;
    a.blocks_per_agent = per < 16 ? per : 16;
    int64_t total = (int64_t)a.n * a.blocks_per_agent;
    if (total > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_segment, dim3((unsigned)total), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_imu(const ImuArgs& a, hipStream_t st) {
    if (a.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_imu, dim3((a.n + 127) / 128), dim3(128), 0, st, a);
    return hipGetLastError();
}

}  // namespace vf
