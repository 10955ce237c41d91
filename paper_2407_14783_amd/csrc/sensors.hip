// Sensor extensions (Table I sensor set; Sec. III-D, Table II noise models).
//
// k_noise applies the Table II models of noise.h to rendered images in place: depth (misses keep their
// depth), planar colour and segmentation labels, one pixel per lane.  The draws are keyed by
// (seed, agent key, pixel, stream), so the noise of an agent's image does not depend on which other
// agents share the launch, and the render kernel's epilogue form gives the same bits.
// Segmentation: label of the hit triangle from the scene's per-triangle labels (or the triangle index
// if the scene has none), -1 on a miss, -2 - j on swarm member j.
// IMU: specific force (F_b + d) / m in the body frame and the body rates, at the given state, with
// optional Normal noise (stream 7, one draw pair per axis).
#include "dynamics.h"
#include "noise.h"
#include "vf_internal.h"

namespace vf {

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
        const int64_t at = vw.out_offset + pix;
        if (a.depth && a.cfg.depth_model != VF_NOISE_NONE) {
            const bool hit = a.tri_id ? a.tri_id[at] >= 0 : true;
            if (hit) a.depth[at] = noisy_depth_px(a.cfg, key, (uint32_t)pix, a.depth[at], vw.near_clip, vw.far_clip);
        }
        if (a.rgb && a.cfg.rgb_model != VF_NOISE_NONE) {
            const int64_t plane = (int64_t)npx;
            uint8_t* px = a.rgb + 3 * vw.out_offset + pix;
            uint8_t ch[3] = {px[0], px[plane], px[2 * plane]};
            noisy_rgb_px(a.cfg, key, (uint32_t)pix, ch);
            px[0] = ch[0];
            px[plane] = ch[1];
            px[2 * plane] = ch[2];
        }
        if (a.seg && a.cfg.seg_model != VF_NOISE_NONE) a.seg[at] = noisy_label_px(a.cfg, key, (uint32_t)pix, a.seg[at]);
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
            Philox4 d = noise_draws(a.seed, key, (uint32_t)k, kStreamImu);
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
