// Table II sensor-noise models on the device (Sec. III-D), shared by the separate noise pass and the
// render kernel's epilogue so that both give the same bits.
//
// Draws come from Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC 2011): the four output words of a
// (seed, key, pixel, stream, attempt) counter are integer arithmetic, identical everywhere.
//   uniform   (w >> 8) 2^-24 in [0, 1) from one word (exact in float32);
//             ((w0 >> 5) 2^26 + (w1 >> 6)) 2^-53 from two words (exact in FP64)
//   normal    Box-Muller in float32: sqrt(-2 ln(1 - u1)) cos(2 pi u2)
//   Poisson   in FP64: for a rate below 10 inversion (the smallest k with u < F(k), the terms
//             p_k = p_{k-1} lam / k summed in order); from 10 up the transformed rejection with
//             squeeze of Hoermann (1993), attempt i drawing its two uniforms from counter word 3 = i
// Models (misses keep their depth; colour noise acts on every pixel; segmentation noise on labelled
// pixels, label >= 0):
//   depth   NORMAL D + s n; SPECKLE D (1 + s n); SALT_PEPPER u < p/2 -> far, u < p -> near;
//           POISSON P(D c) / c with c counts per metre
//   colour  NORMAL v + s n, SPECKLE v (1 + s n), POISSON P(v c) / c per channel (streams 1 + ch),
//           rounded half up and clamped to [0, 255]; SALT_PEPPER (stream 4) whole pixel 255 / 0
//   labels  NORMAL l + floor(s n + 1/2); SPECKLE floor(l (1 + s n) + 1/2) (both in FP64 from the
//           float32 normal); POISSON floor(P(l c) / c + 1/2); SALT_PEPPER p/2 -> the salt label,
//           p/2 -> -1 (stream 5); results clamped to the int32 range
// Every expression is evaluated as written (no contraction of a multiply and an add), so the two
// callers compile it to the same operations.
#pragma once

#include "vf_internal.h"

namespace vf {

struct Philox4 {
    uint32_t x[4];
};

__device__ __forceinline__ Philox4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                                 uint32_t k1) {
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
        const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
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

enum : uint32_t { kStreamDepth = 0, kStreamRgb0 = 1, kStreamRgbSp = 4, kStreamSeg = 5, kStreamImu = 7 };

__device__ __forceinline__ Philox4 noise_draws(uint64_t seed, uint32_t key, uint32_t pixel, uint32_t stream,
                                               uint32_t attempt = 0u) {
    return philox4x32_10(pixel, key, stream, attempt, (uint32_t)seed, (uint32_t)(seed >> 32));
}

__device__ __forceinline__ float uniform01(uint32_t w) { return (float)(w >> 8) * 5.9604644775390625e-8f; }

__device__ __forceinline__ double uniform53(uint32_t hi, uint32_t lo) {
    return ((double)(hi >> 5) * 67108864.0 + (double)(lo >> 6)) * 1.1102230246251565404e-16;
}

__device__ __forceinline__ float normal01(uint32_t w1, uint32_t w2) {
#pragma clang fp contract(off)
    const float u1 = uniform01(w1), u2 = uniform01(w2);
    return sqrtf(-2.0f * logf(1.0f - u1)) * cosf(6.28318530717958647692f * u2);
}

constexpr double kPoissonSmall = 10.0;   // below: inversion; at and above: transformed rejection
constexpr int kPoissonMaxInv = 200;      // inversion stops here (F(200) = 1 in FP64 for rates below 10)
constexpr int kPoissonMaxAttempts = 64;  // rejection attempts (each accepts with probability > 0.8)

// One Poisson(lam) draw (an integer value held in a double).
__device__ __noinline__ double poisson_draw(double lam, uint64_t seed, uint32_t key, uint32_t pixel,
                                           uint32_t stream) {
#pragma clang fp contract(off)
    if (!(lam > 0.0)) return 0.0;
    if (lam < kPoissonSmall) {
        const Philox4 w = noise_draws(seed, key, pixel, stream, 0u);
        const double u = uniform53(w.x[0], w.x[1]);
        double p = exp(-lam);
        double f = p;
        int k = 0;
        while (u >= f && k < kPoissonMaxInv) {
            ++k;
            p = p * (lam / (double)k);
            f = f + p;
        }
        return (double)k;
    }
    const double slam = sqrt(lam), loglam = log(lam);
    const double b = 0.931 + 2.53 * slam;
    const double a = -0.059 + 0.02483 * b;
    const double inv_alpha = 1.1239 + 1.1328 / (b - 3.4);
    const double v_r = 0.9277 - 3.6224 / (b - 2.0);
    for (uint32_t attempt = 0; attempt < (uint32_t)kPoissonMaxAttempts; ++attempt) {
        const Philox4 w = noise_draws(seed, key, pixel, stream, attempt);
        const double u = uniform53(w.x[0], w.x[1]) - 0.5;
        const double v = uniform53(w.x[2], w.x[3]);
        const double us = 0.5 - fabs(u);
        const double x = (2.0 * a / us + b) * u + lam + 0.43;
        const double k = floor(x);
        if (us >= 0.07 && v <= v_r) return k;
        if (k < 0.0 || (us < 0.013 && v > us)) continue;
        const double lhs = log(v) + log(inv_alpha) - log(a / (us * us) + b);
        const double rhs = -lam + k * loglam - lgamma(k + 1.0);
        if (lhs <= rhs) return k;
    }
    return floor(lam);
}

__device__ __forceinline__ float noisy_depth_px(const vf_noise& cfg, uint32_t key, uint32_t pix, float dv,
                                                float near_clip, float far_clip) {
#pragma clang fp contract(off)
    switch (cfg.depth_model) {
        case VF_NOISE_NORMAL: {
            const Philox4 w = noise_draws(cfg.seed, key, pix, kStreamDepth);
            return dv + cfg.depth_sigma * normal01(w.x[0], w.x[1]);
        }
        case VF_NOISE_SPECKLE: {
            const Philox4 w = noise_draws(cfg.seed, key, pix, kStreamDepth);
            return dv * (1.0f + cfg.depth_sigma * normal01(w.x[0], w.x[1]));
        }
        case VF_NOISE_SALT_PEPPER: {
            const Philox4 w = noise_draws(cfg.seed, key, pix, kStreamDepth);
            const float u = uniform01(w.x[2]);
            return u < cfg.depth_p * 0.5f ? far_clip : (u < cfg.depth_p ? near_clip : dv);
        }
        case VF_NOISE_POISSON: {
            const double c = (double)cfg.depth_scale;
            const double k = poisson_draw((double)dv * c, cfg.seed, key, pix, kStreamDepth);
            return (float)(k / c);
        }
        default:
            return dv;
    }
}

// Colour noise of one pixel's three channels (in place).
__device__ __forceinline__ void noisy_rgb_px(const vf_noise& cfg, uint32_t key, uint32_t pix, uint8_t ch[3]) {
#pragma clang fp contract(off)
    if (cfg.rgb_model == VF_NOISE_SALT_PEPPER) {
        const Philox4 w = noise_draws(cfg.seed, key, pix, kStreamRgbSp);
        const float u = uniform01(w.x[2]);
        if (u < cfg.rgb_p) {
            const uint8_t v = u < cfg.rgb_p * 0.5f ? 255 : 0;
            ch[0] = v;
            ch[1] = v;
            ch[2] = v;
        }
        return;
    }
    if (cfg.rgb_model == VF_NOISE_POISSON) {
        const double c = (double)cfg.rgb_scale;
        for (int k = 0; k < 3; ++k) {
            const double n = poisson_draw((double)ch[k] * c, cfg.seed, key, pix, kStreamRgb0 + (uint32_t)k);
            const double x = floor(n / c + 0.5);
            ch[k] = (uint8_t)(x < 0.0 ? 0.0 : (x > 255.0 ? 255.0 : x));
        }
        return;
    }
    if (cfg.rgb_model != VF_NOISE_NORMAL && cfg.rgb_model != VF_NOISE_SPECKLE) return;
    for (int k = 0; k < 3; ++k) {
        const Philox4 w = noise_draws(cfg.seed, key, pix, kStreamRgb0 + (uint32_t)k);
        const float n = normal01(w.x[0], w.x[1]);
        const float v = (float)ch[k];
        float val = cfg.rgb_model == VF_NOISE_NORMAL ? v + cfg.rgb_sigma * n : v * (1.0f + cfg.rgb_sigma * n);
        val = fminf(fmaxf(floorf(val + 0.5f), 0.0f), 255.0f);
        ch[k] = (uint8_t)val;
    }
}

// Label noise of one labelled pixel (label >= 0); other pixels keep their value.
__device__ __forceinline__ int32_t noisy_label_px(const vf_noise& cfg, uint32_t key, uint32_t pix, int32_t lab) {
#pragma clang fp contract(off)
    if (lab < 0 || cfg.seg_model == VF_NOISE_NONE) return lab;
    const Philox4 w = noise_draws(cfg.seed, key, pix, kStreamSeg);
    const double lim = 2147483647.0;
    switch (cfg.seg_model) {
        case VF_NOISE_NORMAL: {
            const double n = (double)normal01(w.x[0], w.x[1]);
            const double x = (double)lab + floor((double)cfg.seg_sigma * n + 0.5);
            return (int32_t)(x > lim ? lim : x);
        }
        case VF_NOISE_SPECKLE: {
            const double n = (double)normal01(w.x[0], w.x[1]);
            const double x = floor((double)lab * (1.0 + (double)cfg.seg_sigma * n) + 0.5);
            return (int32_t)(x > lim ? lim : (x < -lim - 1.0 ? -lim - 1.0 : x));
        }
        case VF_NOISE_POISSON: {
            const double c = (double)cfg.seg_scale;
            const double k = poisson_draw((double)lab * c, cfg.seed, key, pix, kStreamSeg);
            const double x = floor(k / c + 0.5);
            return (int32_t)(x > lim ? lim : x);
        }
        case VF_NOISE_SALT_PEPPER: {
            const float u = uniform01(w.x[2]);
            return u < cfg.seg_p * 0.5f ? cfg.seg_salt_label : (u < cfg.seg_p ? -1 : lab);
        }
        default:
            return lab;
    }
}

}  // namespace vf
