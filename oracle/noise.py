"""Sensor noise and derived sensors (Sec. III-D, Table II; Table I sensor set), FP64 reference.

Random numbers come from the counter-based generator Philox4x32-10 (Salmon,
Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC 2011):
ten rounds of two 32x32->64-bit multiplies with the round keys bumped by the
Weyl constants.  A draw is keyed by (seed, agent key, pixel, stream, attempt) so
it does not depend on batch composition.

Readings (Table II names the models only; every model below is applied to the
image as a plain array of values, as an image-noise library would):
  uniform   u = (x >> 8) * 2^-24 in [0, 1) from one 32-bit output word;
            u53 = ((x0 >> 5) 2^26 + (x1 >> 6)) 2^-53 from two words
  normal    Box-Muller: sqrt(-2 ln(1 - u1)) * cos(2 pi u2)
  Poisson   P(lam): for lam < 10 inversion, the smallest k with u53 < F(k) summed
            term by term (p_0 = e^-lam, p_k = p_{k-1} (lam / k)); for lam >= 10 the
            transformed rejection with squeeze of Hoermann (1993, "The transformed
            rejection method for generating Poisson random variables"), attempt i
            taking its two uniforms from counter word 3 = i
  depth     Normal:  D + sigma n          Speckle: D (1 + sigma n)
            Poisson: P(D s) / s (s counts per metre)
            Salt & pepper: with probability p/2 -> far (salt), p/2 -> near (pepper)
            misses keep their depth
  colour    Normal / speckle / Poisson (P(v s) / s) per channel on the 0..255 value,
            rounded to nearest (floor(x + 1/2)) and clamped; salt & pepper -> 255 / 0
            for the whole pixel
  segmentation  label = per-triangle label of the hit triangle (-1 on a miss); noise acts
            on pixels with a label >= 0: Normal l + floor(sigma n + 1/2), Speckle
            floor(l (1 + sigma n) + 1/2), Poisson floor(P(l s) / s + 1/2), salt & pepper
            p/2 -> the given salt label, p/2 -> -1 (nothing)
  IMU       accelerometer: specific force (F_b + d) / m in the body frame at the state;
            gyro: body rates; optional Normal noise per axis
Streams: depth 0, colour channel c 1 + c, colour salt & pepper 4, segmentation 5, IMU 7.
Salt & pepper compares u with p / 2 and p where p is the float32 the device receives
(rounded once) and halved exactly: u, p / 2 and p are all exact in float32 and in FP64,
so the decision is the definition's, with no rounding of its own.
Every other value is computed in FP64.  The functions return, beside the values, the
margin of each pixel's discrete decisions (how far a compared quantity was from its
threshold, or a value from a rounding boundary), so that a comparison can set aside
the pixels where one unit in the last place of a transcendental could tip a decision.
The RedWood depth model is not built (its parameters are not in the paper).
"""
import math

import numpy as np

from . import dynamics

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """ctr: uint [..., 4], key: uint [..., 2] -> uint64 arrays [..., 4] holding 32-bit words."""
    c = [np.asarray(ctr[..., i], dtype=np.uint64) & MASK for i in range(4)]
    k0 = np.asarray(key[..., 0], dtype=np.uint64) & MASK
    k1 = np.asarray(key[..., 1], dtype=np.uint64) & MASK
    for _ in range(10):
        p0 = c[0] * np.uint64(M0)
        p1 = c[2] * np.uint64(M1)
        hi0, lo0 = p0 >> np.uint64(32), p0 & np.uint64(MASK)
        hi1, lo1 = p1 >> np.uint64(32), p1 & np.uint64(MASK)
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
        k0 = (k0 + np.uint64(W0)) & np.uint64(MASK)
        k1 = (k1 + np.uint64(W1)) & np.uint64(MASK)
    return np.stack(c, axis=-1)


def draws(seed, agent_key, pixel, stream, attempt=0):
    """Four 32-bit words for each (agent key, pixel) at the given stream index and attempt."""
    agent_key = np.asarray(agent_key, dtype=np.uint64)
    pixel = np.asarray(pixel, dtype=np.uint64)
    shape = np.broadcast(agent_key, pixel).shape
    ctr = np.zeros(shape + (4,), dtype=np.uint64)
    ctr[..., 0] = pixel
    ctr[..., 1] = agent_key
    ctr[..., 2] = stream
    ctr[..., 3] = attempt
    key = np.zeros(shape + (2,), dtype=np.uint64)
    key[..., 0] = seed & MASK
    key[..., 1] = (seed >> 32) & MASK
    return philox4x32_10(ctr, key)


def uniform(word):
    """[0, 1) from a 32-bit word: the top 24 bits times 2^-24 (exact in float32)."""
    return (np.asarray(word, dtype=np.uint64) >> np.uint64(8)).astype(np.float64) * 2.0 ** -24


def uniform53(w_hi, w_lo):
    """[0, 1) with 53 random bits from two 32-bit words (exact in FP64)."""
    a = (np.asarray(w_hi, dtype=np.uint64) >> np.uint64(5)).astype(np.float64)
    b = (np.asarray(w_lo, dtype=np.uint64) >> np.uint64(6)).astype(np.float64)
    return (a * 67108864.0 + b) * 2.0 ** -53


def normal(w1, w2):
    u1, u2 = uniform(w1), uniform(w2)
    return np.sqrt(-2.0 * np.log(1.0 - u1)) * np.cos(2.0 * np.pi * u2)


def _frac_margin(x):
    """Distance of x from the nearest integer (where floor() changes)."""
    x = np.asarray(x, dtype=np.float64)
    return np.abs(x - np.round(x))


POISSON_SMALL = 10.0        # below: inversion; at and above: transformed rejection
POISSON_MAX_INV = 200       # inversion stops here (F(200) = 1 to FP64 precision for lam < 10)
POISSON_MAX_ATTEMPTS = 64   # rejection attempts (acceptance > 0.8 each)


def poisson_one(lam, seed, agent_key, pixel, stream):
    """One Poisson(lam) draw and its decision margin (see the module docstring)."""
    lam = float(lam)
    if not lam > 0.0:
        return 0, math.inf
    margin = math.inf
    if lam < POISSON_SMALL:
        w = draws(seed, agent_key, pixel, stream, 0)
        u = float(uniform53(w[0], w[1]))
        p = math.exp(-lam)
        f = p
        k = 0
        margin = abs(u - f)
        while u >= f and k < POISSON_MAX_INV:
            k += 1
            p = p * (lam / k)
            f = f + p
            margin = min(margin, abs(u - f))
        return k, margin
    slam = math.sqrt(lam)
    loglam = math.log(lam)
    b = 0.931 + 2.53 * slam
    a = -0.059 + 0.02483 * b
    inv_alpha = 1.1239 + 1.1328 / (b - 3.4)
    v_r = 0.9277 - 3.6224 / (b - 2.0)
    for attempt in range(POISSON_MAX_ATTEMPTS):
        w = draws(seed, agent_key, pixel, stream, attempt)
        u = float(uniform53(w[0], w[1])) - 0.5
        v = float(uniform53(w[2], w[3]))
        us = 0.5 - abs(u)
        x = (2.0 * a / us + b) * u + lam + 0.43
        k = math.floor(x)
        margin = min(margin, float(_frac_margin(x)) / max(1.0, abs(x)), abs(v - v_r))
        if us >= 0.07 and v <= v_r:
            return k, margin
        if k < 0 or (us < 0.013 and v > us):
            continue
        lhs = math.log(v) + math.log(inv_alpha) - math.log(a / (us * us) + b)
        rhs = -lam + k * loglam - math.lgamma(k + 1.0)
        margin = min(margin, abs(lhs - rhs) / max(1.0, abs(rhs)))
        if lhs <= rhs:
            return k, margin
    return math.floor(lam), margin


def poisson(lam, seed, agent_key, pixels, stream):
    """Poisson draws [P] (int64) of rates lam [P] and their margins [P]."""
    lam = np.broadcast_to(np.asarray(lam, dtype=np.float64), np.shape(pixels))
    ks = np.zeros(len(pixels), dtype=np.int64)
    ms = np.zeros(len(pixels), dtype=np.float64)
    for i, px in enumerate(np.asarray(pixels)):
        ks[i], ms[i] = poisson_one(lam[i], seed, agent_key, int(px), stream)
    return ks, ms


NOISE_NONE, NOISE_NORMAL, NOISE_SPECKLE, NOISE_SALT_PEPPER, NOISE_POISSON = 0, 1, 2, 3, 4
DEPTH_NONE, DEPTH_NORMAL, DEPTH_SPECKLE, DEPTH_SALT_PEPPER, DEPTH_POISSON = 0, 1, 2, 3, 4
STREAM_DEPTH, STREAM_RGB0, STREAM_RGB_SP, STREAM_SEG, STREAM_IMU = 0, 1, 4, 5, 7


def _salt_pepper(word, p):
    """(salt, pepper) masks: u < p/2 and p/2 <= u < p, with p the float32 the device receives."""
    u = uniform(word)                                  # exact multiple of 2^-24
    p32 = float(np.float32(p))                         # the one rounding: the ABI carries p as float32
    return u < 0.5 * p32, (u >= 0.5 * p32) & (u < p32)


def noisy_depth(depth, hit, model, sigma, p, seed, agent_key, near, far, scale=1.0, with_margin=False):
    """Depth image [P] with Table II noise; misses keep the miss value.  The result is the FP64 value
    (the device rounds it to float32 once); with_margin adds the per-pixel decision margins."""
    depth = np.asarray(depth, dtype=np.float64)
    n_px = depth.shape[0]
    w = draws(seed, agent_key, np.arange(n_px), STREAM_DEPTH)
    out = depth.copy()
    margin = np.full(n_px, np.inf)
    if model == NOISE_NORMAL:
        out = depth + sigma * normal(w[:, 0], w[:, 1])
    elif model == NOISE_SPECKLE:
        out = depth * (1.0 + sigma * normal(w[:, 0], w[:, 1]))
    elif model == NOISE_SALT_PEPPER:
        salt, pepper = _salt_pepper(w[:, 2], p)
        out = np.where(salt, far, np.where(pepper, near, depth))
    elif model == NOISE_POISSON:
        idx = np.nonzero(hit)[0]
        k, m = poisson(depth[idx] * float(np.float32(scale)), seed, agent_key, idx, STREAM_DEPTH)
        out[idx] = k / float(np.float32(scale))
        margin[idx] = m
    out = np.where(hit, out, depth)
    return (out, margin) if with_margin else out


def _round_half_up(x):
    return np.floor(x + 0.5)


def noisy_rgb(rgb, model, sigma, p, seed, agent_key, scale=1.0, with_margin=False):
    """Planar colour [3, P] uint8 with Table II noise (per channel; salt & pepper per pixel)."""
    rgb = np.asarray(rgb)
    n_px = rgb.shape[1]
    out = rgb.astype(np.float64)
    margin = np.full(n_px, np.inf)
    if model in (NOISE_NORMAL, NOISE_SPECKLE, NOISE_POISSON):
        for c in range(3):
            if model == NOISE_POISSON:
                s32 = float(np.float32(scale))
                k, m = poisson(out[c] * s32, seed, agent_key, np.arange(n_px), STREAM_RGB0 + c)
                x = k / s32 + 0.5
                margin = np.minimum(margin, m)
            else:
                w = draws(seed, agent_key, np.arange(n_px), STREAM_RGB0 + c)
                n = normal(w[:, 0], w[:, 1])
                x = (out[c] + sigma * n if model == NOISE_NORMAL else out[c] * (1.0 + sigma * n)) + 0.5
            margin = np.minimum(margin, _frac_margin(x))
            out[c] = np.clip(np.floor(x), 0, 255)
        res = out.astype(np.uint8)
    elif model == NOISE_SALT_PEPPER:
        w = draws(seed, agent_key, np.arange(n_px), STREAM_RGB_SP)
        salt, pepper = _salt_pepper(w[:, 2], p)
        out[:, salt] = 255
        out[:, pepper] = 0
        res = out.astype(np.uint8)
    else:
        res = rgb.copy()
    return (res, margin) if with_margin else res


def segmentation(tri_id, labels):
    tri_id = np.asarray(tri_id)
    labels = np.asarray(labels)
    return np.where(tri_id >= 0, labels[np.maximum(tri_id, 0)], -1)


def noisy_segmentation(seg, model, sigma, p, seed, agent_key, scale=1.0, salt_label=0, with_margin=False):
    """Label image [P] int32 with Table II noise on its labelled pixels (label >= 0)."""
    seg = np.asarray(seg, dtype=np.int64)
    n_px = seg.shape[0]
    lab = seg >= 0
    out = seg.copy()
    margin = np.full(n_px, np.inf)
    w = draws(seed, agent_key, np.arange(n_px), STREAM_SEG)
    if model in (NOISE_NORMAL, NOISE_SPECKLE):
        n = normal(w[:, 0], w[:, 1])
        if model == NOISE_NORMAL:
            x = sigma * n + 0.5
            new = seg + np.floor(x)
        else:
            x = seg * (1.0 + sigma * n) + 0.5
            new = np.floor(x)
        margin = np.where(lab, _frac_margin(x), np.inf)
        out = np.where(lab, np.clip(new, -2.0 ** 31, 2.0 ** 31 - 1), seg)
    elif model == NOISE_POISSON:
        idx = np.nonzero(lab)[0]
        s32 = float(np.float32(scale))
        k, m = poisson(seg[idx] * s32, seed, agent_key, idx, STREAM_SEG)
        x = k / s32 + 0.5
        out[idx] = np.minimum(np.floor(x), 2.0 ** 31 - 1)
        margin[idx] = np.minimum(m, _frac_margin(x))
    elif model == NOISE_SALT_PEPPER:
        salt, pepper = _salt_pepper(w[:, 2], p)
        out = np.where(lab & salt, salt_label, np.where(lab & pepper, -1, seg))
    res = out.astype(np.int32)
    return (res, margin) if with_margin else res


def imu(state, params, sigma_acc=0.0, sigma_gyro=0.0, seed=0, agent_key=None):
    """[N, 6]: specific force (body frame, m/s^2) and body rates, with optional Normal noise."""
    s = np.asarray(state, dtype=np.float64)
    n = s.shape[0]
    d = dynamics.derivative(s[:, 0:13], s[:, 13:17], params)
    rot = dynamics.quat_to_rot(s[:, 3:7] / np.linalg.norm(s[:, 3:7], axis=1, keepdims=True))
    g = np.array([0.0, 0.0, -params["g"]])
    f_world = d[:, 7:10] - g                              # non-gravitational acceleration
    f_body = np.einsum("nji,nj->ni", rot, f_world)
    out = np.concatenate([f_body, s[:, 10:13]], axis=1)
    if sigma_acc > 0 or sigma_gyro > 0:
        keys = np.arange(n) if agent_key is None else np.asarray(agent_key)
        w = draws(seed, keys[:, None], np.arange(6)[None, :], 7)
        nz = normal(w[..., 0], w[..., 1])
        out[:, 0:3] += sigma_acc * nz[:, 0:3]
        out[:, 3:6] += sigma_gyro * nz[:, 3:6]
    return out
