"""Sensor noise and derived sensors (Sec. III-D, Table II; Table I sensor set), FP64 reference.

Random numbers come from the counter-based generator Philox4x32-10 (Salmon,
Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC 2011):
ten rounds of two 32x32->64-bit multiplies with the round keys bumped by the
Weyl constants.  A draw is keyed by (seed, agent key, pixel, stream) so it does
not depend on batch composition.

Readings (Table II names the models only):
  uniform   u = (x >> 8) * 2^-24 in [0, 1) from one 32-bit output word
  normal    Box-Muller: sqrt(-2 ln(1 - u1)) * cos(2 pi u2)
  depth     Normal:  D + sigma n          Speckle: D (1 + sigma n)
            Salt & pepper: with probability p/2 -> far (salt), p/2 -> near (pepper)
  colour    Normal / speckle per channel on the 0..255 value, rounded to nearest and clamped;
            salt & pepper -> 255 / 0 for the whole pixel
  segmentation label = per-triangle label of the hit triangle (-1 on a miss)
  IMU       accelerometer: specific force (F_b + d) / m in the body frame at the state;
            gyro: body rates; optional Normal noise per axis
Poisson and the RedWood depth model are not built (parameters not in the paper).
"""
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


def draws(seed, agent_key, pixel, stream):
    """Four 32-bit words for each (agent key, pixel) at the given stream index."""
    agent_key = np.asarray(agent_key, dtype=np.uint64)
    pixel = np.asarray(pixel, dtype=np.uint64)
    shape = np.broadcast(agent_key, pixel).shape
    ctr = np.zeros(shape + (4,), dtype=np.uint64)
    ctr[..., 0] = pixel
    ctr[..., 1] = agent_key
    ctr[..., 2] = stream
    key = np.zeros(shape + (2,), dtype=np.uint64)
    key[..., 0] = seed & MASK
    key[..., 1] = (seed >> 32) & MASK
    return philox4x32_10(ctr, key)


def uniform(word):
    """[0, 1) from a 32-bit word: the top 24 bits times 2^-24 (exact in float32)."""
    return (np.asarray(word, dtype=np.uint64) >> np.uint64(8)).astype(np.float64) * 2.0 ** -24


def normal(w1, w2):
    u1, u2 = uniform(w1), uniform(w2)
    return np.sqrt(-2.0 * np.log(1.0 - u1)) * np.cos(2.0 * np.pi * u2)


DEPTH_NONE, DEPTH_NORMAL, DEPTH_SPECKLE, DEPTH_SALT_PEPPER = 0, 1, 2, 3


def noisy_depth(depth, hit, model, sigma, p, seed, agent_key, near, far):
    """Depth image [P] with Table II noise; misses keep the miss value."""
    depth = np.asarray(depth, dtype=np.float64)
    w = draws(seed, agent_key, np.arange(depth.shape[0]), 0)
    out = depth.copy()
    if model == DEPTH_NORMAL:
        out = depth + sigma * normal(w[:, 0], w[:, 1])
    elif model == DEPTH_SPECKLE:
        out = depth * (1.0 + sigma * normal(w[:, 0], w[:, 1]))
    elif model == DEPTH_SALT_PEPPER:
        u = uniform(w[:, 2]).astype(np.float32)
        p32 = np.float32(p)
        out = np.where(u < p32 * np.float32(0.5), far, np.where(u < p32, near, depth))
    return np.where(hit, out, depth)


def noisy_rgb(rgb, model, sigma, p, seed, agent_key):
    """Planar colour [3, P] uint8 with Table II noise (per channel; salt & pepper per pixel)."""
    rgb = np.asarray(rgb)
    n_px = rgb.shape[1]
    out = rgb.astype(np.float64)
    if model in (DEPTH_NORMAL, DEPTH_SPECKLE):
        for c in range(3):
            w = draws(seed, agent_key, np.arange(n_px), 1 + c)
            n = normal(w[:, 0], w[:, 1])
            val = out[c] + sigma * n if model == DEPTH_NORMAL else out[c] * (1.0 + sigma * n)
            out[c] = np.clip(np.floor(val + 0.5), 0, 255)
        return out.astype(np.uint8)
    if model == DEPTH_SALT_PEPPER:
        w = draws(seed, agent_key, np.arange(n_px), 4)
        u = uniform(w[:, 2]).astype(np.float32)
        p32 = np.float32(p)
        salt = u < p32 * np.float32(0.5)
        pepper = (~salt) & (u < p32)
        out[:, salt] = 255
        out[:, pepper] = 0
        return out.astype(np.uint8)
    return rgb.copy()


def segmentation(tri_id, labels):
    tri_id = np.asarray(tri_id)
    labels = np.asarray(labels)
    return np.where(tri_id >= 0, labels[np.maximum(tri_id, 0)], -1)


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
