"""Pins of the oracle's sensor-noise generator and derived sensors (Sec. III-D Table II, Table I sensors)."""
import json
import math
import os

import numpy as np
import pytest

from oracle import noise
from oracle import dynamics as dyn
from workloads import default_params
from workloads.agents import make_states, hover_rotor, yaw_quat


def test_philox_known_answers():
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "philox_kat.json")))
    for v in gold["vectors"]:
        ctr = np.array([int(x, 16) for x in v["ctr"]], dtype=np.uint64)
        key = np.array([int(x, 16) for x in v["key"]], dtype=np.uint64)
        out = noise.philox4x32_10(ctr, key)
        assert ["%08x" % int(x) for x in out] == v["out"]


def test_uniform_and_normal_statistics():
    w = noise.draws(12345, 7, np.arange(200_000), 0)
    u = noise.uniform(w[:, 0])
    assert u.min() >= 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 0.005 and abs(u.var() - 1 / 12) < 0.002
    z = noise.normal(w[:, 0], w[:, 1])
    assert abs(z.mean()) < 0.01 and abs(z.std() - 1.0) < 0.01
    # different streams / keys give different draws
    assert not np.array_equal(noise.draws(12345, 8, np.arange(10), 0), noise.draws(12345, 7, np.arange(10), 0))
    assert not np.array_equal(noise.draws(12345, 7, np.arange(10), 1), noise.draws(12345, 7, np.arange(10), 0))


def test_depth_noise_models():
    n = 100_000
    depth = np.full(n, 5.0)
    hit = np.ones(n, dtype=bool)
    hit[:10] = False
    out = noise.noisy_depth(depth, hit, noise.DEPTH_NORMAL, 0.02, 0.0, 9, 3, 0.01, 100.0)
    assert np.all(out[:10] == 5.0)
    assert abs(np.std(out[10:]) - 0.02) < 0.001 and abs(np.mean(out[10:]) - 5.0) < 0.001
    out = noise.noisy_depth(depth, hit, noise.DEPTH_SPECKLE, 0.1, 0.0, 9, 3, 0.01, 100.0)
    assert abs(np.std(out[10:]) - 0.5) < 0.01
    out = noise.noisy_depth(depth, hit, noise.DEPTH_SALT_PEPPER, 0.0, 0.2, 9, 3, 0.01, 100.0)
    assert abs(np.mean(out[10:] == 100.0) - 0.1) < 0.005 and abs(np.mean(out[10:] == 0.01) - 0.1) < 0.005
    assert np.all((out[10:] == 5.0) | (out[10:] == 100.0) | (out[10:] == 0.01))


def test_rgb_noise_models():
    rgb = np.full((3, 50_000), 128, dtype=np.uint8)
    out = noise.noisy_rgb(rgb, noise.DEPTH_NORMAL, 10.0, 0.0, 5, 1)
    assert abs(out.astype(float).std() - 10.0) < 0.3 and out.dtype == np.uint8
    out = noise.noisy_rgb(rgb, noise.DEPTH_SALT_PEPPER, 0.0, 0.1, 5, 1)
    white = np.all(out == 255, axis=0)
    black = np.all(out == 0, axis=0)
    assert abs(white.mean() - 0.05) < 0.005 and abs(black.mean() - 0.05) < 0.005


def test_segmentation_lookup():
    labels = np.array([7, 7, 3, 9])
    assert noise.segmentation(np.array([0, 2, -1, 3]), labels).tolist() == [7, 3, -1, 9]


def test_imu_closed_forms():
    p = default_params()
    hov = make_states([[0, 0, 5.0]], p, quat=yaw_quat([0.8]), omega=[[0.1, -0.2, 0.3]]).astype(np.float64)
    hov[:, 13:17] = hover_rotor(p)
    out = noise.imu(hov, p)
    # hover thrust, at rest: the accelerometer reads +g along body z, the gyro the body rates
    assert np.allclose(out[0, 0:3], [0, 0, p["g"]], atol=1e-12) and np.allclose(out[0, 3:6], [0.1, -0.2, 0.3])
    # tilted, moving, rotors off, no drag: free fall reads zero specific force
    p0 = default_params(k_lin=(0.0, 0.0, 0.0))
    q = np.array([math.cos(0.3), math.sin(0.3), 0.0, 0.0])
    ff = make_states([[0, 0, 5.0]], p0, quat=[q], vel=[[1.0, 2.0, -3.0]], rotor=[[0, 0, 0, 0]]).astype(np.float64)
    assert np.allclose(noise.imu(ff, p0)[0, 0:3], 0.0, atol=1e-12)
    # with linear drag the reading is the drag acceleration -k v_B / m
    ffd = ff.copy()
    out = noise.imu(ffd, p)
    rot = dyn.quat_to_rot(ffd[0, 3:7] / np.linalg.norm(ffd[0, 3:7]))
    assert np.allclose(out[0, 0:3], -0.1 * rot.T @ ffd[0, 7:10] / p["mass"], atol=1e-12)


# ---------------------------------------------------------------------------
# Table II remainder: Poisson, speckle colour, segmentation noise
# ---------------------------------------------------------------------------

def _pmf(k, lam):
    return math.exp(-lam + k * math.log(lam) - math.lgamma(k + 1.0))


def _draw_many(lam, n, seed=77, stream=3):
    return noise.poisson(np.full(n, lam), seed, 5, np.arange(n), stream)[0]


@pytest.mark.parametrize("lam", [0.3, 2.5, 9.9, 10.0, 37.5, 1000.0])
def test_poisson_mean_equals_variance(lam):
    """Poisson(lam) has mean = variance = lam (inversion below 10, transformed rejection at and above)."""
    n = 20000
    k = _draw_many(lam, n)
    assert k.min() >= 0
    se_mean = math.sqrt(lam / n)
    assert abs(k.mean() - lam) < 5 * se_mean, (k.mean(), lam)
    # variance of the sample variance of a Poisson: (lam + 2 lam^2 (n / (n - 1))) / n ~ (lam + 2 lam^2) / n
    se_var = math.sqrt((lam + 2 * lam * lam) / n)
    assert abs(k.var(ddof=1) - lam) < 5 * se_var, (k.var(ddof=1), lam)


def test_poisson_zero_rate_and_determinism():
    k, m = noise.poisson(np.zeros(5), 1, 2, np.arange(5), 3)
    assert np.all(k == 0)
    a = _draw_many(12.5, 300)
    b = _draw_many(12.5, 300)
    assert np.array_equal(a, b)
    assert not np.array_equal(a, _draw_many(12.5, 300, seed=78))


@pytest.mark.parametrize("lam", [4.0, 12.0, 30.0])
def test_poisson_histogram_matches_pmf(lam):
    """Chi-square goodness of fit of the draws against e^-lam lam^k / k! (bins of expected count >= 20,
    tails pooled); a wrong constant of the rejection method or a slip in the inversion distorts it."""
    from scipy.stats import chi2
    n = 60000
    k = _draw_many(lam, n, seed=1234)
    kmax = int(lam + 12 * math.sqrt(lam) + 10)
    p = np.array([_pmf(j, lam) for j in range(kmax + 1)])
    obs = np.bincount(np.minimum(k, kmax), minlength=kmax + 1).astype(float)
    p[-1] += max(0.0, 1.0 - p.sum())
    exp = p * n
    # pool bins from both ends until each expected count is >= 20
    bins_o, bins_e, acc_o, acc_e = [], [], 0.0, 0.0
    for o, e in zip(obs, exp):
        acc_o += o
        acc_e += e
        if acc_e >= 20:
            bins_o.append(acc_o)
            bins_e.append(acc_e)
            acc_o = acc_e = 0.0
    bins_o[-1] += acc_o
    bins_e[-1] += acc_e
    stat = float(np.sum((np.array(bins_o) - np.array(bins_e)) ** 2 / np.array(bins_e)))
    dof = len(bins_o) - 1
    assert stat < chi2.ppf(0.9999, dof), (stat, dof)


def test_poisson_inversion_is_the_cdf_definition():
    """Below the switch the draw is the smallest k with u < F(k), F summed exactly from the pmf."""
    for lam in (0.7, 3.3, 8.0):
        for px in range(200):
            k, _ = noise.poisson_one(lam, 99, 3, px, 6)
            w = noise.draws(99, 3, px, 6, 0)
            u = float(noise.uniform53(w[0], w[1]))
            f_k = math.fsum(_pmf(j, lam) for j in range(k + 1))
            f_prev = math.fsum(_pmf(j, lam) for j in range(k))
            assert f_prev - 1e-12 <= u < f_k + 1e-12, (lam, px, k, u, f_prev, f_k)


def test_uniform53_exact_and_in_range():
    w = noise.draws(5, 6, np.arange(50000), 0)
    u = noise.uniform53(w[:, 0], w[:, 1])
    assert u.min() >= 0.0 and u.max() < 1.0 and abs(u.mean() - 0.5) < 0.005
    # every value is a multiple of 2^-53 built from the top 27 and 26 bits of the two words
    a = (w[:, 0] >> np.uint64(5)).astype(np.uint64)
    b = (w[:, 1] >> np.uint64(6)).astype(np.uint64)
    assert np.array_equal((u * 2.0 ** 53).astype(np.uint64), (a << np.uint64(26)) | b)


def test_depth_poisson_mean_and_variance():
    """Depth Poisson at s counts per metre: mean D, variance D / s; misses untouched."""
    n, d, s = 20000, 4.0, 50.0
    depth = np.full(n, d)
    hit = np.ones(n, dtype=bool)
    hit[:7] = False
    out = noise.noisy_depth(depth, hit, noise.NOISE_POISSON, 0.0, 0.0, 3, 11, 0.01, 100.0, scale=s)
    assert np.all(out[:7] == d)
    v = out[7:]
    assert abs(v.mean() - d) < 5 * math.sqrt(d / s / n)
    assert abs(v.var() - d / s) < 0.05 * d / s
    # values are multiples of 1 / s
    assert np.allclose(v * s, np.round(v * s), atol=1e-9)


def test_rgb_speckle_std_scales_with_value():
    """Speckle: v (1 + sigma n) rounded, so the spread is sigma v (plus the rounding's 1/12 variance) and a
    zero channel stays zero."""
    n, sigma = 50000, 0.1
    for v in (40, 100):
        rgb = np.full((3, n), v, dtype=np.uint8)
        out = noise.noisy_rgb(rgb, noise.NOISE_SPECKLE, sigma, 0.0, 8, 2).astype(float)
        assert abs(out.mean() - v) < 0.05
        assert abs(out.std() - math.sqrt((sigma * v) ** 2 + 1 / 12)) < 0.02 * sigma * v
    zero = noise.noisy_rgb(np.zeros((3, 100), dtype=np.uint8), noise.NOISE_SPECKLE, 0.5, 0.0, 8, 2)
    assert np.all(zero == 0)


def test_rgb_poisson_mean_and_variance():
    n, v, s = 40000, 60, 4.0
    rgb = np.full((3, n), v, dtype=np.uint8)
    out, m = noise.noisy_rgb(rgb, noise.NOISE_POISSON, 0.0, 0.0, 21, 4, scale=s, with_margin=True)
    out = out.astype(float)
    # exact moments of floor(K / s + 1/2) for K ~ Poisson(v s), summed over the pmf (the round-half-up
    # rule biases the mean by about +1/8 at s = 4)
    ks = np.arange(int(v * s + 30 * math.sqrt(v * s)))
    pk = np.array([_pmf(int(k), v * s) for k in ks])
    vals = np.floor(ks / s + 0.5)
    mean = float((pk * vals).sum())
    var = float((pk * vals * vals).sum() - mean * mean)
    assert abs(out.mean() - mean) < 5 * math.sqrt(var / (3 * n))
    assert abs(out.var() - var) < 0.05 * var
    assert np.all(m >= 0)
    dark = noise.noisy_rgb(np.zeros((3, 10), dtype=np.uint8), noise.NOISE_POISSON, 0.0, 0.0, 21, 4, scale=s)
    assert np.all(dark == 0)


def test_salt_pepper_threshold_is_the_float32_p():
    """The decision compares the 24-bit uniform with the float32 p (and p / 2): a p that float32 rounds
    down moves the threshold below a uniform that sits between the two."""
    w = noise.draws(1, 2, np.arange(4000), noise.STREAM_DEPTH)
    u = noise.uniform(w[:, 2])
    depth = np.full(4000, 3.0)
    hit = np.ones(4000, dtype=bool)
    p = 0.1 + 1e-12                                   # float32(p) = 0.100000001490116...
    out = noise.noisy_depth(depth, hit, noise.NOISE_SALT_PEPPER, 0.0, p, 1, 2, 0.01, 100.0)
    p32 = float(np.float32(p))
    assert np.array_equal(out == 100.0, u < p32 / 2)
    assert np.array_equal(out == 0.01, (u >= p32 / 2) & (u < p32))


def test_segmentation_noise_models():
    n = 40000
    seg = np.full(n, 7, dtype=np.int32)
    seg[:100] = -1                                   # misses
    seg[100:200] = -3                                # a swarm member's label
    out = noise.noisy_segmentation(seg, noise.NOISE_NORMAL, 1.5, 0.0, 4, 9)
    assert np.all(out[:200] == seg[:200])
    off = out[200:].astype(float) - 7
    assert np.all(off == np.round(off)) and abs(off.mean()) < 0.05
    assert abs(off.var() - (1.5 ** 2 + 1 / 12)) < 0.1
    out = noise.noisy_segmentation(seg, noise.NOISE_SALT_PEPPER, 0.0, 0.2, 4, 9, salt_label=42)
    body = out[200:]
    assert abs(np.mean(body == 42) - 0.1) < 0.01 and abs(np.mean(body == -1) - 0.1) < 0.01
    assert np.all((body == 7) | (body == 42) | (body == -1)) and np.all(out[:200] == seg[:200])
    out = noise.noisy_segmentation(seg, noise.NOISE_POISSON, 0.0, 0.0, 4, 9, scale=1.0)
    assert abs(out[200:].mean() - 7) < 0.05 and abs(out[200:].var() - 7) < 0.3
    out = noise.noisy_segmentation(seg, noise.NOISE_SPECKLE, 0.1, 0.0, 4, 9)
    assert abs(out[200:].std() - math.sqrt(0.49 + 1 / 12)) < 0.05
    zero = noise.noisy_segmentation(np.zeros(50, dtype=np.int32), noise.NOISE_SPECKLE, 0.5, 0.0, 4, 9)
    assert np.all(zero == 0)
