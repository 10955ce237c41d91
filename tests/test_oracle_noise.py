"""Pins of the oracle's sensor-noise generator and derived sensors (Sec. III-D Table II, Table I sensors)."""
import json
import math
import os

import numpy as np

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
