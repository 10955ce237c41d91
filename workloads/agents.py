"""Seeded start states and action sequences.

State row layout (17 float32 per agent):
  [0:3]   p      position, world frame, m
  [3:7]   q      unit quaternion (w, x, y, z), body -> world, Hamilton convention
  [7:10]  v      velocity, world frame, m/s
  [10:13] Omega  body angular rate, rad/s
  [13:17] w      normalised rotor speeds (thrust of rotor i is w_i^2, N)
Action row (4 float32): CTBR (collective acceleration m/s^2, body-rate
command x, y, z rad/s) or SRT (four rotor thrusts, N).

Initial-state randomisation follows Sec. III-D (uniform positions, random
yaw, agents started away from obstacles).
"""
import math

import numpy as np

STATE_DIM = 17
ACTION_DIM = 4


def hover_rotor(params):
    """Normalised rotor speed at which four rotors carry the weight."""
    return math.sqrt(params["mass"] * params["g"] / 4.0)


def yaw_quat(yaw):
    yaw = np.asarray(yaw, dtype=np.float64)
    return np.stack([np.cos(yaw / 2), np.zeros_like(yaw), np.zeros_like(yaw), np.sin(yaw / 2)], axis=-1)


def make_states(pos, params, quat=None, vel=None, omega=None, rotor=None):
    """Assemble [N,17] float32 states; rotors default to hover."""
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    n = pos.shape[0]
    s = np.zeros((n, STATE_DIM), dtype=np.float64)
    s[:, 0:3] = pos
    s[:, 3:7] = np.array([1.0, 0.0, 0.0, 0.0]) if quat is None else np.asarray(quat, dtype=np.float64).reshape(-1, 4)
    if vel is not None:
        s[:, 7:10] = np.asarray(vel, dtype=np.float64).reshape(-1, 3)
    if omega is not None:
        s[:, 10:13] = np.asarray(omega, dtype=np.float64).reshape(-1, 3)
    s[:, 13:17] = hover_rotor(params) if rotor is None else np.asarray(rotor, dtype=np.float64).reshape(-1, 4)
    return s.astype(np.float32)


def random_actions(seed, steps, n, params, c_range=(0.5, 2.0), rate=3.0):
    """CTBR actions [steps, n, 4]: c ~ U(c_range) * g, body rates ~ U(-rate, rate)^3."""
    rng = np.random.default_rng(seed)
    a = np.empty((steps, n, 4), dtype=np.float64)
    a[..., 0] = rng.uniform(c_range[0], c_range[1], size=(steps, n)) * params["g"]
    a[..., 1:4] = rng.uniform(-rate, rate, size=(steps, n, 3))
    return a.astype(np.float32)


def box_room_start(params, start=(5.0, 5.0, 2.0)):
    return make_states(np.asarray(start)[None], params)


def forest_starts(seed, n, scene, params, margin=0.5, span=18.0, z_range=(1.0, 3.0)):
    """Uniform free-space starts in the forest: clear of every trunk by r + margin."""
    rng = np.random.default_rng(seed)
    trees = scene["trees"]
    pos = np.empty((n, 3))
    k = 0
    while k < n:
        xy = rng.uniform(-span, span, size=2)
        d = np.hypot(trees[:, 0] - xy[0], trees[:, 1] - xy[1]) - trees[:, 2]
        if np.all(d > margin):
            pos[k, :2] = xy
            pos[k, 2] = rng.uniform(*z_range)
            k += 1
    yaw = rng.uniform(-math.pi, math.pi, size=n)
    return make_states(pos, params, quat=yaw_quat(yaw))


def room_graph_starts(seed, n, scene, params, margin=0.3, z_range=(1.0, 2.0)):
    """Free-space starts inside random rooms, clear of boxes and pillars by margin."""
    rng = np.random.default_rng(seed)
    g, room = scene["grid"], scene["room"]
    blo, bhi, pil = scene["box_lo"], scene["box_hi"], scene["pillars"]
    pos = np.empty((n, 3))
    k = 0
    while k < n:
        cell = rng.integers(0, g * g)
        x = (cell // g) * room + rng.uniform(0.5, room - 0.5)
        y = (cell % g) * room + rng.uniform(0.5, room - 0.5)
        z = rng.uniform(*z_range)
        p = np.array([x, y, z])
        inside = np.all((p >= blo - margin) & (p <= bhi + margin), axis=1)
        near_pil = np.hypot(pil[:, 0] - x, pil[:, 1] - y) < pil[:, 2] + margin
        if not inside.any() and not near_pil.any():
            pos[k] = p
            k += 1
    yaw = rng.uniform(-math.pi, math.pi, size=n)
    return make_states(pos, params, quat=yaw_quat(yaw))


def multi_scene_split(seed, n_agents, n_scenes, min_per=16):
    """Agents per scene ~ multinomial(n, Dirichlet(1)) with a floor of min_per each."""
    rng = np.random.default_rng(seed)
    while True:
        w = rng.dirichlet(np.ones(n_scenes))
        c = rng.multinomial(n_agents, w)
        if c.min() >= min_per:
            return c
