"""Pins of the oracle's PS / LV outer loops (controller paragraph of Sec. III-A).

The paper names the position (PS) and linear-velocity (LV) controllers and
cites geometric control on SE(3); the law is restated in oracle/dynamics.py.
Fig. 2's step responses are not printed as data, so the pins are closed forms
of the law itself (rate command from a yaw or tilt error, lift, limits),
equilibria, a closed-form steady state, and a frame invariance.  A sign slip,
a transposed R_d or a swapped b1/b2 fails at least one of them.
"""
import math

import numpy as np

from oracle import dynamics as dyn
from workloads import default_params
from workloads.agents import hover_rotor, make_states, yaw_quat


def _state(pos=(0.0, 0.0, 2.0), yaw=0.0, vel=(0.0, 0.0, 0.0), p=None):
    p = p or default_params()
    s = make_states([pos], p, quat=yaw_quat([yaw]), vel=[vel]).astype(np.float64)
    s[:, 3:7] = yaw_quat([yaw])               # exact FP64 values
    s[:, 0:3] = pos
    s[:, 7:10] = vel
    s[:, 13:17] = hover_rotor(p)
    return s


def test_ps_equilibrium_at_setpoint():
    p = default_params(ctrl=dyn.PS)
    s = _state(pos=(1.0, -2.0, 3.0), yaw=0.6, p=p)
    a = np.array([[1.0, -2.0, 3.0, 0.6]])
    c, om = dyn.outer_loop(s, a, p)
    assert abs(c[0] - p["g"]) < 1e-12 and np.max(np.abs(om)) < 1e-12
    out = s.copy()
    for _ in range(50):
        out = dyn.step(out, a, p)
    assert np.max(np.abs(out[:, 0:13] - s[:, 0:13])) < 1e-11


def test_lv_constant_velocity_without_drag():
    """LV with v = v_d, level, no drag: the velocity is held and p moves on a straight line."""
    p = default_params(ctrl=dyn.LV, k_lin=(0.0, 0.0, 0.0))
    v = (0.7, -0.4, 0.25)
    s = _state(vel=v, yaw=-1.1, p=p)
    a = np.array([[*v, -1.1]])
    out = s.copy()
    for k in range(1, 41):
        out = dyn.step(out, a, p)
        assert np.allclose(out[0, 7:10], v, atol=1e-11)
        assert np.allclose(out[0, 0:3], np.array([0, 0, 2.0]) + np.array(v) * k * p["dt"], atol=1e-10)


def test_yaw_error_rate_command():
    """Level, yaw psi, command psi_d: Omega_des = (0, 0, -k_att_z sin(psi - psi_d)), c = g."""
    p = default_params(ctrl=dyn.PS)
    for psi, psi_d in ((0.3, 0.0), (-2.0, 1.5), (3.0, -3.0)):
        s = _state(yaw=psi, p=p)
        c, om = dyn.outer_loop(s, np.array([[0.0, 0.0, 2.0, psi_d]]), p)
        assert abs(c[0] - p["g"]) < 1e-12
        assert np.allclose(om[0], [0.0, 0.0, -p["k_att"][2] * math.sin(psi - psi_d)], atol=1e-12)


def test_horizontal_error_tilts_toward_the_goal():
    """Level, yaw 0, goal +x by e: F = (k_p e, 0, g); R_d is a pitch by theta with sin theta = a / |F|,
    so Omega_des = (0, k_att_y sin theta, 0) (positive pitch tips thrust toward +x); a goal +y gives a
    negative roll rate of the same form."""
    p = default_params(ctrl=dyn.PS)
    g = p["g"]
    for e in (0.1, 0.5, -0.3):
        s = _state(p=p)
        c, om = dyn.outer_loop(s, np.array([[e, 0.0, 2.0, 0.0]]), p)
        acc = p["k_pos"][0] * e
        assert abs(c[0] - g) < 1e-12
        assert np.allclose(om[0], [0.0, p["k_att"][1] * acc / math.hypot(acc, g), 0.0], atol=1e-12)
        c, om = dyn.outer_loop(s, np.array([[0.0, e, 2.0, 0.0]]), p)
        acc = p["k_pos"][1] * e
        assert np.allclose(om[0], [-p["k_att"][0] * acc / math.hypot(acc, g), 0.0, 0.0], atol=1e-12)


def test_velocity_damping_and_vertical_lift():
    """PS: a velocity v_x at the setpoint commands a = -k_v v_x; a height error gives c = g - k_p e_z."""
    p = default_params(ctrl=dyn.PS)
    s = _state(vel=(0.5, 0.0, 0.0), p=p)
    c, om = dyn.outer_loop(s, np.array([[0.0, 0.0, 2.0, 0.0]]), p)
    acc = -p["k_vel"][0] * 0.5
    assert np.allclose(om[0], [0.0, p["k_att"][1] * acc / math.hypot(acc, p["g"]), 0.0], atol=1e-12)
    s = _state(p=p)
    c, om = dyn.outer_loop(s, np.array([[0.0, 0.0, 2.7, 0.0]]), p)
    assert abs(c[0] - (p["g"] + p["k_pos"][2] * 0.7)) < 1e-12 and np.max(np.abs(om)) < 1e-12


def test_tilt_and_lift_limits():
    p = default_params(ctrl=dyn.PS)
    s = _state(p=p)
    # far goal along +x: the commanded tilt is exactly max_tilt, and the lift stays g
    c, om = dyn.outer_loop(s, np.array([[100.0, 0.0, 2.0, 0.0]]), p)
    assert abs(c[0] - p["g"]) < 1e-12
    assert np.allclose(om[0], [0.0, p["k_att"][1] * math.sin(p["max_tilt"]), 0.0], atol=1e-12)
    # goal far below: the vertical command is raised to g / 4
    c, om = dyn.outer_loop(s, np.array([[0.0, 0.0, -50.0, 0.0]]), p)
    assert abs(c[0] - 0.25 * p["g"]) < 1e-12 and np.max(np.abs(om)) < 1e-12


def test_frame_invariance_about_z():
    """Rotating positions, velocities, goal and yaw together about z leaves c and the body-frame
    rate command unchanged."""
    p = default_params(ctrl=dyn.PS)
    rng = np.random.default_rng(0)
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    base = _state(pos=(0.3, -0.2, 1.5), vel=(0.4, 0.1, -0.2), p=p)
    base[:, 3:7] = q
    goal = np.array([[1.2, 0.5, 2.5, 0.4]])
    c0, om0 = dyn.outer_loop(base, goal, p)
    for gam in (0.7, -2.1):
        rz = dyn.quat_to_rot(yaw_quat([gam]))[0]
        s = base.copy()
        s[0, 0:3] = rz @ base[0, 0:3]
        s[0, 7:10] = rz @ base[0, 7:10]
        s[0, 3:7] = dyn.quat_mul(yaw_quat([gam]), base[:, 3:7])[0]
        g2 = goal.copy()
        g2[0, 0:3] = rz @ goal[0, 0:3]
        g2[0, 3] = goal[0, 3] + gam
        c1, om1 = dyn.outer_loop(s, g2, p)
        assert abs(c1[0] - c0[0]) < 1e-12 and np.allclose(om1, om0, atol=1e-12)


def test_step_responses_settle():
    """PS settles on the setpoint and yaw; LV settles at the drag-balanced speed
    k_v v_d / (k_v + k_lin / m) (level flight, isotropic linear drag)."""
    p = default_params(ctrl=dyn.PS)
    s = _state(p=p)
    a = np.array([[1.0, -0.5, 2.5, 0.8]])
    for _ in range(500):
        s = dyn.step(s, a, p)
    assert np.allclose(s[0, 0:3], a[0, 0:3], atol=1e-5)
    assert abs(2 * math.atan2(s[0, 6], s[0, 3]) - 0.8) < 1e-5
    p = default_params(ctrl=dyn.LV)
    s = _state(p=p)
    vd = np.array([1.0, 0.5, -0.2])
    a = np.array([[*vd, -0.5]])
    for _ in range(400):
        s = dyn.step(s, a, p)
    kv, kl = p["k_vel"][0], p["k_lin"][0] / p["mass"]
    assert np.allclose(s[0, 7:10], kv * vd / (kv + kl), atol=1e-6)
