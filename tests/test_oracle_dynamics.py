"""Pins of the FP64 dynamics oracle (Sec. III-A, Eqs. 1-4) against closed forms.

Each pin is chosen so that a plausible slip in the oracle (a dropped term, a
sign, a transposed rotation, a wrong RK4 weight) fails at least one of them.
"""
import math

import numpy as np
import pytest

from oracle import dynamics as dyn
from workloads import default_params
from workloads.agents import make_states, hover_rotor, yaw_quat


def _p(**kw):
    return default_params(**kw)


def test_hover_equilibrium_zero_acceleration():
    """P5: level attitude, zero rates, hover rotors, CTBR (g, 0, 0, 0) -> zero acceleration."""
    p = _p()
    s = make_states([[1.0, 2.0, 3.0]], p).astype(np.float64)
    s[:, 13:17] = hover_rotor(p)            # exact FP64 hover speed (the float32 input rounds it)
    a = np.array([[p["g"], 0.0, 0.0, 0.0]])
    s_out = s.copy()
    for _ in range(100):
        s_out = dyn.step(s_out, a, p)
    assert np.max(np.abs(s_out[0, 0:3] - s[0, 0:3])) < 1e-12
    assert np.max(np.abs(s_out[0, 7:13])) < 1e-12
    assert np.allclose(s_out[0, 13:17], hover_rotor(p), atol=1e-12)


def test_free_fall_without_drag_is_exact_quadratic():
    """P6: zero thrust (SRT 0, rotors 0) and no drag: p = p0 + v0 t - g t^2/2 z exactly (RK4 is exact)."""
    p = _p(ctrl=dyn.SRT, k_lin=(0.0, 0.0, 0.0))
    v0 = np.array([0.3, -0.2, 1.5])
    s = make_states([[0.0, 0.0, 10.0]], p, vel=[v0], rotor=[[0, 0, 0, 0]], quat=yaw_quat([0.7])).astype(np.float64)
    v0 = s[0, 7:10].copy()                  # the float32-rounded start velocity
    a = np.zeros((1, 4))
    for k in range(1, 51):
        s = dyn.step(s, a, p)
        t = k * p["dt"]
        expect = np.array([0.0, 0.0, 10.0]) + v0 * t - 0.5 * p["g"] * t * t * np.array([0, 0, 1.0])
        assert np.allclose(s[0, 0:3], expect, atol=1e-11, rtol=0)
        assert np.allclose(s[0, 7:10], v0 - p["g"] * t * np.array([0, 0, 1.0]), atol=1e-11, rtol=0)


def test_free_fall_linear_drag_matches_rk4_amplification():
    """P6: v' = -(k/m)(v - v_inf): one RK4 step multiplies v - v_inf by the 4th-order Taylor polynomial of e^z."""
    k, m = 0.1, 1.0
    p = _p(ctrl=dyn.SRT, k_lin=(k, k, k), mass=m)
    v0 = np.array([2.0, -1.0, 3.0])
    q = np.array([[math.cos(0.4), 0.3, -0.2, math.sin(0.4)]])
    q /= np.linalg.norm(q)
    s = make_states([[0.0, 0.0, 0.0]], p, vel=[v0], rotor=[[0, 0, 0, 0]], quat=q).astype(np.float64)
    v0 = s[0, 7:10].copy()
    v_inf = np.array([0.0, 0.0, -m * p["g"] / k])
    z = -k * p["dt"] / m
    amp = 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24
    for n in range(1, 41):
        s = dyn.step(s, np.zeros((1, 4)), p)
        assert np.allclose(s[0, 7:10], v_inf + (v0 - v_inf) * amp ** n, atol=1e-11, rtol=0)
    # and it tracks the exact exponential within the RK4 local error bound
    t = 40 * p["dt"]
    exact = v_inf + (v0 - v_inf) * math.exp(-k * t / m)
    assert np.allclose(s[0, 7:10], exact, atol=1e-9)


def _spin_state(p, om, quat=None):
    f = hover_rotor(p) ** 2
    return make_states([[0.0, 0.0, 5.0]], p, omega=[om], quat=quat, rotor=[[math.sqrt(f)] * 4]).astype(np.float64), \
        np.full((1, 4), f)


def test_principal_axis_spin_rk4_quaternion_factor():
    """P7: equal thrusts (zero torque), Omega = w e_z: each step turns yaw by 2 atan2(th - th^3/6, 1 - th^2/2 + th^4/24)."""
    p = _p(ctrl=dyn.SRT)
    wz = 2.5
    s, a = _spin_state(p, [0.0, 0.0, wz])
    th = wz * p["dt"] / 2
    per_step = 2 * math.atan2(th - th ** 3 / 6, 1 - th ** 2 / 2 + th ** 4 / 24)
    for n in range(1, 31):
        s = dyn.step(s, a, p)
        expect = yaw_quat(n * per_step)
        assert np.allclose(s[0, 3:7], expect, atol=1e-12)
        assert np.allclose(s[0, 10:13], [0, 0, wz], atol=1e-12)


def test_torque_free_precession_rk4_factor():
    """P8: J_x = J_y: Omega_x + i Omega_y is multiplied by the RK4 polynomial of i*lam*h, lam = (Jz-Jx)/Jx Omega_z."""
    p = _p(ctrl=dyn.SRT)
    jx, jz = p["J"][0], p["J"][2]
    om0 = np.array([0.7, -0.4, 3.0])
    s, a = _spin_state(p, om0)
    om0 = s[0, 10:13].copy()                 # the float32-rounded start rates
    lam = (jz - jx) / jx * om0[2]
    z = 1j * lam * p["dt"]
    amp = 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24
    c0 = om0[0] + 1j * om0[1]
    for n in range(1, 51):
        s = dyn.step(s, a, p)
        c = c0 * amp ** n
        assert abs(s[0, 10] - c.real) < 1e-12 and abs(s[0, 11] - c.imag) < 1e-12
        assert abs(s[0, 12] - om0[2]) < 1e-12
    t = 50 * p["dt"]
    exact = c0 * np.exp(1j * lam * t)
    assert abs(s[0, 10] + 1j * s[0, 11] - exact) < 1e-6


def test_rotor_lag_step_response():
    """P9: constant command f_des: thrust after k steps is (w_des + (w0 - w_des) e^{-k h / tau})^2."""
    p = _p(ctrl=dyn.SRT)
    f_des = np.array([[1.0, 2.0, 3.0, 4.0]])
    s = make_states([[0, 0, 5.0]], p, rotor=[[0.5, 0.5, 2.5, 0.0]]).astype(np.float64)
    w0 = s[0, 13:17].copy()
    for k in range(1, 21):
        s = dyn.step(s, f_des, p)
        w = np.sqrt(f_des[0]) + (w0 - np.sqrt(f_des[0])) * math.exp(-k * p["dt"] / p["tau_motor"])
        assert np.allclose(s[0, 13:17] ** 2, w ** 2, atol=1e-12)


def test_thrust_clamped_to_limits():
    p = _p(ctrl=dyn.SRT)
    f = dyn.controller(np.zeros((1, 17)), np.array([[-1.0, 100.0, 0.5, p["f_max"]]]), p)
    assert np.allclose(f, [[0.0, p["f_max"], 0.5, p["f_max"]]])


def test_single_rotor_torque_signs():
    """Physical sign pins of Eq. (3): a right-side rotor rolls left-side-down (tau_x < 0), a front rotor pitches nose up (tau_y < 0)."""
    p = _p()
    r, _ = dyn.rotor_layout(p)
    for i in range(4):
        f = np.zeros((1, 4))
        f[0, i] = 1.0
        force, torque = dyn.wrench(f, p)
        assert force[0, 2] == 1.0 and force[0, 0] == 0 and force[0, 1] == 0
        assert np.sign(torque[0, 0]) == np.sign(r[i, 1])        # rotor at +y lifts the left side
        assert np.sign(torque[0, 1]) == -np.sign(r[i, 0])       # rotor at +x lifts the nose
    # geometry: the arm length is the distance of every rotor from the centre
    assert np.allclose(np.linalg.norm(r, axis=1), p["arm"])


def test_yaw_reaction_and_roll_from_srt():
    """Spin pair (+1) faster than the (-1) pair -> positive yaw acceleration, no roll/pitch."""
    p = _p(ctrl=dyn.SRT)
    s = make_states([[0, 0, 5.0]], p).astype(np.float64)
    f = np.array([[3.0, 3.0, 2.0, 2.0]])
    s[0, 13:17] = np.sqrt(f[0])
    out = dyn.step(s, f, p)
    assert out[0, 12] > 0
    assert abs(out[0, 10]) < 1e-12 and abs(out[0, 11]) < 1e-12
    # yaw acceleration magnitude: kappa * (3+3-2-2) / Jz integrated over one step (rotors constant)
    assert np.isclose(out[0, 12], p["kappa_yaw"] * 2.0 / p["J"][2] * p["dt"], rtol=1e-12)


def test_ctbr_tracks_rate_command():
    """CTBR: a constant, feasible rate command is tracked (the rate loop is stable)."""
    p = _p()
    s = make_states([[0, 0, 5.0]], p).astype(np.float64)
    om_des = np.array([0.5, -0.3, 0.8])
    a = np.array([[p["g"], *om_des]])
    for _ in range(100):
        s = dyn.step(s, a, p)
    assert np.allclose(s[0, 10:13], om_des, atol=2e-3)


def test_ctbr_collective_thrust_vertical_acceleration():
    """CTBR with c = 1.5 g at level attitude: the commanded rotor thrusts sum to 1.5 m g."""
    p = _p()
    s = make_states([[0, 0, 5.0]], p).astype(np.float64)
    f = dyn.controller(s, np.array([[1.5 * p["g"], 0, 0, 0]]), p)
    assert np.isclose(f.sum(), 1.5 * p["mass"] * p["g"], rtol=1e-14)
    assert np.allclose(f, f[0, 0])


def test_quaternion_stays_unit_and_rotation_convention():
    p = _p()
    rng = np.random.default_rng(0)
    s = make_states(rng.uniform(-1, 1, (8, 3)), p, quat=yaw_quat(rng.uniform(-3, 3, 8))).astype(np.float64)
    for _ in range(50):
        a = np.concatenate([rng.uniform(0.5, 2, (8, 1)) * p["g"], rng.uniform(-3, 3, (8, 3))], axis=1)
        s = dyn.step(s, a, p)
    assert np.allclose(np.linalg.norm(s[:, 3:7], axis=1), 1.0, atol=1e-15)
    # R(q) of a yaw by +90 deg maps body x onto world y
    rot = dyn.quat_to_rot(yaw_quat(np.array([math.pi / 2])))[0]
    assert np.allclose(rot @ [1, 0, 0], [0, 1, 0], atol=1e-15)
    # R is orthonormal with det +1 for a random unit quaternion, and R(q1 q2) = R(q1) R(q2)
    q1 = rng.normal(size=4); q1 /= np.linalg.norm(q1)
    q2 = rng.normal(size=4); q2 /= np.linalg.norm(q2)
    r1, r2 = dyn.quat_to_rot(q1), dyn.quat_to_rot(q2)
    assert np.allclose(r1 @ r1.T, np.eye(3), atol=1e-14) and np.isclose(np.linalg.det(r1), 1.0)
    assert np.allclose(dyn.quat_to_rot(dyn.quat_mul(q1, q2)), r1 @ r2, atol=1e-14)


def test_body_rate_integrates_in_body_frame():
    """q_dot = 1/2 q (x) Omega uses body rates: after a yaw of +90 deg, a body-x rate turns about world +y."""
    p = _p(ctrl=dyn.SRT)
    f = hover_rotor(p) ** 2
    s = make_states([[0, 0, 5.0]], p, quat=yaw_quat([math.pi / 2]), omega=[[0.5, 0, 0]]).astype(np.float64)
    for _ in range(10):
        s = dyn.step(s, np.full((1, 4), f), p)
    rot = dyn.quat_to_rot(s[0, 3:7])
    angle = 0.5 * 10 * p["dt"]
    # a positive turn about world +y carries world z to (sin a, 0, cos a)
    assert np.allclose(rot[:, 2], [math.sin(angle), 0.0, math.cos(angle)], atol=1e-9)


def test_euler_free_fall_closed_form():
    """Explicit Euler: v exact, p_n = p0 + v0 t_n - g h^2 n(n-1)/2."""
    p = _p(ctrl=dyn.SRT, k_lin=(0.0, 0.0, 0.0), integrator=dyn.EULER)
    v0 = np.array([1.0, 0.0, 2.0])
    s = make_states([[0, 0, 0.0]], p, vel=[v0], rotor=[[0, 0, 0, 0]]).astype(np.float64)
    h = p["dt"]
    for n in range(1, 21):
        s = dyn.step(s, np.zeros((1, 4)), p)
        assert np.allclose(s[0, 0:3], v0 * n * h - np.array([0, 0, 1.0]) * p["g"] * h * h * n * (n - 1) / 2, atol=1e-12)


def test_substeps_free_fall_exact():
    p = _p(ctrl=dyn.SRT, k_lin=(0.0, 0.0, 0.0), n_sub=4)
    s = make_states([[0, 0, 0.0]], p, rotor=[[0, 0, 0, 0]]).astype(np.float64)
    for _ in range(10):
        s = dyn.step(s, np.zeros((1, 4)), p)
    t = 10 * p["dt"]
    assert np.isclose(s[0, 2], -0.5 * p["g"] * t * t, atol=1e-12)


@pytest.mark.parametrize("n_sub", [1, 4])
def test_rk4_convergence_order(n_sub):
    """RK4 global error shrinks ~16x when the step halves (SRT with a constant command: a smooth ODE)."""
    base = _p(n_sub=n_sub, ctrl=dyn.SRT)
    s0 = make_states([[0, 0, 5.0]], base, omega=[[0.3, -0.2, 0.4]], vel=[[1.0, 0.5, -0.2]]).astype(np.float64)
    a = np.array([[2.2, 2.9, 3.1, 2.4]])

    def run(dt, steps):
        p = _p(dt=dt, n_sub=n_sub, ctrl=dyn.SRT)
        s = s0.copy()
        for _ in range(steps):
            s = dyn.step(s, a, p)
        return s

    ref = run(0.0025, 160)
    e1 = np.abs(run(0.02, 20) - ref)[0, :13].max()
    e2 = np.abs(run(0.01, 40) - ref)[0, :13].max()
    assert 12.0 < e1 / e2 < 20.0


# ---------------------------------------------------------------------------
# quadratic drag (Eq. 2, the c_quad term, read as -c |v_B| v_B per body axis)
# ---------------------------------------------------------------------------

def _drag_run(p, s, steps):
    out = [s.copy()]
    for _ in range(steps):
        s = dyn.step(s, np.zeros((1, 4)), p)
        out.append(s.copy())
    return np.stack(out)


@pytest.mark.parametrize("c", [0.05, 0.2])
def test_quadratic_drag_vertical_fall_tanh(c):
    """Level attitude, rotors off, no linear drag: a fall from rest obeys v' = -g + (c/m) v^2, so
    v(t) = -sqrt(m g / c) tanh(t sqrt(g c / m)) and the speed approaches the terminal sqrt(m g / c).
    RK4 follows it within its global error, which falls ~16x when the step halves."""
    m = 1.0
    g = 9.81
    p = _p(ctrl=dyn.SRT, k_lin=(0.0, 0.0, 0.0), c_quad=(c, c, c), mass=m)
    s0 = make_states([[0.0, 0.0, 100.0]], p, rotor=[[0, 0, 0, 0]], quat=yaw_quat([0.3])).astype(np.float64)
    v_term = math.sqrt(m * g / c)
    rate = math.sqrt(g * c / m)

    def err(dt, steps):
        pp = dict(p, dt=dt)
        tr = _drag_run(pp, s0.copy(), steps)
        t = np.arange(steps + 1) * dt
        exact = -v_term * np.tanh(t * rate)
        assert np.allclose(tr[:, 0, 7:9], 0.0, atol=1e-14)       # the fall stays vertical
        return np.abs(tr[:, 0, 9] - exact).max(), tr
    e1, tr = err(0.02, 400)
    e2, _ = err(0.01, 800)
    assert e1 < 1e-6 * v_term, f"RK4 error {e1:.3e}"
    assert 12.0 < e1 / e2 < 20.0, f"error ratio {e1 / e2:.2f}"
    # after 8 s (several time constants) the speed is within 1e-3 of the terminal speed
    assert abs(-tr[-1, 0, 9] - v_term) < 1e-3 * v_term
    # position: integral of v, -(v_term / rate) log cosh(rate t)
    t_end = 400 * 0.02
    z_exact = 100.0 - v_term / rate * math.log(math.cosh(rate * t_end))
    assert abs(tr[-1, 0, 2] - z_exact) < 1e-5 * v_term * t_end


@pytest.mark.parametrize("yaw,factor", [(0.0, 1.0), (math.pi / 4, 1.0 / math.sqrt(2.0))])
def test_quadratic_drag_is_per_body_axis(yaw, factor):
    """No gravity, rotors off, velocity v0 along world x: with yaw 0 the body x axis carries all of it and
    v' = -(c/m) v^2; with yaw 45 deg it splits equally over body x and y, the two drag components
    -c (v/sqrt2)|v/sqrt2| and +c (v/sqrt2)|v/sqrt2| turn back onto world x, and v' = -(c/(sqrt2 m)) v^2.
    Either way v(t) = v0 / (1 + k v0 t) with k = factor c / m, and the motion stays on world x.
    A transposed rotation, a dropped |v_B| or a sign slip breaks one of the two cases."""
    c, m, v0 = 0.1, 0.8, 12.0
    p = _p(ctrl=dyn.SRT, k_lin=(0.0, 0.0, 0.0), c_quad=(c, c, c), mass=m, g=0.0)
    s = make_states([[0.0, 0.0, 0.0]], p, rotor=[[0, 0, 0, 0]], vel=[[v0, 0.0, 0.0]],
                    quat=yaw_quat([yaw])).astype(np.float64)
    tr = _drag_run(p, s, 200)
    k = factor * c / m
    t = np.arange(201) * p["dt"]
    exact = v0 / (1.0 + k * v0 * t)
    assert np.abs(tr[:, 0, 7] - exact).max() < 1e-6 * v0
    # off-track velocity only from the float32 rounding of the yaw quaternion (a transposed rotation would
    # turn the drag of the 45 degree case onto world y, at the scale of v0)
    assert np.abs(tr[:, 0, 8:10]).max() < 1e-7 * v0
    # position: x(t) = log(1 + k v0 t) / k
    assert abs(tr[-1, 0, 0] - math.log(1 + k * v0 * t[-1]) / k) < 1e-5 * v0


def test_quadratic_drag_anisotropic_coefficients():
    """Drift along body y with c_quad = (0, c, 0) decelerates as v0 / (1 + (c/m) v0 t); the same drift
    along body x feels no drag at all (its coefficient is 0): each body axis has its own coefficient."""
    c, m = 0.3, 1.0
    p = _p(ctrl=dyn.SRT, k_lin=(0.0, 0.0, 0.0), c_quad=(0.0, c, 0.0), mass=m, g=0.0)
    rot90 = yaw_quat([math.pi / 2])        # body y = world -x, body x = world y
    s = make_states([[0, 0, 0.0]], p, rotor=[[0, 0, 0, 0]], vel=[[-5.0, 3.0, 0.0]], quat=rot90).astype(np.float64)
    tr = _drag_run(p, s, 100)
    t = np.arange(101) * p["dt"]
    v_by = 5.0 / (1 + c / m * 5.0 * t)      # speed along body y (world -x)
    assert np.abs(-tr[:, 0, 7] - v_by).max() < 1e-6 * 5
    assert np.allclose(tr[:, 0, 8], 3.0, atol=1e-12)     # world y = body x: no drag
