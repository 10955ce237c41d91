"""FP64 quadrotor dynamics (Sec. III-A, Eqs. 1-4), vectorised over agents with NumPy.

State row (17): p(3) world position, q(4) quaternion (w,x,y,z) body->world,
v(3) world velocity, Omega(3) body rates, w(4) normalised rotor speeds.

Readings of the passages the paper leaves open:
  * Eq. (2) as printed is never negative, so it cannot oppose motion; the drag
    used is d = -k_lin (.) v_B - c_quad (.) |v_B| (.) v_B in the body frame
    (element-wise), with the benchmark's linear coefficient and c_quad = 0.
  * Eq. (3) has no yaw term for vertical thrusts; a rotor reaction torque
    kappa * s_i * f_i about body z is added.  T_i is read as the rotor position
    r_i of an X frame: arm l at +-45 deg,
        r = l/sqrt(2) * {(+1,-1), (-1,+1), (+1,+1), (-1,-1)},  s = (+1,+1,-1,-1).
  * Eq. (4) with k1 = k0 = 0: the state stores w_i = sqrt(k2) * omega_i, so the
    rotor thrust is w_i^2; c = 1 / tau_motor and t is the time since the start
    of the sub-step, the commanded speed being held over the sub-step.
  * CTBR (controller paragraph of Sec. III-A): action = (c [m/s^2], Omega_des);
    F = m c,  tau = J K (Omega_des - Omega) + Omega x J Omega; rotor thrusts
    solve the 4x4 allocation [F; tau] = A f and are clamped to [0, f_max].
    SRT: the action is the four rotor thrusts, clamped the same way.
  * Eq. (1): q_dot = 1/2 q (x) (0, Omega) with the Hamilton product, R from the
    normalised q; gravity (0, 0, -g).  After every sub-step q is normalised.
  * PS and LV (same paragraph; geometric control after Lee, Leok and McClamroch,
    CDC 2010, cascaded onto the CTBR rate loop):
        PS action (x_d, y_d, z_d, psi_d):  a = -K_p (p - p_d) - K_v v
        LV action (vx_d, vy_d, vz_d, psi_d): a = -K_v (v - v_d)
        F = a + g e_z, its vertical part raised to at least g/4 and its
        horizontal part shortened so the tilt of F stays within max_tilt;
        b3 = F/|F|, b2 = b3 x (cos psi_d, sin psi_d, 0) normalised, b1 = b2 x b3,
        R_d = [b1 b2 b3];  c = F . R e_z;  e_R = 1/2 (R_d^T R - R^T R_d)^vee;
        Omega_des = -K_R e_R, then the CTBR law with (c, Omega_des).
"""
import numpy as np

RK4 = 0
EULER = 1
CTBR = 0
SRT = 1
PS = 2
LV = 3
MIN_LIFT = 0.25     # vertical part of the commanded acceleration at least MIN_LIFT * g


def quat_mul(a, b):
    """Hamilton product a (x) b of scalar-first quaternions, [...,4]."""
    aw, ax, ay, az = a[..., 0], a[..., 1], a[..., 2], a[..., 3]
    bw, bx, by, bz = b[..., 0], b[..., 1], b[..., 2], b[..., 3]
    return np.stack([
        aw * bw - ax * bx - ay * by - az * bz,
        aw * bx + ax * bw + ay * bz - az * by,
        aw * by - ax * bz + ay * bw + az * bx,
        aw * bz + ax * by - ay * bx + az * bw,
    ], axis=-1)


def quat_to_rot(q):
    """Rotation matrix R_WB of a unit quaternion (w,x,y,z): v_W = R v_B.  [...,3,3]"""
    w, x, y, z = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    r = np.empty(q.shape[:-1] + (3, 3))
    r[..., 0, 0] = 1 - 2 * (y * y + z * z)
    r[..., 0, 1] = 2 * (x * y - w * z)
    r[..., 0, 2] = 2 * (x * z + w * y)
    r[..., 1, 0] = 2 * (x * y + w * z)
    r[..., 1, 1] = 1 - 2 * (x * x + z * z)
    r[..., 1, 2] = 2 * (y * z - w * x)
    r[..., 2, 0] = 2 * (x * z - w * y)
    r[..., 2, 1] = 2 * (y * z + w * x)
    r[..., 2, 2] = 1 - 2 * (x * x + y * y)
    return r


def rotor_layout(params):
    """Rotor positions r_i (body frame, [4,3]) and spin signs s_i ([4]) of the X frame."""
    a = params["arm"] / np.sqrt(2.0)
    r = np.array([[a, -a, 0.0], [-a, a, 0.0], [a, a, 0.0], [-a, -a, 0.0]])
    s = np.array([1.0, 1.0, -1.0, -1.0])
    return r, s


def wrench(f, params):
    """Eq. (3) plus yaw reaction: body force (0,0,sum f_i) and torque sum r_i x f_i e_z + kappa s_i f_i e_z."""
    r, s = rotor_layout(params)
    n = f.shape[0]
    force = np.zeros((n, 3))
    force[:, 2] = f.sum(axis=1)
    fz = np.zeros((n, 4, 3))
    fz[:, :, 2] = f
    torque = np.cross(np.broadcast_to(r, fz.shape), fz).sum(axis=1)
    torque[:, 2] += params["kappa_yaw"] * (f * s).sum(axis=1)
    return force, torque


def allocation_matrix(params):
    """A with [F, tau_x, tau_y, tau_z] = A f, read off the wrench of unit rotor thrusts."""
    a = np.empty((4, 4))
    for i in range(4):
        e = np.zeros((1, 4))
        e[0, i] = 1.0
        force, torque = wrench(e, params)
        a[:, i] = [force[0, 2], torque[0, 0], torque[0, 1], torque[0, 2]]
    return a


def vee(m):
    """The vector of a skew-symmetric matrix: vee([w]_x) = w.  [...,3,3] -> [...,3]"""
    return np.stack([m[..., 2, 1], m[..., 0, 2], m[..., 1, 0]], axis=-1)


def outer_loop(state, action, params):
    """PS / LV: collective acceleration c [N] and body-rate command Omega_des [N,3] for the rate loop."""
    p, q, v = state[:, 0:3], state[:, 3:7], state[:, 7:10]
    rot = quat_to_rot(q / np.linalg.norm(q, axis=1, keepdims=True))
    kp = np.asarray(params["k_pos"], dtype=np.float64)
    kv = np.asarray(params["k_vel"], dtype=np.float64)
    ka = np.asarray(params["k_att"], dtype=np.float64)
    g = params["g"]
    if params["ctrl"] == PS:
        acc = -kp * (p - action[:, 0:3]) - kv * v
    else:
        acc = -kv * (v - action[:, 0:3])
    f = acc + np.array([0.0, 0.0, g])
    f[:, 2] = np.maximum(f[:, 2], MIN_LIFT * g)
    horiz = np.hypot(f[:, 0], f[:, 1])
    limit = f[:, 2] * np.tan(params["max_tilt"])
    scale = np.where(horiz > limit, limit / np.where(horiz > 0, horiz, 1.0), 1.0)
    f[:, 0:2] *= scale[:, None]
    b3 = f / np.linalg.norm(f, axis=1, keepdims=True)
    psi = action[:, 3]
    heading = np.stack([np.cos(psi), np.sin(psi), np.zeros_like(psi)], axis=1)
    b2 = np.cross(b3, heading)
    b2 /= np.linalg.norm(b2, axis=1, keepdims=True)
    b1 = np.cross(b2, b3)
    rd = np.stack([b1, b2, b3], axis=2)                      # columns b1, b2, b3
    c = np.einsum("ni,ni->n", f, rot[:, :, 2])
    rdt_r = np.einsum("nji,njk->nik", rd, rot)
    e_r = 0.5 * vee(rdt_r - np.swapaxes(rdt_r, 1, 2))
    return c, -ka * e_r


def controller(state, action, params):
    """Desired rotor thrusts f_des [N,4] from CTBR, SRT, PS or LV commands (held over a sub-step)."""
    f_max = params["f_max"]
    if params["ctrl"] == SRT:
        return np.clip(action.astype(np.float64), 0.0, f_max)
    jd = np.asarray(params["J"], dtype=np.float64)
    kr = np.asarray(params["k_rate"], dtype=np.float64)
    om = state[:, 10:13]
    if params["ctrl"] in (PS, LV):
        c, om_des = outer_loop(state, action, params)
    else:
        c = action[:, 0]
        om_des = action[:, 1:4]
    force = params["mass"] * c
    torque = jd * kr * (om_des - om) + np.cross(om, jd * om)
    rhs = np.concatenate([force[:, None], torque], axis=1)
    a = allocation_matrix(params)
    f = np.linalg.solve(np.broadcast_to(a, (rhs.shape[0], 4, 4)), rhs[:, :, None])[:, :, 0]
    return np.clip(f, 0.0, f_max)


def rotor_speed(w0, w_des, tau, params):
    """Eq. (4): w(tau) = w_des + (w0 - w_des) exp(-tau / tau_motor)."""
    return w_des + (w0 - w_des) * np.exp(-tau / params["tau_motor"])


def derivative(y, w, params):
    """Eq. (1) right-hand side for y = (p, q, v, Omega) [N,13] at rotor speeds w [N,4]."""
    q = y[:, 3:7]
    v = y[:, 7:10]
    om = y[:, 10:13]
    jd = np.asarray(params["J"], dtype=np.float64)
    k_lin = np.asarray(params["k_lin"], dtype=np.float64)
    c_quad = np.asarray(params["c_quad"], dtype=np.float64)
    force, torque = wrench(w * w, params)
    qn = q / np.linalg.norm(q, axis=1, keepdims=True)
    rot = quat_to_rot(qn)
    v_b = np.einsum("nji,nj->ni", rot, v)                      # R^T v
    drag = -k_lin * v_b - c_quad * np.abs(v_b) * v_b           # Eq. (2), signed
    acc = np.einsum("nij,nj->ni", rot, force + drag) / params["mass"]
    acc[:, 2] -= params["g"]
    om_quat = np.concatenate([np.zeros((y.shape[0], 1)), om], axis=1)
    qdot = 0.5 * quat_mul(q, om_quat)
    omdot = (torque - np.cross(om, jd * om)) / jd
    return np.concatenate([v, qdot, acc, omdot], axis=1)


def substep(state, action, params, h):
    """One sub-step of length h: controller (zero-order hold), rotor lag, RK4 or Euler, normalise q."""
    f_des = controller(state, action, params)
    w_des = np.sqrt(f_des)
    w0 = state[:, 13:17]
    y = state[:, 0:13]
    if params["integrator"] == EULER:
        y_new = y + h * derivative(y, rotor_speed(w0, w_des, 0.0, params), params)
    else:
        k1 = derivative(y, rotor_speed(w0, w_des, 0.0, params), params)
        k2 = derivative(y + 0.5 * h * k1, rotor_speed(w0, w_des, 0.5 * h, params), params)
        k3 = derivative(y + 0.5 * h * k2, rotor_speed(w0, w_des, 0.5 * h, params), params)
        k4 = derivative(y + h * k3, rotor_speed(w0, w_des, h, params), params)
        y_new = y + (h / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
    out = np.empty_like(state)
    out[:, 0:13] = y_new
    out[:, 3:7] /= np.linalg.norm(out[:, 3:7], axis=1, keepdims=True)
    out[:, 13:17] = rotor_speed(w0, w_des, h, params)
    return out


def step(state, action, params):
    """One control step: n_sub sub-steps of dt / n_sub with the same action."""
    s = np.asarray(state, dtype=np.float64)
    a = np.asarray(action, dtype=np.float64)
    h = params["dt"] / params["n_sub"]
    for _ in range(int(params["n_sub"])):
        s = substep(s, a, params, h)
    return s


def rollout(state0, actions, params):
    """States [H+1, N, 17] from s0 and actions [H, N, 4]."""
    out = [np.asarray(state0, dtype=np.float64)]
    for a in actions:
        out.append(step(out[-1], a, params))
    return np.stack(out)
