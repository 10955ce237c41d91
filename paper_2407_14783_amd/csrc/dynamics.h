// Device-side quadrotor dynamics (Sec. III-A): Eq. (1) rigid body, Eq. (2) drag,
// Eq. (3) thrust and moment with a rotor reaction yaw torque, Eq. (4) first-order
// rotor lag, the CTBR, SRT, PS and LV controllers, RK4 or explicit Euler with sub-steps.
//
// Readings of what the paper leaves open (all shared with the oracle's docstring
// by statement, not by code): X frame with rotors at a (1,-1), a (-1,1), a (1,1),
// a (-1,-1), a = arm / sqrt(2), spin signs (+,+,-,-); the allocation inverse is
// the scaled transpose of that +-1 pattern.  Rotor speeds are normalised so the
// thrust of rotor i is w_i^2; the commanded speed is held over a sub-step and
// the lag is evaluated in closed form at the RK4 stage times (e^{-h/2tau},
// e^{-h/tau} come precomputed).  Drag d = -k_lin v_B - c_quad |v_B| v_B in the
// body frame.  q is renormalised after every sub-step.
#pragma once

#include "vf_internal.h"

namespace vf {

struct Vec13 {
    float p[3], q[4], v[3], w[3];
};

// Rotor thrusts -> body force z and body torque (Eq. 3 + yaw reaction).
__device__ __forceinline__ void rotor_wrench(const DynConst& c, const float f[4], float& fz, float tau[3]) {
    fz = (f[0] + f[1]) + (f[2] + f[3]);
    tau[0] = c.arm_a * ((f[1] + f[2]) - (f[0] + f[3]));
    tau[1] = c.arm_a * ((f[1] + f[3]) - (f[0] + f[2]));
    tau[2] = c.kappa * ((f[0] + f[1]) - (f[2] + f[3]));
}

// R(q/|q|) as 9 floats, row major.
__device__ __forceinline__ void quat_rot(const float q[4], float r[9]) {
    float inv = 1.0f / sqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    float w = q[0] * inv, x = q[1] * inv, y = q[2] * inv, z = q[3] * inv;
    float xx = x * x, yy = y * y, zz = z * z, xy = x * y, xz = x * z, yz = y * z, wx = w * x, wy = w * y, wz = w * z;
    r[0] = 1.0f - 2.0f * (yy + zz); r[1] = 2.0f * (xy - wz);        r[2] = 2.0f * (xz + wy);
    r[3] = 2.0f * (xy + wz);        r[4] = 1.0f - 2.0f * (xx + zz); r[5] = 2.0f * (yz - wx);
    r[6] = 2.0f * (xz - wy);        r[7] = 2.0f * (yz + wx);        r[8] = 1.0f - 2.0f * (xx + yy);
}

// Camera pose of a view: origin p + R mount_t and rotation R R(mount_q) (row major).
// A mount quaternion with zero vector part is no rotation.
__device__ __forceinline__ void camera_pose(const float pose[17], const vf_view& vw, float o[3], float rc[9]) {
    float r[9];
    quat_rot(pose + 3, r);
    for (int i = 0; i < 3; ++i)
        o[i] = pose[i] + (r[3 * i] * vw.mount_t[0] + r[3 * i + 1] * vw.mount_t[1] + r[3 * i + 2] * vw.mount_t[2]);
    if (vw.mount_q[1] == 0.0f && vw.mount_q[2] == 0.0f && vw.mount_q[3] == 0.0f) {
        for (int i = 0; i < 9; ++i) rc[i] = r[i];
        return;
    }
    float m[9];
    quat_rot(vw.mount_q, m);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) rc[3 * i + j] = r[3 * i] * m[j] + r[3 * i + 1] * m[3 + j] + r[3 * i + 2] * m[6 + j];
}

// Eq. (1) right-hand side at rotor speeds w.
__device__ __forceinline__ void derivative(const DynConst& c, const Vec13& y, const float w[4], Vec13& d) {
    float f[4] = {w[0] * w[0], w[1] * w[1], w[2] * w[2], w[3] * w[3]};
    float fz, tau[3];
    rotor_wrench(c, f, fz, tau);
    float r[9];
    quat_rot(y.q, r);
    // body-frame velocity v_B = R^T v and drag (Eq. 2, signed)
    float vb[3];
    for (int i = 0; i < 3; ++i) vb[i] = r[0 + i] * y.v[0] + r[3 + i] * y.v[1] + r[6 + i] * y.v[2];
    float fb[3];
    for (int i = 0; i < 3; ++i) fb[i] = -c.k_lin[i] * vb[i] - c.c_quad[i] * fabsf(vb[i]) * vb[i];
    fb[2] += fz;
    for (int i = 0; i < 3; ++i) {
        d.p[i] = y.v[i];
        d.v[i] = (r[3 * i] * fb[0] + r[3 * i + 1] * fb[1] + r[3 * i + 2] * fb[2]) * c.inv_mass;
    }
    d.v[2] -= c.g;
    // q_dot = 1/2 q (x) (0, Omega)
    const float* q = y.q;
    const float* om = y.w;
    d.q[0] = 0.5f * (-q[1] * om[0] - q[2] * om[1] - q[3] * om[2]);
    d.q[1] = 0.5f * (q[0] * om[0] + q[2] * om[2] - q[3] * om[1]);
    d.q[2] = 0.5f * (q[0] * om[1] - q[1] * om[2] + q[3] * om[0]);
    d.q[3] = 0.5f * (q[0] * om[2] + q[1] * om[1] - q[2] * om[0]);
    // Omega_dot = J^-1 (tau - Omega x J Omega)
    float jo[3] = {c.J[0] * om[0], c.J[1] * om[1], c.J[2] * om[2]};
    float cx = om[1] * jo[2] - om[2] * jo[1];
    float cy = om[2] * jo[0] - om[0] * jo[2];
    float cz = om[0] * jo[1] - om[1] * jo[0];
    d.w[0] = (tau[0] - cx) * c.inv_J[0];
    d.w[1] = (tau[1] - cy) * c.inv_J[1];
    d.w[2] = (tau[2] - cz) * c.inv_J[2];
}

// PS / LV outer loop (geometric control on SE(3), cascaded onto the rate loop):
// commanded acceleration -> thrust direction b3 (lift at least g/4, tilt at most
// max_tilt) -> R_d = [b1 b2 b3] with b2 = b3 x heading(yaw_d) normalised ->
// collective c = F . R e_z and rate command Omega_des = -k_att e_R,
// e_R = 1/2 (R_d^T R - R^T R_d)^vee.
__device__ __forceinline__ void outer_loop(const DynConst& c, const float s[17], const float a[4], float& cc,
                                           float om_des[3]) {
    float f[3];
    if (c.ctrl == VF_PS) {
        for (int i = 0; i < 3; ++i) f[i] = -c.k_pos[i] * (s[i] - a[i]) - c.k_vel[i] * s[7 + i];
    } else {
        for (int i = 0; i < 3; ++i) f[i] = -c.k_vel[i] * (s[7 + i] - a[i]);
    }
    f[2] = fmaxf(f[2] + c.g, c.min_lift);
    float hz = sqrtf(f[0] * f[0] + f[1] * f[1]);
    float lim = f[2] * c.tan_tilt;
    if (hz > lim) {
        float sc = lim / hz;
        f[0] *= sc;
        f[1] *= sc;
    }
    float inv = 1.0f / sqrtf(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
    float b3[3] = {f[0] * inv, f[1] * inv, f[2] * inv};
    float sp, cp;
    sincosf(a[3], &sp, &cp);
    // b3 x (cos, sin, 0); its norm is at least b3_z > 0
    float b2[3] = {-b3[2] * sp, b3[2] * cp, b3[0] * sp - b3[1] * cp};
    float in2 = 1.0f / sqrtf(b2[0] * b2[0] + b2[1] * b2[1] + b2[2] * b2[2]);
    for (int i = 0; i < 3; ++i) b2[i] *= in2;
    float b1[3] = {b2[1] * b3[2] - b2[2] * b3[1], b2[2] * b3[0] - b2[0] * b3[2], b2[0] * b3[1] - b2[1] * b3[0]};
    float r[9];
    quat_rot(s + 3, r);
    cc = f[0] * r[2] + f[1] * r[5] + f[2] * r[8];
    // M = R_d^T R: M_ij = b_i . (column j of R)
    auto dotc = [&](const float b[3], int j) { return b[0] * r[j] + b[1] * r[3 + j] + b[2] * r[6 + j]; };
    float m21 = dotc(b3, 1), m12 = dotc(b2, 2), m02 = dotc(b1, 2), m20 = dotc(b3, 0), m10 = dotc(b2, 0),
          m01 = dotc(b1, 1);
    om_des[0] = -c.k_att[0] * 0.5f * (m21 - m12);
    om_des[1] = -c.k_att[1] * 0.5f * (m02 - m20);
    om_des[2] = -c.k_att[2] * 0.5f * (m10 - m01);
}

// Desired rotor thrusts (clamped) from the action at the sub-step start.
__device__ __forceinline__ void controller(const DynConst& c, const float s[17], const float a[4], float f[4]) {
    if (c.ctrl == VF_SRT) {
        for (int i = 0; i < 4; ++i) f[i] = a[i];
    } else {
        float cmd[4] = {a[0], a[1], a[2], a[3]};
        if (c.ctrl == VF_PS || c.ctrl == VF_LV) outer_loop(c, s, a, cmd[0], cmd + 1);
        const float* om = s + 10;
        float jo[3] = {c.J[0] * om[0], c.J[1] * om[1], c.J[2] * om[2]};
        float t0 = c.kJ[0] * (cmd[1] - om[0]) + (om[1] * jo[2] - om[2] * jo[1]);
        float t1 = c.kJ[1] * (cmd[2] - om[1]) + (om[2] * jo[0] - om[0] * jo[2]);
        float t2 = c.kJ[2] * (cmd[3] - om[2]) + (om[0] * jo[1] - om[1] * jo[0]);
        float u0 = c.mass * cmd[0], u1 = t0 * c.inv_a, u2 = t1 * c.inv_a, u3 = t2 * c.inv_kappa;
        f[0] = 0.25f * ((u0 + u3) - (u1 + u2));
        f[1] = 0.25f * ((u0 + u3) + (u1 + u2));
        f[2] = 0.25f * ((u0 - u3) + (u1 - u2));
        f[3] = 0.25f * ((u0 - u3) - (u1 - u2));
    }
    for (int i = 0; i < 4; ++i) f[i] = fminf(fmaxf(f[i], 0.0f), c.f_max);
}

__device__ __forceinline__ void axpy13(Vec13& o, const Vec13& y, float h, const Vec13& k) {
    for (int i = 0; i < 3; ++i) o.p[i] = y.p[i] + h * k.p[i];
    for (int i = 0; i < 4; ++i) o.q[i] = y.q[i] + h * k.q[i];
    for (int i = 0; i < 3; ++i) o.v[i] = y.v[i] + h * k.v[i];
    for (int i = 0; i < 3; ++i) o.w[i] = y.w[i] + h * k.w[i];
}

// One control step of one agent: s (17 floats, in) -> o (17 floats, out). o may alias s.
__device__ __forceinline__ void dyn_step(const DynConst& c, const float s_in[17], const float a[4], float o[17]) {
    float s[17];
    for (int i = 0; i < 17; ++i) s[i] = s_in[i];
    for (int sub = 0; sub < c.n_sub; ++sub) {
        float fdes[4], wd[4], w0[4], wh[4], wf[4];
        controller(c, s, a, fdes);
        for (int i = 0; i < 4; ++i) {
            wd[i] = sqrtf(fdes[i]);
            w0[i] = s[13 + i];
            wh[i] = wd[i] + (w0[i] - wd[i]) * c.e_half;
            wf[i] = wd[i] + (w0[i] - wd[i]) * c.e_full;
        }
        Vec13 y;
        for (int i = 0; i < 3; ++i) { y.p[i] = s[i]; y.v[i] = s[7 + i]; y.w[i] = s[10 + i]; }
        for (int i = 0; i < 4; ++i) y.q[i] = s[3 + i];
        Vec13 k1, k2, k3, k4, t;
        const float h = c.h;
        derivative(c, y, w0, k1);
        if (c.integrator == VF_EULER) {
            axpy13(y, y, h, k1);
        } else {
            axpy13(t, y, 0.5f * h, k1);
            derivative(c, t, wh, k2);
            axpy13(t, y, 0.5f * h, k2);
            derivative(c, t, wh, k3);
            axpy13(t, y, h, k3);
            derivative(c, t, wf, k4);
            const float h6 = h * (1.0f / 6.0f);
            for (int i = 0; i < 3; ++i) {
                y.p[i] += h6 * (k1.p[i] + 2.0f * (k2.p[i] + k3.p[i]) + k4.p[i]);
                y.v[i] += h6 * (k1.v[i] + 2.0f * (k2.v[i] + k3.v[i]) + k4.v[i]);
                y.w[i] += h6 * (k1.w[i] + 2.0f * (k2.w[i] + k3.w[i]) + k4.w[i]);
            }
            for (int i = 0; i < 4; ++i) y.q[i] += h6 * (k1.q[i] + 2.0f * (k2.q[i] + k3.q[i]) + k4.q[i]);
        }
        float inv = 1.0f / sqrtf(y.q[0] * y.q[0] + y.q[1] * y.q[1] + y.q[2] * y.q[2] + y.q[3] * y.q[3]);
        for (int i = 0; i < 3; ++i) { s[i] = y.p[i]; s[7 + i] = y.v[i]; s[10 + i] = y.w[i]; }
        for (int i = 0; i < 4; ++i) { s[3 + i] = y.q[i] * inv; s[13 + i] = wf[i]; }
    }
    for (int i = 0; i < 17; ++i) o[i] = s[i];
}

}  // namespace vf
