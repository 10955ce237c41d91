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
//
// The functions are templates on the arithmetic type.  A control step (dyn_step)
// reads the float32 state, runs every sub-step in FP64 and rounds the new state to
// float32 once, so a step adds one rounding of the stored state and nothing else of
// note.  Every expression is evaluated as written (no multiply-add contraction), so
// every kernel that steps agents -- the dynamics kernel, the fused render, the
// server's batches -- computes the same bits.  The adjoint (grad.hip) recomputes the
// same FP64 sub-steps and linearises them in FP64 too: in reverse mode by hand for
// CTBR and SRT, and for PS and LV by running dyn_substep itself on dual numbers.
#pragma once

#include "vf_internal.h"

namespace vf {

template <typename T>
struct Vec13T {
    T p[3], q[4], v[3], w[3];
};
using Vec13 = Vec13T<float>;

__device__ __forceinline__ float vsqrt(float x) { return sqrtf(x); }
__device__ __forceinline__ double vsqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float vabs(float x) { return fabsf(x); }
__device__ __forceinline__ double vabs(double x) { return fabs(x); }
__device__ __forceinline__ float vmin(float a, float b) { return fminf(a, b); }
__device__ __forceinline__ double vmin(double a, double b) { return fmin(a, b); }
__device__ __forceinline__ float vmax(float a, float b) { return fmaxf(a, b); }
__device__ __forceinline__ double vmax(double a, double b) { return fmax(a, b); }
__device__ __forceinline__ void vsincos(float x, float* s, float* c) { sincosf(x, s, c); }
__device__ __forceinline__ void vsincos(double x, double* s, double* c) { sincos(x, s, c); }

// Rotor thrusts -> body force z and body torque (Eq. 3 + yaw reaction).
template <typename T>
__device__ __forceinline__ void rotor_wrench(const DynConstT<T>& c, const T f[4], T& fz, T tau[3]) {
#pragma clang fp contract(off)
    fz = (f[0] + f[1]) + (f[2] + f[3]);
    tau[0] = c.arm_a * ((f[1] + f[2]) - (f[0] + f[3]));
    tau[1] = c.arm_a * ((f[1] + f[3]) - (f[0] + f[2]));
    tau[2] = c.kappa * ((f[0] + f[1]) - (f[2] + f[3]));
}

// R(q/|q|) as 9 values, row major (the dynamics' rotation).
template <typename T>
__device__ __forceinline__ void body_rot(const T q[4], T r[9]) {
#pragma clang fp contract(off)
    const T inv = T(1) / vsqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    const T w = q[0] * inv, x = q[1] * inv, y = q[2] * inv, z = q[3] * inv;
    const T xx = x * x, yy = y * y, zz = z * z, xy = x * y, xz = x * z, yz = y * z, wx = w * x, wy = w * y,
            wz = w * z;
    r[0] = T(1) - T(2) * (yy + zz); r[1] = T(2) * (xy - wz);        r[2] = T(2) * (xz + wy);
    r[3] = T(2) * (xy + wz);        r[4] = T(1) - T(2) * (xx + zz); r[5] = T(2) * (yz - wx);
    r[6] = T(2) * (xz - wy);        r[7] = T(2) * (yz + wx);        r[8] = T(1) - T(2) * (xx + yy);
}

// R(q/|q|) in float32 as 9 floats, row major (cameras, swarm boxes, the depth adjoint).
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
template <typename T>
__device__ __forceinline__ void derivative(const DynConstT<T>& c, const Vec13T<T>& y, const T w[4], Vec13T<T>& d) {
#pragma clang fp contract(off)
    const T f[4] = {w[0] * w[0], w[1] * w[1], w[2] * w[2], w[3] * w[3]};
    T fz, tau[3];
    rotor_wrench(c, f, fz, tau);
    T r[9];
    body_rot(y.q, r);
    // body-frame velocity v_B = R^T v and drag (Eq. 2, signed)
    T vb[3];
    for (int i = 0; i < 3; ++i) vb[i] = r[0 + i] * y.v[0] + r[3 + i] * y.v[1] + r[6 + i] * y.v[2];
    T fb[3];
    for (int i = 0; i < 3; ++i) fb[i] = -c.k_lin[i] * vb[i] - c.c_quad[i] * vabs(vb[i]) * vb[i];
    fb[2] += fz;
    for (int i = 0; i < 3; ++i) {
        d.p[i] = y.v[i];
        d.v[i] = (r[3 * i] * fb[0] + r[3 * i + 1] * fb[1] + r[3 * i + 2] * fb[2]) * c.inv_mass;
    }
    d.v[2] -= c.g;
    // q_dot = 1/2 q (x) (0, Omega)
    const T* q = y.q;
    const T* om = y.w;
    d.q[0] = T(0.5) * (-q[1] * om[0] - q[2] * om[1] - q[3] * om[2]);
    d.q[1] = T(0.5) * (q[0] * om[0] + q[2] * om[2] - q[3] * om[1]);
    d.q[2] = T(0.5) * (q[0] * om[1] - q[1] * om[2] + q[3] * om[0]);
    d.q[3] = T(0.5) * (q[0] * om[2] + q[1] * om[1] - q[2] * om[0]);
    // Omega_dot = J^-1 (tau - Omega x J Omega)
    const T jo[3] = {c.J[0] * om[0], c.J[1] * om[1], c.J[2] * om[2]};
    const T cx = om[1] * jo[2] - om[2] * jo[1];
    const T cy = om[2] * jo[0] - om[0] * jo[2];
    const T cz = om[0] * jo[1] - om[1] * jo[0];
    d.w[0] = (tau[0] - cx) * c.inv_J[0];
    d.w[1] = (tau[1] - cy) * c.inv_J[1];
    d.w[2] = (tau[2] - cz) * c.inv_J[2];
}

// PS / LV outer loop (geometric control on SE(3), cascaded onto the rate loop):
// commanded acceleration -> thrust direction b3 (lift at least g/4, tilt at most
// max_tilt) -> R_d = [b1 b2 b3] with b2 = b3 x heading(yaw_d) normalised ->
// collective c = F . R e_z and rate command Omega_des = -k_att e_R,
// e_R = 1/2 (R_d^T R - R^T R_d)^vee.
template <typename T>
__device__ __forceinline__ void outer_loop(const DynConstT<T>& c, const T s[17], const T a[4], T& cc, T om_des[3]) {
#pragma clang fp contract(off)
    T f[3];
    if (c.ctrl == VF_PS) {
        for (int i = 0; i < 3; ++i) f[i] = -c.k_pos[i] * (s[i] - a[i]) - c.k_vel[i] * s[7 + i];
    } else {
        for (int i = 0; i < 3; ++i) f[i] = -c.k_vel[i] * (s[7 + i] - a[i]);
    }
    f[2] = vmax(f[2] + c.g, c.min_lift);
    const T hz = vsqrt(f[0] * f[0] + f[1] * f[1]);
    const T lim = f[2] * c.tan_tilt;
    if (hz > lim) {
        const T sc = lim / hz;
        f[0] *= sc;
        f[1] *= sc;
    }
    const T inv = T(1) / vsqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
    const T b3[3] = {f[0] * inv, f[1] * inv, f[2] * inv};
    T sp, cp;
    vsincos(a[3], &sp, &cp);
    // b3 x (cos, sin, 0); its norm is at least b3_z > 0
    T b2[3] = {-b3[2] * sp, b3[2] * cp, b3[0] * sp - b3[1] * cp};
    const T in2 = T(1) / vsqrt(b2[0] * b2[0] + b2[1] * b2[1] + b2[2] * b2[2]);
    for (int i = 0; i < 3; ++i) b2[i] *= in2;
    const T b1[3] = {b2[1] * b3[2] - b2[2] * b3[1], b2[2] * b3[0] - b2[0] * b3[2], b2[0] * b3[1] - b2[1] * b3[0]};
    T r[9];
    body_rot(s + 3, r);
    cc = f[0] * r[2] + f[1] * r[5] + f[2] * r[8];
    // M = R_d^T R: M_ij = b_i . (column j of R)
    auto dotc = [&](const T b[3], int j) { return b[0] * r[j] + b[1] * r[3 + j] + b[2] * r[6 + j]; };
    const T m21 = dotc(b3, 1), m12 = dotc(b2, 2), m02 = dotc(b1, 2), m20 = dotc(b3, 0), m10 = dotc(b2, 0),
            m01 = dotc(b1, 1);
    om_des[0] = -c.k_att[0] * T(0.5) * (m21 - m12);
    om_des[1] = -c.k_att[1] * T(0.5) * (m02 - m20);
    om_des[2] = -c.k_att[2] * T(0.5) * (m10 - m01);
}

// Desired rotor thrusts (clamped) from the action at the sub-step start.
template <typename T>
__device__ __forceinline__ void controller(const DynConstT<T>& c, const T s[17], const T a[4], T f[4]) {
#pragma clang fp contract(off)
    if (c.ctrl == VF_SRT) {
        for (int i = 0; i < 4; ++i) f[i] = a[i];
    } else {
        T cmd[4] = {a[0], a[1], a[2], a[3]};
        if (c.ctrl == VF_PS || c.ctrl == VF_LV) outer_loop(c, s, a, cmd[0], cmd + 1);
        const T* om = s + 10;
        const T jo[3] = {c.J[0] * om[0], c.J[1] * om[1], c.J[2] * om[2]};
        const T t0 = c.kJ[0] * (cmd[1] - om[0]) + (om[1] * jo[2] - om[2] * jo[1]);
        const T t1 = c.kJ[1] * (cmd[2] - om[1]) + (om[2] * jo[0] - om[0] * jo[2]);
        const T t2 = c.kJ[2] * (cmd[3] - om[2]) + (om[0] * jo[1] - om[1] * jo[0]);
        const T u0 = c.mass * cmd[0], u1 = t0 * c.inv_a, u2 = t1 * c.inv_a, u3 = t2 * c.inv_kappa;
        f[0] = T(0.25) * ((u0 + u3) - (u1 + u2));
        f[1] = T(0.25) * ((u0 + u3) + (u1 + u2));
        f[2] = T(0.25) * ((u0 - u3) + (u1 - u2));
        f[3] = T(0.25) * ((u0 - u3) - (u1 - u2));
    }
    for (int i = 0; i < 4; ++i) f[i] = vmin(vmax(f[i], T(0)), c.f_max);
}

template <typename T>
__device__ __forceinline__ void axpy13(Vec13T<T>& o, const Vec13T<T>& y, T h, const Vec13T<T>& k) {
#pragma clang fp contract(off)
    for (int i = 0; i < 3; ++i) o.p[i] = y.p[i] + h * k.p[i];
    for (int i = 0; i < 4; ++i) o.q[i] = y.q[i] + h * k.q[i];
    for (int i = 0; i < 3; ++i) o.v[i] = y.v[i] + h * k.v[i];
    for (int i = 0; i < 3; ++i) o.w[i] = y.w[i] + h * k.w[i];
}

// One sub-step of length c.h: s (17) and the held action a (4) -> s, in place.  The control step runs it in
// FP64; the forward-mode adjoint runs it on dual numbers, whose values take the same operations.
template <typename T>
__device__ __forceinline__ void dyn_substep(const DynConstT<T>& c, T s[17], const T a[4]) {
#pragma clang fp contract(off)
    T fdes[4], wd[4], w0[4], wh[4], wf[4];
    controller(c, s, a, fdes);
    for (int i = 0; i < 4; ++i) {
        wd[i] = vsqrt(fdes[i]);
        w0[i] = s[13 + i];
        wh[i] = wd[i] + (w0[i] - wd[i]) * c.e_half;
        wf[i] = wd[i] + (w0[i] - wd[i]) * c.e_full;
    }
    Vec13T<T> y;
    for (int i = 0; i < 3; ++i) { y.p[i] = s[i]; y.v[i] = s[7 + i]; y.w[i] = s[10 + i]; }
    for (int i = 0; i < 4; ++i) y.q[i] = s[3 + i];
    Vec13T<T> k1, k2, k3, k4, t;
    const T h = c.h;
    derivative(c, y, w0, k1);
    if (c.integrator == VF_EULER) {
        axpy13(y, y, h, k1);
    } else {
        axpy13(t, y, T(0.5) * h, k1);
        derivative(c, t, wh, k2);
        axpy13(t, y, T(0.5) * h, k2);
        derivative(c, t, wh, k3);
        axpy13(t, y, h, k3);
        derivative(c, t, wf, k4);
        const T h6 = h / T(6);
        for (int i = 0; i < 3; ++i) {
            y.p[i] += h6 * (k1.p[i] + T(2) * (k2.p[i] + k3.p[i]) + k4.p[i]);
            y.v[i] += h6 * (k1.v[i] + T(2) * (k2.v[i] + k3.v[i]) + k4.v[i]);
            y.w[i] += h6 * (k1.w[i] + T(2) * (k2.w[i] + k3.w[i]) + k4.w[i]);
        }
        for (int i = 0; i < 4; ++i) y.q[i] += h6 * (k1.q[i] + T(2) * (k2.q[i] + k3.q[i]) + k4.q[i]);
    }
    const T inv = T(1) / vsqrt(y.q[0] * y.q[0] + y.q[1] * y.q[1] + y.q[2] * y.q[2] + y.q[3] * y.q[3]);
    for (int i = 0; i < 3; ++i) { s[i] = y.p[i]; s[7 + i] = y.v[i]; s[10 + i] = y.w[i]; }
    for (int i = 0; i < 4; ++i) { s[3 + i] = y.q[i] * inv; s[13 + i] = wf[i]; }
}

// One control step of one agent: s (17 float32, in) -> o (17 float32, out), all sub-steps in FP64 and
// one rounding at the end.  o may alias s_in.
__device__ __forceinline__ void dyn_step(const DynConstD& c, const float s_in[17], const float a_in[4], float o[17]) {
    double s[17], a[4];
    for (int i = 0; i < 17; ++i) s[i] = (double)s_in[i];
    for (int i = 0; i < 4; ++i) a[i] = (double)a_in[i];
    for (int sub = 0; sub < c.n_sub; ++sub) dyn_substep(c, s, a);
    for (int i = 0; i < 17; ++i) o[i] = (float)s[i];
}

}  // namespace vf
