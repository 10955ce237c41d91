// Adjoint kernels for the differentiable forms (Sec. III-A: differentiable
// dynamics whose analytic gradients drive learning).
//
// k_step_backward: reverse mode of one control step, written out by hand, in FP64
// like the forward step.  The forward sub-steps are recomputed from the saved state
// (for sub-step j the forward runs j sub-steps from the start, so n_sub sub-steps cost
// n_sub(n_sub+1)/2 forward sub-steps; n_sub is small).  Within a sub-step the RK4 stages are
// recomputed and walked backwards: normalisation, the RK4 combination, the four
// stage derivatives (Eq. 1 with Eq. 2 drag and Eq. 3 wrench), the closed-form
// rotor lag (Eq. 4), the square root, the clamp (zero gradient when clamped)
// and the CTBR mixer / rate controller.
//
// k_step_backward_tangent: the same step's Jacobian-transpose product by forward mode (dual numbers
// through the templated FP64 sub-steps), one thread per agent and input coordinate; used for the PS and LV
// controllers.
//
// k_render_backward (in FP64): depth t = n.(V0 - o) / n.d on the hit triangle's plane;
// dt/do = -n / n.d, dt/dd = -t n / n.d, d = R(q/|q|) d_B with d_B = R_m d_cam and
// o = p + R t_m for a camera mounted at (R_m, t_m).  Per agent the pixel
// sums of grad * dt/do and of (grad * dt/dd) d_B^T (a 3x3 matrix, kept as three vector sums since d_B is
// affine in the pixel's image-plane coordinates) are reduced in a fixed order (accumulated in FP64), then
// chained through R and the quaternion normalisation.  One workgroup per agent; each thread has several
// pixels' id, triangle and gradient loads in flight at once.
#include "dynamics.h"
#include "vf_internal.h"

namespace vf {

// d/dq of sum_ij G_ij R_ij(q) for a unit quaternion q (no normalisation term).
template <typename T>
__device__ __forceinline__ void rot_vjp(const T q[4], const T G[9], T out[4]) {
    const T w = q[0], x = q[1], y = q[2], z = q[3];
    out[0] = T(2) * (-z * G[1] + y * G[2] + z * G[3] - x * G[5] - y * G[6] + x * G[7]);
    out[1] = T(2) * (y * G[1] + z * G[2] + y * G[3] - T(2) * x * G[4] - w * G[5] + z * G[6] + w * G[7] - T(2) * x * G[8]);
    out[2] = T(2) * (-T(2) * y * G[0] + x * G[1] + w * G[2] + x * G[3] + z * G[5] - w * G[6] + z * G[7] - T(2) * y * G[8]);
    out[3] = T(2) * (-T(2) * z * G[0] - w * G[1] + x * G[2] + w * G[3] - T(2) * z * G[4] + y * G[5] + x * G[6] + y * G[7]);
}

// lambda_q of q -> q/|q| given lambda on the normalised value.
template <typename T>
__device__ __forceinline__ void normalize_vjp(const T q[4], const T lam_n[4], T lam_q[4]) {
    const T n = vsqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    const T inv = T(1) / n;
    const T qn[4] = {q[0] * inv, q[1] * inv, q[2] * inv, q[3] * inv};
    const T dot = qn[0] * lam_n[0] + qn[1] * lam_n[1] + qn[2] * lam_n[2] + qn[3] * lam_n[3];
    for (int i = 0; i < 4; ++i) lam_q[i] = (lam_n[i] - qn[i] * dot) * inv;
}

// VJP of c(om) = om x (J om): returns d/d om of lam . c.
template <typename T>
__device__ __forceinline__ void gyro_vjp(const DynConstT<T>& c, const T om[3], const T lam[3], T out[3]) {
    const T j[3] = {c.J[0] * om[0], c.J[1] * om[1], c.J[2] * om[2]};
    // j x lam
    const T a0 = j[1] * lam[2] - j[2] * lam[1];
    const T a1 = j[2] * lam[0] - j[0] * lam[2];
    const T a2 = j[0] * lam[1] - j[1] * lam[0];
    // J (lam x om)
    const T b0 = c.J[0] * (lam[1] * om[2] - lam[2] * om[1]);
    const T b1 = c.J[1] * (lam[2] * om[0] - lam[0] * om[2]);
    const T b2 = c.J[2] * (lam[0] * om[1] - lam[1] * om[0]);
    out[0] = a0 + b0;
    out[1] = a1 + b1;
    out[2] = a2 + b2;
}

// Reverse of derivative(): given the cotangent L of d = F(y, w), accumulate into ly, lw.
template <typename T>
__device__ __forceinline__ void derivative_vjp(const DynConstT<T>& c, const Vec13T<T>& y, const T w[4],
                                               const Vec13T<T>& L, Vec13T<T>& ly, T lw[4]) {
    const T f[4] = {w[0] * w[0], w[1] * w[1], w[2] * w[2], w[3] * w[3]};
    T fz, tau[3];
    rotor_wrench(c, f, fz, tau);
    T r[9];
    body_rot(y.q, r);
    T vb[3];
    for (int i = 0; i < 3; ++i) vb[i] = r[0 + i] * y.v[0] + r[3 + i] * y.v[1] + r[6 + i] * y.v[2];
    T fb[3];
    for (int i = 0; i < 3; ++i) fb[i] = -c.k_lin[i] * vb[i] - c.c_quad[i] * vabs(vb[i]) * vb[i];
    fb[2] += fz;
    // d.p = v
    for (int i = 0; i < 3; ++i) ly.v[i] += L.p[i];
    // d.v = R fb / m - g z
    const T lv[3] = {L.v[0] * c.inv_mass, L.v[1] * c.inv_mass, L.v[2] * c.inv_mass};
    T G[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) G[3 * i + j] = lv[i] * fb[j];
    T lfb[3];
    for (int j = 0; j < 3; ++j) lfb[j] = r[j] * lv[0] + r[3 + j] * lv[1] + r[6 + j] * lv[2];
    const T lfz = lfb[2];
    T lvb[3];
    for (int i = 0; i < 3; ++i) lvb[i] = lfb[i] * (-c.k_lin[i] - T(2) * c.c_quad[i] * vabs(vb[i]));
    // vb_i = sum_j R_ji v_j
    for (int j = 0; j < 3; ++j) ly.v[j] += r[3 * j + 0] * lvb[0] + r[3 * j + 1] * lvb[1] + r[3 * j + 2] * lvb[2];
    for (int j = 0; j < 3; ++j)
        for (int i = 0; i < 3; ++i) G[3 * j + i] += y.v[j] * lvb[i];
    // R = R(q/|q|)
    {
        const T n = vsqrt(y.q[0] * y.q[0] + y.q[1] * y.q[1] + y.q[2] * y.q[2] + y.q[3] * y.q[3]);
        const T inv = T(1) / n;
        const T qn[4] = {y.q[0] * inv, y.q[1] * inv, y.q[2] * inv, y.q[3] * inv};
        T lqn[4], lq[4];
        rot_vjp(qn, G, lqn);
        normalize_vjp(y.q, lqn, lq);
        for (int i = 0; i < 4; ++i) ly.q[i] += lq[i];
    }
    // d.q = 1/2 q (x) (0, om)
    {
        const T* q = y.q;
        const T* om = y.w;
        const T a = T(0.5) * L.q[0], b = T(0.5) * L.q[1], cc = T(0.5) * L.q[2], d = T(0.5) * L.q[3];
        ly.q[0] += b * om[0] + cc * om[1] + d * om[2];
        ly.q[1] += -a * om[0] - cc * om[2] + d * om[1];
        ly.q[2] += -a * om[1] + b * om[2] - d * om[0];
        ly.q[3] += -a * om[2] - b * om[1] + cc * om[0];
        ly.w[0] += -a * q[1] + b * q[0] + cc * q[3] - d * q[2];
        ly.w[1] += -a * q[2] - b * q[3] + cc * q[0] + d * q[1];
        ly.w[2] += -a * q[3] + b * q[2] - cc * q[1] + d * q[0];
    }
    // d.w = J^-1 (tau - om x J om)
    const T ltau[3] = {L.w[0] * c.inv_J[0], L.w[1] * c.inv_J[1], L.w[2] * c.inv_J[2]};
    {
        const T lc[3] = {-ltau[0], -ltau[1], -ltau[2]};
        T g[3];
        gyro_vjp(c, y.w, lc, g);
        for (int i = 0; i < 3; ++i) ly.w[i] += g[i];
    }
    // tau, fz from f
    const T a = c.arm_a, k = c.kappa;
    T lf[4];
    lf[0] = lfz - a * ltau[0] - a * ltau[1] + k * ltau[2];
    lf[1] = lfz + a * ltau[0] + a * ltau[1] + k * ltau[2];
    lf[2] = lfz + a * ltau[0] - a * ltau[1] - k * ltau[2];
    lf[3] = lfz - a * ltau[0] + a * ltau[1] - k * ltau[2];
    for (int i = 0; i < 4; ++i) lw[i] += T(2) * w[i] * lf[i];
}

template <typename T>
__device__ __forceinline__ void zero13(Vec13T<T>& v) {
    for (int i = 0; i < 3; ++i) { v.p[i] = T(0); v.v[i] = T(0); v.w[i] = T(0); }
    for (int i = 0; i < 4; ++i) v.q[i] = T(0);
}

template <typename T>
__device__ __forceinline__ void load13(Vec13T<T>& y, const T s[17]) {
    for (int i = 0; i < 3; ++i) { y.p[i] = s[i]; y.v[i] = s[7 + i]; y.w[i] = s[10 + i]; }
    for (int i = 0; i < 4; ++i) y.q[i] = s[3 + i];
}

// Reverse of one CTBR / SRT sub-step (dyn_substep) starting at state s with action act, in FP64; lam (17)
// is the cotangent of the sub-step output and is overwritten with the cotangent of s; la (4) accumulates
// the action cotangent.
__device__ void substep_vjp(const DynConstD& c, const double s[17], const double act[4], double lam[17],
                            double la[4]) {
#pragma clang fp contract(off)
    // ---- recompute the forward sub-step ----
    double fraw[4], fdes[4], wd[4], w0[4], wh[4], wf[4];
    if (c.ctrl == VF_SRT) {
        for (int i = 0; i < 4; ++i) fraw[i] = act[i];
    } else {
        const double* om = s + 10;
        const double jo[3] = {c.J[0] * om[0], c.J[1] * om[1], c.J[2] * om[2]};
        const double t0 = c.kJ[0] * (act[1] - om[0]) + (om[1] * jo[2] - om[2] * jo[1]);
        const double t1 = c.kJ[1] * (act[2] - om[1]) + (om[2] * jo[0] - om[0] * jo[2]);
        const double t2 = c.kJ[2] * (act[3] - om[2]) + (om[0] * jo[1] - om[1] * jo[0]);
        const double u0 = c.mass * act[0], u1 = t0 * c.inv_a, u2 = t1 * c.inv_a, u3 = t2 * c.inv_kappa;
        fraw[0] = 0.25 * ((u0 + u3) - (u1 + u2));
        fraw[1] = 0.25 * ((u0 + u3) + (u1 + u2));
        fraw[2] = 0.25 * ((u0 - u3) + (u1 - u2));
        fraw[3] = 0.25 * ((u0 - u3) - (u1 - u2));
    }
    for (int i = 0; i < 4; ++i) {
        fdes[i] = fmin(fmax(fraw[i], 0.0), c.f_max);
        wd[i] = sqrt(fdes[i]);
        w0[i] = s[13 + i];
        wh[i] = wd[i] + (w0[i] - wd[i]) * c.e_half;
        wf[i] = wd[i] + (w0[i] - wd[i]) * c.e_full;
    }
    const double h = c.h;
    Vec13T<double> y, y1, y2, y3, k1, k2, k3, k4, yn;
    load13(y, s);
    derivative(c, y, w0, k1);
    const bool euler = c.integrator == VF_EULER;
    if (euler) {
        axpy13(yn, y, h, k1);
    } else {
        axpy13(y1, y, 0.5 * h, k1);
        derivative(c, y1, wh, k2);
        axpy13(y2, y, 0.5 * h, k2);
        derivative(c, y2, wh, k3);
        axpy13(y3, y, h, k3);
        derivative(c, y3, wf, k4);
        const double h6 = h / 6.0;
        for (int i = 0; i < 3; ++i) {
            yn.p[i] = y.p[i] + h6 * (k1.p[i] + 2.0 * (k2.p[i] + k3.p[i]) + k4.p[i]);
            yn.v[i] = y.v[i] + h6 * (k1.v[i] + 2.0 * (k2.v[i] + k3.v[i]) + k4.v[i]);
            yn.w[i] = y.w[i] + h6 * (k1.w[i] + 2.0 * (k2.w[i] + k3.w[i]) + k4.w[i]);
        }
        for (int i = 0; i < 4; ++i) yn.q[i] = y.q[i] + h6 * (k1.q[i] + 2.0 * (k2.q[i] + k3.q[i]) + k4.q[i]);
    }
    // ---- reverse ----
    double lwf[4], lwh[4] = {0.0, 0.0, 0.0, 0.0}, lw0[4] = {0.0, 0.0, 0.0, 0.0};
    for (int i = 0; i < 4; ++i) lwf[i] = lam[13 + i];
    Vec13T<double> lyn;
    for (int i = 0; i < 3; ++i) { lyn.p[i] = lam[i]; lyn.v[i] = lam[7 + i]; lyn.w[i] = lam[10 + i]; }
    {
        const double lqn[4] = {lam[3], lam[4], lam[5], lam[6]};
        normalize_vjp(yn.q, lqn, lyn.q);
    }
    Vec13T<double> ly = lyn;
    if (euler) {
        Vec13T<double> lk1;
        for (int i = 0; i < 3; ++i) { lk1.p[i] = h * lyn.p[i]; lk1.v[i] = h * lyn.v[i]; lk1.w[i] = h * lyn.w[i]; }
        for (int i = 0; i < 4; ++i) lk1.q[i] = h * lyn.q[i];
        derivative_vjp(c, y, w0, lk1, ly, lw0);
    } else {
        const double h6 = h / 6.0, h3 = h / 3.0;
        Vec13T<double> lk1, lk2, lk3, lk4, l3, l2, l1;
        for (int i = 0; i < 3; ++i) {
            lk1.p[i] = h6 * lyn.p[i]; lk2.p[i] = h3 * lyn.p[i]; lk3.p[i] = h3 * lyn.p[i]; lk4.p[i] = h6 * lyn.p[i];
            lk1.v[i] = h6 * lyn.v[i]; lk2.v[i] = h3 * lyn.v[i]; lk3.v[i] = h3 * lyn.v[i]; lk4.v[i] = h6 * lyn.v[i];
            lk1.w[i] = h6 * lyn.w[i]; lk2.w[i] = h3 * lyn.w[i]; lk3.w[i] = h3 * lyn.w[i]; lk4.w[i] = h6 * lyn.w[i];
        }
        for (int i = 0; i < 4; ++i) {
            lk1.q[i] = h6 * lyn.q[i]; lk2.q[i] = h3 * lyn.q[i]; lk3.q[i] = h3 * lyn.q[i]; lk4.q[i] = h6 * lyn.q[i];
        }
        // k4 = F(y3, wf), y3 = y + h k3
        zero13(l3);
        derivative_vjp(c, y3, wf, lk4, l3, lwf);
        axpy13(ly, ly, 1.0, l3);
        axpy13(lk3, lk3, h, l3);
        // k3 = F(y2, wh), y2 = y + h/2 k2
        zero13(l2);
        derivative_vjp(c, y2, wh, lk3, l2, lwh);
        axpy13(ly, ly, 1.0, l2);
        axpy13(lk2, lk2, 0.5 * h, l2);
        // k2 = F(y1, wh), y1 = y + h/2 k1
        zero13(l1);
        derivative_vjp(c, y1, wh, lk2, l1, lwh);
        axpy13(ly, ly, 1.0, l1);
        axpy13(lk1, lk1, 0.5 * h, l1);
        // k1 = F(y, w0)
        derivative_vjp(c, y, w0, lk1, ly, lw0);
    }
    // rotor lag: wh = wd + (w0 - wd) e_half, wf = wd + (w0 - wd) e_full
    double lwd[4], lf[4];
    for (int i = 0; i < 4; ++i) {
        lw0[i] += c.e_half * lwh[i] + c.e_full * lwf[i];
        lwd[i] = (1.0 - c.e_half) * lwh[i] + (1.0 - c.e_full) * lwf[i];
        // wd = sqrt(fdes), fdes = clamp(fraw)
        const bool inside = fraw[i] > 0.0 && fraw[i] < c.f_max;
        lf[i] = (inside && wd[i] > 0.0) ? lwd[i] * 0.5 / wd[i] : 0.0;
    }
    double lom_ctrl[3] = {0.0, 0.0, 0.0};
    if (c.ctrl == VF_SRT) {
        for (int i = 0; i < 4; ++i) la[i] += lf[i];
    } else {
        const double lu0 = 0.25 * ((lf[0] + lf[1]) + (lf[2] + lf[3]));
        const double lu1 = 0.25 * ((lf[1] + lf[2]) - (lf[0] + lf[3]));
        const double lu2 = 0.25 * ((lf[1] + lf[3]) - (lf[0] + lf[2]));
        const double lu3 = 0.25 * ((lf[0] + lf[1]) - (lf[2] + lf[3]));
        const double lt[3] = {lu1 * c.inv_a, lu2 * c.inv_a, lu3 * c.inv_kappa};
        la[0] += c.mass * lu0;
        for (int k = 0; k < 3; ++k) {
            la[1 + k] += c.kJ[k] * lt[k];
            lom_ctrl[k] -= c.kJ[k] * lt[k];
        }
        double g[3];
        gyro_vjp(c, s + 10, lt, g);
        for (int k = 0; k < 3; ++k) lom_ctrl[k] += g[k];
    }
    for (int i = 0; i < 3; ++i) {
        lam[i] = ly.p[i];
        lam[7 + i] = ly.v[i];
        lam[10 + i] = ly.w[i] + lom_ctrl[i];
    }
    for (int i = 0; i < 4; ++i) {
        lam[3 + i] = ly.q[i];
        lam[13 + i] = lw0[i];
    }
}

// One thread per agent: the control step's sub-step states are recomputed from the saved state in FP64
// exactly as dyn_step computed them, then walked in reverse; the cotangents are carried in FP64 and
// rounded to float32 once at the end.
__global__ void __launch_bounds__(128) k_step_backward(StepBackArgs a) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    double s0[17], act[4], lam[17], la[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k = 0; k < 17; ++k) {
        s0[k] = (double)a.state_in[(int64_t)i * 17 + k];
        lam[k] = (double)a.grad_out[(int64_t)i * 17 + k];
    }
    for (int k = 0; k < 4; ++k) act[k] = (double)a.action[(int64_t)i * 4 + k];
    for (int sub = a.dyn.n_sub - 1; sub >= 0; --sub) {
        double s[17];
        for (int k = 0; k < 17; ++k) s[k] = s0[k];
        for (int j = 0; j < sub; ++j) dyn_substep(a.dyn, s, act);
        substep_vjp(a.dyn, s, act, lam, la);
    }
    for (int k = 0; k < 17; ++k) a.grad_in[(int64_t)i * 17 + k] = (float)lam[k];
    for (int k = 0; k < 4; ++k) a.grad_action[(int64_t)i * 4 + k] = (float)la[k];
}

// ---------------------------------------------------------------------------
// Forward-mode form of the step adjoint (every controller; the launcher takes it for PS and LV, whose
// outer loop has no hand-written reverse): dual numbers v + d eps carry one tangent through the same
// templated sub-steps.  Each value is the FP64 operation the control step performs (contraction off, as
// there), so the tangent is the derivative of exactly the computation the forward runs.  Branches (the
// tilt limit) and clamps take the derivative of the side the value took.
// ---------------------------------------------------------------------------
struct Dual {
    double v, d;
    __device__ Dual() : v(0.0), d(0.0) {}
    __device__ Dual(double x) : v(x), d(0.0) {}
    __device__ Dual(double x, double dx) : v(x), d(dx) {}
};
__device__ __forceinline__ Dual operator+(Dual a, Dual b) {
#pragma clang fp contract(off)
    return Dual(a.v + b.v, a.d + b.d);
}
__device__ __forceinline__ Dual operator-(Dual a, Dual b) {
#pragma clang fp contract(off)
    return Dual(a.v - b.v, a.d - b.d);
}
__device__ __forceinline__ Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
__device__ __forceinline__ Dual operator*(Dual a, Dual b) {
#pragma clang fp contract(off)
    return Dual(a.v * b.v, a.d * b.v + a.v * b.d);
}
__device__ __forceinline__ Dual operator/(Dual a, Dual b) {
#pragma clang fp contract(off)
    const double q = a.v / b.v;
    return Dual(q, (a.d - q * b.d) / b.v);
}
__device__ __forceinline__ Dual& operator+=(Dual& a, Dual b) { return a = a + b; }
__device__ __forceinline__ Dual& operator-=(Dual& a, Dual b) { return a = a - b; }
__device__ __forceinline__ Dual& operator*=(Dual& a, Dual b) { return a = a * b; }
__device__ __forceinline__ bool operator>(Dual a, Dual b) { return a.v > b.v; }
__device__ __forceinline__ bool operator<(Dual a, Dual b) { return a.v < b.v; }
__device__ __forceinline__ Dual vsqrt(Dual x) {
    const double r = sqrt(x.v);
    // a clamped zero (tangent 0) stays flat instead of 0 / 0
    return Dual(r, x.d == 0.0 ? 0.0 : x.d / (2.0 * r));
}
__device__ __forceinline__ Dual vabs(Dual x) { return x.v < 0.0 ? -x : x; }
// the operand fmin / fmax return (the non-NaN one, the first at a tie) with its tangent
__device__ __forceinline__ Dual vmin(Dual a, Dual b) { return fmin(a.v, b.v) == a.v ? a : b; }
__device__ __forceinline__ Dual vmax(Dual a, Dual b) { return fmax(a.v, b.v) == a.v ? a : b; }
__device__ __forceinline__ void vsincos(Dual x, Dual* s, Dual* c) {
    double sv, cv;
    sincos(x.v, &sv, &cv);
    *s = Dual(sv, cv * x.d);
    *c = Dual(cv, -sv * x.d);
}

__device__ __forceinline__ DynConstT<Dual> dual_const(const DynConstD& c) {
    DynConstT<Dual> o;
    o.h = c.h;
    o.n_sub = c.n_sub;
    o.integrator = c.integrator;
    o.ctrl = c.ctrl;
    o.mass = c.mass;
    o.inv_mass = c.inv_mass;
    o.g = c.g;
    for (int i = 0; i < 3; ++i) {
        o.J[i] = c.J[i];
        o.inv_J[i] = c.inv_J[i];
        o.kJ[i] = c.kJ[i];
        o.k_lin[i] = c.k_lin[i];
        o.c_quad[i] = c.c_quad[i];
        o.k_pos[i] = c.k_pos[i];
        o.k_vel[i] = c.k_vel[i];
        o.k_att[i] = c.k_att[i];
    }
    o.arm_a = c.arm_a;
    o.inv_a = c.inv_a;
    o.kappa = c.kappa;
    o.inv_kappa = c.inv_kappa;
    o.f_max = c.f_max;
    o.e_half = c.e_half;
    o.e_full = c.e_full;
    o.tan_tilt = c.tan_tilt;
    o.min_lift = c.min_lift;
    return o;
}

// One thread per (agent, input coordinate j of the 17 state and 4 action values): the control step on
// dual numbers seeded with e_j gives column j of the step Jacobian, and its dot product with the output
// cotangent is component j of the input cotangent.  The n_sub sub-steps run once each.
constexpr int kTangentThreads = 64;
__global__ void __launch_bounds__(kTangentThreads) k_step_backward_tangent(StepBackArgs a) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)a.n * 21) return;
    const int64_t i = t / 21;
    const int j = (int)(t - i * 21);
    const DynConstT<Dual> c = dual_const(a.dyn);
    Dual s[17], act[4];
    for (int k = 0; k < 17; ++k) s[k] = Dual((double)a.state_in[i * 17 + k], k == j ? 1.0 : 0.0);
    for (int k = 0; k < 4; ++k) act[k] = Dual((double)a.action[i * 4 + k], 17 + k == j ? 1.0 : 0.0);
    for (int sub = 0; sub < a.dyn.n_sub; ++sub) dyn_substep(c, s, act);
    double g = 0.0;
    for (int k = 0; k < 17; ++k) g += (double)a.grad_out[i * 17 + k] * s[k].d;
    if (j < 17)
        a.grad_in[i * 17 + j] = (float)g;
    else
        a.grad_action[i * 4 + (j - 17)] = (float)g;
}

// The workgroup's per-agent constants are the same in every lane: held in scalar registers they leave the
// vector registers to the pixel batch.
__device__ __forceinline__ double wave_uniform(double x) {
    const uint64_t b = (uint64_t)__double_as_longlong(x);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

constexpr int kBackThreads = 256;
constexpr int kBackBatch = 2;   // pixels per thread whose id, triangle and gradient loads are in flight together

__global__ void __launch_bounds__(kBackThreads) __attribute__((amdgpu_waves_per_eu(4))) k_render_backward(RenderBackArgs a) {
    __shared__ double red[kBackThreads / 64][12];
    const int agent = blockIdx.x;
    vf_view vw = a.views[agent];
    bool ok = vw.scene_id >= 0 && vw.scene_id < a.n_scenes && vw.H >= 1 && vw.W >= 1 && vw.H <= a.max_h &&
              vw.W <= a.max_w && vw.out_offset >= 0 && vw.out_offset + (int64_t)vw.H * vw.W <= a.out_pixels &&
              vw.hfov > 0.f && vw.hfov < 3.1415926f && vw.near_clip > 0.f && vw.far_clip > vw.near_clip;
    if (ok) ok = a.scenes[vw.scene_id].valid != 0;
    if (!ok) {
        if (threadIdx.x == 0) atomicOr(a.err, kErrView);
        return;
    }
    const SceneDesc sc = a.scenes[vw.scene_id];
    const float* st = a.state + (int64_t)agent * 17;
    const double qd[4] = {st[3], st[4], st[5], st[6]};
    double rot[9];
    body_rot(qd, rot);
    // camera mount: origin p + R t_m, body-frame direction R_m d_cam
    double m[9] = {1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 1.0};
    if (!(vw.mount_q[1] == 0.0f && vw.mount_q[2] == 0.0f && vw.mount_q[3] == 0.0f)) {
        const double mq[4] = {vw.mount_q[0], vw.mount_q[1], vw.mount_q[2], vw.mount_q[3]};
        body_rot(mq, m);
    }
    const double tm[3] = {vw.mount_t[0], vw.mount_t[1], vw.mount_t[2]};
    double o[3];
    for (int i = 0; i < 3; ++i)
        o[i] = (double)st[i] + (rot[3 * i] * tm[0] + rot[3 * i + 1] * tm[1] + rot[3 * i + 2] * tm[2]);
    // camera ray of pixel (r, c): d_cam = (1, -u, v), u and v affine in c and r with the same step du;
    // world direction d = C0 - u C1 + v C2, column j of C = R R_m
    const double tan_h = tan(0.5 * (double)vw.hfov);
    const double du = wave_uniform(2.0 * tan_h / (double)vw.W);
    const double u0 = wave_uniform(0.5 * du - tan_h), v0 = wave_uniform(tan_h * (double)vw.H / (double)vw.W - 0.5 * du);
    double C[3][3];   // C[j][i]: component i of column j
    for (int j = 0; j < 3; ++j)
        for (int i = 0; i < 3; ++i)
            C[j][i] = wave_uniform(rot[3 * i] * m[j] + rot[3 * i + 1] * m[3 + j] + rot[3 * i + 2] * m[6 + j]);
    for (int i = 0; i < 3; ++i) o[i] = wave_uniform(o[i]);
    // acc[0..2]: sum s_o n; acc[3..11]: sums of w n, w u n and w v n (w = s_d), from which
    // sum w n d_cam^T follows because d_cam is affine in (u, v)
    double acc[12];
    for (int k = 0; k < 12; ++k) acc[k] = 0.0;
    uint32_t bad = 0;
    const int npix = vw.H * vw.W;
    const int32_t* idp = a.tri_id + vw.out_offset;
    const float* gp = a.grad_depth + vw.out_offset;
    for (int base = threadIdx.x; base < npix; base += kBackBatch * kBackThreads) {
        int32_t slot[kBackBatch];
        float g[kBackBatch];
#pragma unroll
        for (int k = 0; k < kBackBatch; ++k) {
            const int pix = base + k * kBackThreads;
            int32_t id = -1;
            g[k] = 0.0f;
            if (pix < npix) {
                id = idp[pix];
                g[k] = gp[pix];
            }
            slot[k] = -1;
            if (id >= 0 && g[k] != 0.0f) {
                if (id < sc.n_tris)
                    slot[k] = id;
                else if (vw.swarm <= 0)
                    bad = kErrTriId;   // ids past the mesh name swarm members: no gradient
            }
        }
#pragma unroll
        for (int k = 0; k < kBackBatch; ++k)
            if (slot[k] >= 0) slot[k] = sc.sorted_of[slot[k]];
        Tri tr[kBackBatch];
#pragma unroll
        for (int k = 0; k < kBackBatch; ++k)
            if (slot[k] >= 0) tr[k] = sc.tris[slot[k]];
#pragma unroll
        for (int k = 0; k < kBackBatch; ++k) {
            if (slot[k] < 0) continue;
            const int pix = base + k * kBackThreads;
            const int r = pix / vw.W, cc = pix - r * vw.W;
            const double u = u0 + du * (double)cc, v = v0 - du * (double)r;
            double d[3];
            for (int i = 0; i < 3; ++i) d[i] = C[0][i] - u * C[1][i] + v * C[2][i];
            const double e1[3] = {tr[k].e1x, tr[k].e1y, tr[k].e1z}, e2[3] = {tr[k].e2x, tr[k].e2y, tr[k].e2z};
            const double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                                 e1[0] * e2[1] - e1[1] * e2[0]};
            const double nd = n[0] * d[0] + n[1] * d[1] + n[2] * d[2];
            if (nd == 0.0) continue;
            const double inv = 1.0 / nd;
            const double t = (n[0] * ((double)tr[k].v0x - o[0]) + n[1] * ((double)tr[k].v0y - o[1]) +
                              n[2] * ((double)tr[k].v0z - o[2])) * inv;
            const double s_o = -(double)g[k] * inv, w = s_o * t;
            for (int i = 0; i < 3; ++i) {
                const double wn = w * n[i];
                acc[i] += s_o * n[i];
                acc[3 + i] += wn;
                acc[6 + i] += wn * u;
                acc[9 + i] += wn * v;
            }
        }
    }
    if (bad) atomicOr(a.err, bad);
    // fixed-order reduction: butterfly within each wavefront, then the wavefronts in order
    for (int k = 0; k < 12; ++k)
        for (int off = 32; off > 0; off >>= 1) acc[k] += __shfl_xor(acc[k], off);
    if ((threadIdx.x & 63) == 0)
        for (int k = 0; k < 12; ++k) red[threadIdx.x >> 6][k] = acc[k];
    __syncthreads();
    if (threadIdx.x == 0) {
        // re-read after the barrier rather than keep them live through the pixel loop
        const vf_view vw2 = a.views[agent];
        const float* st2 = a.state + (int64_t)agent * 17;
        const double q2[4] = {st2[3], st2[4], st2[5], st2[6]};
        double m2[9] = {1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 1.0};
        if (!(vw2.mount_q[1] == 0.0f && vw2.mount_q[2] == 0.0f && vw2.mount_q[3] == 0.0f)) {
            const double mq[4] = {vw2.mount_q[0], vw2.mount_q[1], vw2.mount_q[2], vw2.mount_q[3]};
            body_rot(mq, m2);
        }
        const double tm2[3] = {vw2.mount_t[0], vw2.mount_t[1], vw2.mount_t[2]};
        double S[12];
        for (int k = 0; k < 12; ++k) {
            S[k] = red[0][k];
            for (int wv = 1; wv < kBackThreads / 64; ++wv) S[k] += red[wv][k];
        }
        float* gs = a.grad_state + (int64_t)agent * 17;
        for (int k = 0; k < 3; ++k) gs[k] += (float)S[k];
        // G = sum w n d_B^T with d_B = R_m d_cam: column j of d_B is m[3j] - u m[3j+1] + v m[3j+2]
        double G[9];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                G[3 * i + j] = S[3 + i] * m2[3 * j] - S[6 + i] * m2[3 * j + 1] + S[9 + i] * m2[3 * j + 2];
        // the origin p + R t_m also moves with R
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) G[3 * i + j] += S[i] * tm2[j];
        const double inv = 1.0 / sqrt(q2[0] * q2[0] + q2[1] * q2[1] + q2[2] * q2[2] + q2[3] * q2[3]);
        const double qn[4] = {q2[0] * inv, q2[1] * inv, q2[2] * inv, q2[3] * inv};
        double lqn[4], lq[4];
        rot_vjp(qn, G, lqn);
        normalize_vjp(q2, lqn, lq);
        for (int k = 0; k < 4; ++k) gs[3 + k] += (float)lq[k];
    }
}

hipError_t launch_step_backward(const StepBackArgs& a, hipStream_t st) {
    if (a.n <= 0) return hipSuccess;
    if (a.dyn.ctrl == VF_PS || a.dyn.ctrl == VF_LV) {
        const int64_t threads = (int64_t)a.n * 21;
        hipLaunchKernelGGL(k_step_backward_tangent, dim3((unsigned)((threads + kTangentThreads - 1) / kTangentThreads)),
                           dim3(kTangentThreads), 0, st, a);
    } else {
        hipLaunchKernelGGL(k_step_backward, dim3((a.n + 127) / 128), dim3(128), 0, st, a);
    }
    return hipGetLastError();
}

hipError_t launch_render_backward(const RenderBackArgs& a, hipStream_t st) {
    if (a.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_render_backward, dim3(a.n), dim3(kBackThreads), 0, st, a);
    return hipGetLastError();
}

}  // namespace vf
