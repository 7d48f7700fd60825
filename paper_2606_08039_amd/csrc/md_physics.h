// md_physics.h -- per-drone device physics shared by the step kernels:
// rotation matrix, Euler angles, cascaded PID, motor model, aerodynamic
// terms and the integrator (paper: Sec. "Quadrotor Dynamics", Sec. "Physics
// Modes", Sec. "Control").
#pragma once

#include "md_internal.h"

namespace md {
namespace phys {

constexpr float kTwoPi = 6.283185307179586f;
constexpr float kPi = 3.141592653589793f;

__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

struct Drone {
    float px, py, pz;
    float qw, qx, qy, qz;
    float vx, vy, vz;
    float wx, wy, wz;
};

// Body->world rotation matrix entries of a unit quaternion.
struct Rot {
    float r00, r01, r02, r10, r11, r12, r20, r21, r22;
};

// The five entries the Z-Y-X angles read.  Their fused multiply-adds are
// written out and no other contraction is allowed, so each entry rounds the
// same way wherever it is inlined: the angles formed for the observation and
// the controller agree bit for bit between the kernels' code paths.
struct RotZYX {
    float r00, r10, r20, r21, r22;
};

__device__ __forceinline__ RotZYX rot_zyx(const Drone &d) {
#pragma clang fp contract(off)
    const float w = d.qw, x = d.qx, y = d.qy, z = d.qz;
    RotZYX e;
    e.r00 = fmaf(-2.f, fmaf(y, y, z * z), 1.f);
    e.r10 = 2.f * fmaf(x, y, w * z);
    e.r20 = 2.f * fmaf(x, z, -(w * y));
    e.r21 = 2.f * fmaf(y, z, w * x);
    e.r22 = fmaf(-2.f, fmaf(x, x, y * y), 1.f);
    return e;
}

__device__ __forceinline__ Rot rot_of(const Drone &d) {
    const float w = d.qw, x = d.qx, y = d.qy, z = d.qz;
    const RotZYX e = rot_zyx(d);
    Rot R;
    R.r00 = e.r00;
    R.r01 = 2.f * (x * y - w * z);
    R.r02 = 2.f * (x * z + w * y);
    R.r10 = e.r10;
    R.r11 = 1.f - 2.f * (x * x + z * z);
    R.r12 = 2.f * (y * z - w * x);
    R.r20 = e.r20;
    R.r21 = e.r21;
    R.r22 = e.r22;
    return R;
}


__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// arctan(a) for a in [0, 1] as a * P(a^2), P of degree 7 fitted to atan(a)/a
// by iteratively reweighted least squares on Chebyshev nodes (max error
// 3.8e-8 rad in exact arithmetic, 1.3e-7 rad evaluated in float32).
__device__ __forceinline__ float atan01(float a) {
    const float s = a * a;
    float p = -4.054536119e-03f;
    p = p * s + 2.186285485e-02f;
    p = p * s - 5.591219459e-02f;
    p = p * s + 9.642189160e-02f;
    p = p * s - 1.390862714e-01f;
    p = p * s + 1.994656539e-01f;
    p = p * s - 3.332986079e-01f;
    p = p * s + 9.999993356e-01f;
    return a * p;
}

// atan2 by octant reduction to atan01 (the quotient of the smaller over the
// larger magnitude, then pi/2 - r, pi - r and the sign of y); 0 for (0, 0).
__device__ __forceinline__ float atan2_poly(float y, float x) {
    const float ax = fabsf(x), ay = fabsf(y);
    const float mx = fmaxf(ax, ay), mn = fminf(ax, ay);
    const float a = mx > 0.f ? mn * rcp(mx) : 0.f;
    float r = atan01(a);
    r = (ay > ax) ? 1.5707963267948966f - r : r;
    r = (x < 0.f) ? 3.141592653589793f - r : r;
    return copysignf(r, y);
}

// asin(s) = atan2(s, sqrt((1 - s)(1 + s))), |s| <= 1
__device__ __forceinline__ float asin_poly(float s) { return atan2_poly(s, fsqrt((1.f - s) * (1.f + s))); }

// Roll, pitch, yaw (Z-Y-X) of the KIN observation from the rotation entries:
// roll = atan2(R21, R22), pitch = asin(-R20), yaw = atan2(R10, R00).
__device__ __forceinline__ void euler_of(const RotZYX &e, float &roll, float &pitch, float &yaw) {
    const float sp = fminf(fmaxf(-e.r20, -1.f), 1.f);
    roll = atan2_poly(e.r21, e.r22);
    pitch = asin_poly(sp);
    yaw = atan2_poly(e.r10, e.r00);
}

__device__ __forceinline__ void euler_zyx(const Drone &d, float &roll, float &pitch, float &yaw) {
    euler_of(rot_zyx(d), roll, pitch, yaw);
}

// One drone's KIN-20 row into ring slot `oslot` ([slot][20][N]) through a
// buffer resource whose base is the slot (wave-uniform, so it lives in
// scalar registers): each row is one buffer store with the lane's byte
// offset and the row offset k N 4 as the scalar offset, no per-row address
// arithmetic on the vector ALU (n_drones <= 2^25 keeps 80 N within 32 bits).
// The row offsets are formed by scalar adds beside the stores (the stride is
// made opaque per call): hoisted out of a step loop, twenty of them overflow
// the scalar registers and the spilled ones return through the vector ALU.
__device__ __forceinline__ void store_obs(float *obs, int oslot, int N, int di, const float row[20]) {
    float *base = obs + (long long)oslot * 20 * N;
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(base, (short)0, (int)0xffffffffu, 0x00020000);
    const int voff = di * 4;
    uint32_t rb = (uint32_t)N * 4u;
    asm volatile("" : "+s"(rb));
    uint32_t so = 0;
#pragma unroll
    for (int k = 0; k < 20; ++k) {
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(row[k]), rs, voff, (int)so, 0);
        so += rb;
    }
}

__device__ __forceinline__ float clampf(float x, float lo, float hi) {
    return fminf(fmaxf(x, lo), hi);
}

__device__ __forceinline__ float wrap_pi(float a) {
    return a - kTwoPi * floorf((a + kPi) * (1.f / kTwoPi));
}

// Roll, pitch, yaw and the yaw's sine and cosine (straight from the atan2
// arguments, no further transcendental).
__device__ __forceinline__ void yaw_sincos(const RotZYX &e, float &sps, float &cps) {
    const float ys = e.r10, yc = e.r00;
    const float h2 = ys * ys + yc * yc;
    const float hinv = h2 > 0.f ? rsqrtf(h2) : 0.f;
    sps = h2 > 0.f ? ys * hinv : 0.f;
    cps = h2 > 0.f ? yc * hinv : 1.f;
}

// Attitude PID and exact allocation inverse shared by the controllers:
// e = (roll* - roll, pitch* - pitch, e_yaw), I += e dt_c clamped,
// tau = Kp e + Ki I + Kd (w*_z z_hat - w); rotor forces clipped to
// [0, kf MAX_RPM^2] (Sec. "Control").
__device__ __forceinline__ void attitude_allocate(const KConst &c, const Drone &d, float roll, float pitch,
                                                  float T, float roll_t, float pitch_t, float e_yaw,
                                                  float wz_t, const float *kp, const float *ki,
                                                  const float *kd, float clamp, float *Ia, float n[4]) {
    const float er = roll_t - roll, ep = pitch_t - pitch;
    Ia[0] = clampf(Ia[0] + er * c.dt_c, -clamp, clamp);
    Ia[1] = clampf(Ia[1] + ep * c.dt_c, -clamp, clamp);
    Ia[2] = clampf(Ia[2] + e_yaw * c.dt_c, -clamp, clamp);
    const float tx = kp[0] * er + ki[0] * Ia[0] - kd[0] * d.wx;
    const float ty = kp[1] * ep + ki[1] * Ia[1] - kd[1] * d.wy;
    const float tz = kp[2] * e_yaw + ki[2] * Ia[2] + kd[2] * (wz_t - d.wz);
    const float a = tx * c.l_inv, b = ty * c.l_inv, e = tz * c.kappa_inv;
    const float F0 = 0.25f * (T + a - b - e);
    const float F1 = 0.25f * (T + a + b + e);
    const float F2 = 0.25f * (T - a + b - e);
    const float F3 = 0.25f * (T - a - b + e);
    n[0] = fsqrt(clampf(F0, 0.f, c.fmax) * c.kf_inv);
    n[1] = fsqrt(clampf(F1, 0.f, c.fmax) * c.kf_inv);
    n[2] = fsqrt(clampf(F2, 0.f, c.fmax) * c.kf_inv);
    n[3] = fsqrt(clampf(F3, 0.f, c.fmax) * c.kf_inv);
}

// Thrust T = m |a*| and the near-hover attitude target at the current yaw.
__device__ __forceinline__ void thrust_direction(const KConst &c, float ax, float ay, float az, float sps,
                                                 float cps, float &T, float &roll_t, float &pitch_t) {
    T = c.m * fsqrt(ax * ax + ay * ay + az * az);
    roll_t = (ax * sps - ay * cps) * c.g_inv;
    pitch_t = (ax * cps + ay * sps) * c.g_inv;
}

// One controller update (Sec. "Control"; Table "Action types"):
//   ACT 1 cascaded PID to waypoint (x, y, z, yaw);
//   ACT 2 VEL: heading-frame velocity + yaw rate, a* = Kd (v* - v) + g;
//   ACT 3 ATTITUDE: collective thrust, roll, pitch, yaw rate;
//   ACT 4 DSL-style PID: rate-limited setpoint sp (x, y, z, yaw) toward the
//         waypoint, own gains and clamps, feed-forward acceleration cmd[4..6].
// control_rpy takes the angles already formed from the same rotation
// entries (euler_of(e)); control forms them itself.
template <int ACT>
__device__ __forceinline__ void control_rpy(const KConst &c, const Drone &d, const RotZYX &e, float roll,
                                            float pitch, float yaw, const float *cmd, float I[6], float sp[4],
                                            float n[4]) {
    float sps, cps;
    yaw_sincos(e, sps, cps);
    if (ACT == 1) {
        const float ex = cmd[0] - d.px, ey = cmd[1] - d.py, ez = cmd[2] - d.pz;
        I[0] = clampf(I[0] + ex * c.dt_c, -c.p_clamp, c.p_clamp);
        I[1] = clampf(I[1] + ey * c.dt_c, -c.p_clamp, c.p_clamp);
        I[2] = clampf(I[2] + ez * c.dt_c, -c.p_clamp, c.p_clamp);
        const float ax = c.pkp[0] * ex + c.pki[0] * I[0] - c.pkd[0] * d.vx;
        const float ay = c.pkp[1] * ey + c.pki[1] * I[1] - c.pkd[1] * d.vy;
        const float az = c.pkp[2] * ez + c.pki[2] * I[2] - c.pkd[2] * d.vz + c.g;
        float T, rt, pt;
        thrust_direction(c, ax, ay, az, sps, cps, T, rt, pt);
        attitude_allocate(c, d, roll, pitch, T, rt, pt, wrap_pi(cmd[3] - yaw), 0.f, c.akp, c.aki, c.akd,
                          c.a_clamp, I + 3, n);
    } else if (ACT == 2) {
        const float vtx = cps * cmd[0] - sps * cmd[1], vty = sps * cmd[0] + cps * cmd[1];
        const float ax = c.pkd[0] * (vtx - d.vx);
        const float ay = c.pkd[1] * (vty - d.vy);
        const float az = c.pkd[2] * (cmd[2] - d.vz) + c.g;
        float T, rt, pt;
        thrust_direction(c, ax, ay, az, sps, cps, T, rt, pt);
        attitude_allocate(c, d, roll, pitch, T, rt, pt, 0.f, cmd[3], c.akp, c.aki, c.akd, c.a_clamp, I + 3, n);
    } else if (ACT == 3) {
        attitude_allocate(c, d, roll, pitch, cmd[0], cmd[1], cmd[2], 0.f, cmd[3], c.akp, c.aki, c.akd,
                          c.a_clamp, I + 3, n);
    } else {
        const float dx = cmd[0] - sp[0], dy = cmd[1] - sp[1], dz = cmd[2] - sp[2];
        const float dn = fsqrt(dx * dx + dy * dy + dz * dz);
        const float sc = dn > c.dsl_step ? c.dsl_step * rcp(dn) : 1.f;
        sp[0] += sc * dx;
        sp[1] += sc * dy;
        sp[2] += sc * dz;
        sp[3] = wrap_pi(sp[3] + clampf(wrap_pi(cmd[3] - sp[3]), -c.dsl_ystep, c.dsl_ystep));
        const float ex = sp[0] - d.px, ey = sp[1] - d.py, ez = sp[2] - d.pz;
        I[0] = clampf(I[0] + ex * c.dt_c, -c.dsl_p_clamp, c.dsl_p_clamp);
        I[1] = clampf(I[1] + ey * c.dt_c, -c.dsl_p_clamp, c.dsl_p_clamp);
        I[2] = clampf(I[2] + ez * c.dt_c, -c.dsl_p_clamp, c.dsl_p_clamp);
        const float ax = c.dsl_pkp[0] * ex + c.dsl_pki[0] * I[0] - c.dsl_pkd[0] * d.vx + cmd[4];
        const float ay = c.dsl_pkp[1] * ey + c.dsl_pki[1] * I[1] - c.dsl_pkd[1] * d.vy + cmd[5];
        const float az = c.dsl_pkp[2] * ez + c.dsl_pki[2] * I[2] - c.dsl_pkd[2] * d.vz + cmd[6] + c.g;
        float T, rt, pt;
        thrust_direction(c, ax, ay, az, sps, cps, T, rt, pt);
        attitude_allocate(c, d, roll, pitch, T, rt, pt, wrap_pi(sp[3] - yaw), 0.f, c.dsl_akp, c.dsl_aki,
                          c.dsl_akd, c.dsl_a_clamp, I + 3, n);
    }
}

template <int ACT>
__device__ __forceinline__ void control(const KConst &c, const Drone &d, const float *cmd, float I[6],
                                        float sp[4], float n[4]) {
    const RotZYX e = rot_zyx(d);
    float roll, pitch, yaw;
    euler_of(e, roll, pitch, yaw);
    control_rpy<ACT>(c, d, e, roll, pitch, yaw, cmd, I, sp, n);
}

// Motor model and X mixer (Eq. 1-3).  Contraction into fused multiply-adds is
// off here: each rotor force is rounded once, so rotors at equal speed cancel
// exactly in the roll, pitch and yaw torques (an unrounded product left over
// by an fma would leave a spurious torque that tilts a hovering drone).
__device__ __forceinline__ void motor(const KConst &c, const float n[4], float &T, float &tx,
                                      float &ty, float &tz) {
#pragma clang fp contract(off)
    const float n0 = n[0] * n[0], n1 = n[1] * n[1], n2 = n[2] * n[2], n3 = n[3] * n[3];
    const float F0 = c.kf * n0, F1 = c.kf * n1, F2 = c.kf * n2, F3 = c.kf * n3;
    T = (F0 + F1) + (F2 + F3);
    tx = c.l_arm * ((F0 - F2) + (F1 - F3));
    ty = c.l_arm * ((F1 - F3) - (F0 - F2));
    tz = c.km * ((n1 - n0) + (n3 - n2));
}

// Semi-implicit Euler plus the exponential map q <- q (x) [cos th, sin th w/|w|],
// th = |w| dt / 2, then renormalisation.  For th < 1/4 the sine and cosine come
// from their Taylor series in th^2 = (dt/2)^2 |w|^2 (truncation error < 4e-10,
// below float32 rounding), which needs no |w|; dt is folded into 1/m and 1/J
// once per launch (the products are loop-invariant).
__device__ __forceinline__ void integrate(const KConst &c, Drone &d, float Fx, float Fy, float Fz,
                                          float tx, float ty, float tz) {
    const float dtm = c.dt * c.m_inv;
    const float dtjx = c.dt * c.Jx_inv, dtjy = c.dt * c.Jy_inv, dtjz = c.dt * c.Jz_inv;
    const float hdt = 0.5f * c.dt;
    const float Jwx = c.Jx * d.wx, Jwy = c.Jy * d.wy, Jwz = c.Jz * d.wz;
    const float cx = d.wy * Jwz - d.wz * Jwy;
    const float cy = d.wz * Jwx - d.wx * Jwz;
    const float cz = d.wx * Jwy - d.wy * Jwx;
    d.vx += dtm * Fx;
    d.vy += dtm * Fy;
    d.vz += dtm * Fz;
    d.wx += dtjx * (tx - cx);
    d.wy += dtjy * (ty - cy);
    d.wz += dtjz * (tz - cz);
    d.px += c.dt * d.vx;
    d.py += c.dt * d.vy;
    d.pz += c.dt * d.vz;
    const float wn2 = d.wx * d.wx + d.wy * d.wy + d.wz * d.wz;
    const float t2 = (hdt * hdt) * wn2;  // th^2
    const bool small = t2 < 0.0625f;
    // no rotation for a non-finite |w|^2 (neither test holds for NaN)
    if (small || wn2 > 0.f) {
        float co, so;  // cos th, sin(th) / |w|
        if (small) {
            co = 1.f + t2 * (-0.5f + t2 * (1.f / 24.f + t2 * (-1.f / 720.f)));
            so = hdt * (1.f + t2 * (-1.f / 6.f + t2 * (1.f / 120.f + t2 * (-1.f / 5040.f))));
        } else {
            const float wn = fsqrt(wn2);
            float sn;
            sincosf(hdt * wn, &sn, &co);
            so = sn / wn;
        }
        const float rx = so * d.wx, ry = so * d.wy, rz = so * d.wz;
        const float w = d.qw, x = d.qx, y = d.qy, z = d.qz;
        d.qw = w * co - x * rx - y * ry - z * rz;
        d.qx = w * rx + x * co + y * rz - z * ry;
        d.qy = w * ry - x * rz + y * co + z * rx;
        d.qz = w * rz + x * ry - y * rx + z * co;
    }
    const float inv = rsqrtf(d.qw * d.qw + d.qx * d.qx + d.qy * d.qy + d.qz * d.qz);
    d.qw *= inv;
    d.qx *= inv;
    d.qy *= inv;
    d.qz *= inv;
}

// Downwash term of one candidate neighbour j on drone i (Eq. 6) without its
// constant factor K1 = C1 r_p^2 / 16 (applied once to the sum), split in two:
// dw_d2 forms the horizontal distance squared and dw_raw the value
// exp(-dxy^2 / (2 beta^2)) / dz^2 for |dz| = adz > 0, with no gate (at
// adz = 0 it is not finite); dw_term applies the gate dz > 0, dxy < 10 m.
// dx, dy, dz = p_j - p_i are formed from stored positions, so the sign of dz
// and dz == 0 are exact.  The Gaussian is evaluated as 2^(-dxy^2 / beta'^2)
// with beta' = sqrt(2 ln 2) beta (C2, C3 pre-scaled on the host); 1/dz and
// 1/beta'^2 both come from the one reciprocal 1/(dz beta'^2).  beta'^2 + 1e-30
// (one fused multiply-add; the addend is below half an ulp of any
// beta'^2 > 2e-23) reproduces the beta -> 0 limit (1 at dxy = 0, 0 at any
// float-representable dxy > 0) and keeps dz beta'^2 a normal number.  The
// fused multiply-adds are written out, so every sweep rounds alike.
__device__ __forceinline__ float dw_d2(float dx, float dy) { return fmaf(dx, dx, dy * dy); }

template <bool DZMIN>
__device__ __forceinline__ float dw_raw(const KConst &c, float d2, float adz) {
    const float dze = DZMIN ? fmaxf(adz, c.dz_min) : adz;
    const float bs = fmaf(c.C2s, dze, c.C3s);
    const float b2 = fmaf(bs, bs, 1e-30f);
    const float inv = rcp(dze * b2);  // one reciprocal for 1/dz and 1/beta'^2
    const float r = b2 * inv;
    const float gauss = __builtin_amdgcn_exp2f(-d2 * (dze * inv));
    return (r * r) * gauss;
}

__device__ __forceinline__ bool dw_near(float d2) { return d2 < 100.f; }

template <bool DZMIN>
__device__ __forceinline__ float dw_term(const KConst &c, float dx, float dy, float dz) {
    const float d2 = dw_d2(dx, dy);
    const float t = dw_raw<DZMIN>(c, d2, fabsf(dz));
    return (dz > 0.f && dw_near(d2)) ? t : 0.f;
}

// Ground effect (Eq. 4) on the world z force: C_gnd T (r_p / 4 h)^2 with
// h = max(z, h_clip), while the body z axis points up (R33 > 0, equivalent to
// |roll|, |pitch| < pi/2 for Z-Y-X angles).
__device__ __forceinline__ float ground_effect(const KConst &c, const Drone &d, const Rot &R, float T) {
    const float h = fmaxf(d.pz, c.h_clip);
    const float ge = c.K_gnd * T * rcp(h * h);
    return (R.r22 > 0.f) ? ge : 0.f;
}

// Blade drag (Eq. 5) in the world frame: R (-diag(c_xy, c_xy, c_z) S R^T v).
// With e3 = (R02, R12, R22) the body z axis and R R^T = I,
// R diag(c_xy, c_xy, c_z) R^T = c_xy I + (c_z - c_xy) e3 e3^T, so the force is
// -S (c_xy v + (c_z - c_xy) (e3 . v) e3): the same vector, formed without
// rotating v into the body frame and back.
__device__ __forceinline__ void drag(const KConst &c, const Drone &d, const Rot &R, const float n[4],
                                     float &Fx, float &Fy, float &Fz) {
    const float S = c.drag_s * (n[0] + n[1] + n[2] + n[3]);
    const float vb = R.r02 * d.vx + R.r12 * d.vy + R.r22 * d.vz;
    const float a = -S * c.c_xy, b = -S * ((c.c_z - c.c_xy) * vb);
    Fx = a * d.vx + b * R.r02;
    Fy = a * d.vy + b * R.r12;
    Fz = a * d.vz + b * R.r22;
}

}  // namespace phys
}  // namespace md
