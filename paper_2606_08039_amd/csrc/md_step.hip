// md_step.hip -- the persistent, ragged-batched explicit quadrotor step (gfx950).
//
// One workgroup runs one bin: a set of whole environments packed into its
// slots.  A drone's state lives in registers for all n_steps of the launch;
// HBM sees the state once in and once out, the per-step actions (RPM mode)
// and the per-step observation rows.  Positions are published to LDS every
// step (double buffered, one barrier per step) so that each drone can sweep
// its environment for the pairwise downwash of Eq. 6.
//
// Physics per step (paper: Sec. "Quadrotor Dynamics", Sec. "Physics Modes"):
//   rotor speeds   RPM action clipped to [0, MAX_RPM] or cascaded PID (Sec. "Control")
//   motor model    F_i = kf n_i^2, X-mixer torques, yaw reaction torques     (Eq. 1-3)
//   ground effect  C_gnd T (r_p / 4 max(z, h_clip))^2 while the body z axis points up (Eq. 4)
//   drag           R (-diag(c_xy, c_xy, c_z) (sum 2 pi n_i / 60) R^T v)    (Eq. 5)
//   downwash       sum over higher drones j of -C1 (r_p/4dz)^2 exp(-(dxy/beta)^2/2) (Eq. 6)
//   integrator     semi-implicit Euler, body-rate exponential map, renormalise (Eq. 7)
#include "md_internal.h"

namespace md {
namespace {

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

__device__ __forceinline__ Rot rot_of(const Drone &d) {
    const float w = d.qw, x = d.qx, y = d.qy, z = d.qz;
    Rot R;
    R.r00 = 1.f - 2.f * (y * y + z * z);
    R.r01 = 2.f * (x * y - w * z);
    R.r02 = 2.f * (x * z + w * y);
    R.r10 = 2.f * (x * y + w * z);
    R.r11 = 1.f - 2.f * (x * x + z * z);
    R.r12 = 2.f * (y * z - w * x);
    R.r20 = 2.f * (x * z - w * y);
    R.r21 = 2.f * (y * z + w * x);
    R.r22 = 1.f - 2.f * (x * x + y * y);
    return R;
}

// Roll, pitch, yaw (Z-Y-X) of the KIN observation.
__device__ __forceinline__ void euler_zyx(const Drone &d, float &roll, float &pitch, float &yaw) {
    const float w = d.qw, x = d.qx, y = d.qy, z = d.qz;
    float sp = 2.f * (w * y - z * x);
    sp = fminf(fmaxf(sp, -1.f), 1.f);
    roll = atan2f(2.f * (w * x + y * z), 1.f - 2.f * (x * x + y * y));
    pitch = asinf(sp);
    yaw = atan2f(2.f * (w * z + x * y), 1.f - 2.f * (y * y + z * z));
}

__device__ __forceinline__ float clampf(float x, float lo, float hi) {
    return fminf(fmaxf(x, lo), hi);
}

// Cascaded PID of Sec. "Control" (position loop -> thrust and small-angle
// attitude target -> attitude PID -> exact allocation inverse, rotor forces
// clipped to [0, kf MAX_RPM^2]).
__device__ __forceinline__ void pid_update(const KConst &c, const Drone &d, const float tgt[4],
                                           float I[6], float n[4]) {
    const float ex = tgt[0] - d.px, ey = tgt[1] - d.py, ez = tgt[2] - d.pz;
    I[0] = clampf(I[0] + ex * c.dt_c, -c.p_clamp, c.p_clamp);
    I[1] = clampf(I[1] + ey * c.dt_c, -c.p_clamp, c.p_clamp);
    I[2] = clampf(I[2] + ez * c.dt_c, -c.p_clamp, c.p_clamp);
    const float ax = c.pkp[0] * ex + c.pki[0] * I[0] - c.pkd[0] * d.vx;
    const float ay = c.pkp[1] * ey + c.pki[1] * I[1] - c.pkd[1] * d.vy;
    const float az = c.pkp[2] * ez + c.pki[2] * I[2] - c.pkd[2] * d.vz + c.g;
    const float T = c.m * sqrtf(ax * ax + ay * ay + az * az);

    const float w = d.qw, x = d.qx, y = d.qy, z = d.qz;
    float sp = clampf(2.f * (w * y - z * x), -1.f, 1.f);
    const float roll = atan2f(2.f * (w * x + y * z), 1.f - 2.f * (x * x + y * y));
    const float pitch = asinf(sp);
    const float ys = 2.f * (w * z + x * y), yc = 1.f - 2.f * (y * y + z * z);
    const float yaw = atan2f(ys, yc);
    // sin and cos of the yaw straight from the atan2 arguments
    const float h2 = ys * ys + yc * yc;
    const float hinv = h2 > 0.f ? rsqrtf(h2) : 0.f;
    const float sps = h2 > 0.f ? ys * hinv : 0.f;
    const float cps = h2 > 0.f ? yc * hinv : 1.f;

    const float roll_t = (ax * sps - ay * cps) * c.g_inv;
    const float pitch_t = (ax * cps + ay * sps) * c.g_inv;
    float dyaw = tgt[3] - yaw;
    dyaw = dyaw - kTwoPi * floorf((dyaw + kPi) * (1.f / kTwoPi));
    const float er = roll_t - roll, ep = pitch_t - pitch;
    I[3] = clampf(I[3] + er * c.dt_c, -c.a_clamp, c.a_clamp);
    I[4] = clampf(I[4] + ep * c.dt_c, -c.a_clamp, c.a_clamp);
    I[5] = clampf(I[5] + dyaw * c.dt_c, -c.a_clamp, c.a_clamp);
    const float tx = c.akp[0] * er + c.aki[0] * I[3] - c.akd[0] * d.wx;
    const float ty = c.akp[1] * ep + c.aki[1] * I[4] - c.akd[1] * d.wy;
    const float tz = c.akp[2] * dyaw + c.aki[2] * I[5] - c.akd[2] * d.wz;

    const float a = tx * c.l_inv, b = ty * c.l_inv, e = tz * c.kappa_inv;
    const float F0 = 0.25f * (T + a - b - e);
    const float F1 = 0.25f * (T + a + b + e);
    const float F2 = 0.25f * (T - a + b - e);
    const float F3 = 0.25f * (T - a - b + e);
    n[0] = sqrtf(clampf(F0, 0.f, c.fmax) * c.kf_inv);
    n[1] = sqrtf(clampf(F1, 0.f, c.fmax) * c.kf_inv);
    n[2] = sqrtf(clampf(F2, 0.f, c.fmax) * c.kf_inv);
    n[3] = sqrtf(clampf(F3, 0.f, c.fmax) * c.kf_inv);
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
// from their Taylor series (truncation error < 4e-10, below float32 rounding).
__device__ __forceinline__ void integrate(const KConst &c, Drone &d, float Fx, float Fy, float Fz,
                                          float tx, float ty, float tz) {
    const float Jwx = c.Jx * d.wx, Jwy = c.Jy * d.wy, Jwz = c.Jz * d.wz;
    const float cx = d.wy * Jwz - d.wz * Jwy;
    const float cy = d.wz * Jwx - d.wx * Jwz;
    const float cz = d.wx * Jwy - d.wy * Jwx;
    d.vx += c.dt * (Fx * c.m_inv);
    d.vy += c.dt * (Fy * c.m_inv);
    d.vz += c.dt * (Fz * c.m_inv);
    d.wx += c.dt * ((tx - cx) * c.Jx_inv);
    d.wy += c.dt * ((ty - cy) * c.Jy_inv);
    d.wz += c.dt * ((tz - cz) * c.Jz_inv);
    d.px += c.dt * d.vx;
    d.py += c.dt * d.vy;
    d.pz += c.dt * d.vz;
    const float wn2 = d.wx * d.wx + d.wy * d.wy + d.wz * d.wz;
    if (wn2 > 0.f) {
        const float wn = sqrtf(wn2);
        const float th = 0.5f * c.dt * wn;
        float co, so;  // cos th, sin(th) / |w|
        if (th < 0.25f) {
            const float t2 = th * th;
            co = 1.f + t2 * (-0.5f + t2 * (1.f / 24.f + t2 * (-1.f / 720.f)));
            so = 0.5f * c.dt * (1.f + t2 * (-1.f / 6.f + t2 * (1.f / 120.f + t2 * (-1.f / 5040.f))));
        } else {
            float sn;
            sincosf(th, &sn, &co);
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

// Downwash term of one candidate neighbour j on drone i (Eq. 6), given the
// coordinate differences dx, dy, dz = p_j - p_i formed from stored positions
// (so the sign of dz, and dz == 0, are exact).  Returns 0 unless dz > 0 and
// dxy < 10 m.
__device__ __forceinline__ float dw_term(const KConst &c, float dx, float dy, float dz) {
    const float d2 = dx * dx + dy * dy;
    const float dze = fmaxf(dz, c.dz_min);
    const float r = rcp(dze);
    const float alpha = c.K1 * (r * r);
    const float beta = c.C2 * dze + c.C3;
    const float b2 = beta * beta;
    // exp(-dxy^2 / (2 beta^2)); the limit for beta -> 0 is 1 at dxy = 0, else 0
    const float t = (d2 == 0.f) ? 0.f : (-0.5f * d2) * rcp(b2);
    const float gauss = __expf(t);
    const bool on = (dz > 0.f) && (d2 < 100.f);
    return on ? alpha * gauss : 0.f;
}

template <uint32_t MASK, int ACT, int LPD, int UNROLL>
__global__ void __launch_bounds__(1024) step_kernel(StepArgs a) {
    extern __shared__ float4 lds_pos[];  // [2][2 * slots]: double-buffered, padded
    const KConst &c = a.c;
    const int slots = blockDim.x / LPD;
    const int slot = threadIdx.x / LPD;
    const int sub = threadIdx.x - slot * LPD;
    const int2 tab = a.bins.slot[blockIdx.x * slots + slot];
    const int di = tab.x;
    const bool valid = di >= 0;
    const int lo = tab.y >> 16;
    const int menv = tab.y & 0xffff;
    const int mmax = a.bins.bin_mmax[blockIdx.x];
    const int N = a.N;
    const bool writer = valid && (sub == 0);

    Drone d{};
    float I[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    float n[4] = {0.f, 0.f, 0.f, 0.f};
    if (valid) {
        d.px = a.s.p[di];
        d.py = a.s.p[N + di];
        d.pz = a.s.p[2 * N + di];
        d.qw = a.s.q[di];
        d.qx = a.s.q[N + di];
        d.qy = a.s.q[2 * N + di];
        d.qz = a.s.q[3 * N + di];
        d.vx = a.s.v[di];
        d.vy = a.s.v[N + di];
        d.vz = a.s.v[2 * N + di];
        d.wx = a.s.w[di];
        d.wy = a.s.w[N + di];
        d.wz = a.s.w[2 * N + di];
        for (int k = 0; k < 4; ++k) n[k] = a.s.rpm[k * N + di];
        if (ACT == 1) {
            for (int k = 0; k < 6; ++k) I[k] = a.s.pid_int[k * N + di];
        }
    } else {
        d.qw = 1.f;
    }

    // PID phase and observation slot advance as counters (no per-step division)
    int phase = (ACT == 1) ? (int)(a.step0 % (long long)c.decim) : 0;
    int oslot = 0;
    for (int step = 0; step < a.n_steps; ++step) {
        float4 *buf = lds_pos + (step & 1) * (2 * slots);
        if (MASK & 4u) {
            if (sub == 0) buf[slot] = make_float4(d.px, d.py, d.pz, 0.f);
            __syncthreads();
        }
        // ---- rotor speeds
        const float *act = a.action + a.act_step_stride * step;
        if (ACT == 0) {
            if (valid) {
                for (int k = 0; k < 4; ++k) n[k] = clampf(act[(long long)k * N + di], 0.f, c.max_rpm);
            }
        } else {
            if (phase == 0 && valid) {
                float tgt[4];
                for (int k = 0; k < 4; ++k) tgt[k] = act[(long long)k * N + di];
                pid_update(c, d, tgt, I, n);
            }
            phase = (phase + 1 == c.decim) ? 0 : phase + 1;
        }
        // ---- motor model and mixer (Eq. 1-3)
        float T, tx, ty, tz;
        motor(c, n, T, tx, ty, tz);
        const Rot R = rot_of(d);
        float Fx = R.r02 * T, Fy = R.r12 * T, Fz = R.r22 * T - c.mg;
        // ---- ground effect (Eq. 4)
        if (MASK & 1u) {
            const float h = fmaxf(d.pz, c.h_clip);
            const float ge = c.K_gnd * T * rcp(h * h);
            Fz += (R.r22 > 0.f) ? ge : 0.f;
        }
        // ---- blade drag (Eq. 5)
        if (MASK & 2u) {
            const float S = c.drag_s * (n[0] + n[1] + n[2] + n[3]);
            const float bx = R.r00 * d.vx + R.r10 * d.vy + R.r20 * d.vz;
            const float by = R.r01 * d.vx + R.r11 * d.vy + R.r21 * d.vz;
            const float bz = R.r02 * d.vx + R.r12 * d.vy + R.r22 * d.vz;
            const float fx = -c.c_xy * S * bx, fy = -c.c_xy * S * by, fz = -c.c_z * S * bz;
            Fx += R.r00 * fx + R.r01 * fy + R.r02 * fz;
            Fy += R.r10 * fx + R.r11 * fy + R.r12 * fz;
            Fz += R.r20 * fx + R.r21 * fy + R.r22 * fz;
        }
        // ---- downwash (Eq. 6): sweep the environment in ascending order
        if (MASK & 4u) {
            float acc = 0.f;
#pragma unroll UNROLL
            for (int j = sub; j < mmax; j += LPD) {
                const float4 pj = buf[lo + j];
                const float term = dw_term(c, pj.x - d.px, pj.y - d.py, pj.z - d.pz);
                acc += (j < menv) ? term : 0.f;
            }
            if (LPD >= 2) {
                const float o = __shfl_xor(acc, 1, 64);
                acc = (sub & 1) ? (o + acc) : (acc + o);
            }
            if (LPD >= 4) {
                const float o = __shfl_xor(acc, 2, 64);
                acc = (sub & 2) ? (o + acc) : (acc + o);
            }
            Fz -= acc;
        }
        // ---- Newton-Euler + exponential map (Eq. 7)
        integrate(c, d, Fx, Fy, Fz, tx, ty, tz);
        // ---- KIN observation
        if (a.obs != nullptr && writer) {
            float roll, pitch, yaw;
            euler_zyx(d, roll, pitch, yaw);
            float *o = a.obs + (long long)oslot * 20 * N + di;
            const float row[20] = {d.px, d.py, d.pz, d.qw, d.qx, d.qy, d.qz, roll, pitch, yaw,
                                   d.vx, d.vy, d.vz, d.wx, d.wy, d.wz, n[0], n[1], n[2], n[3]};
#pragma unroll
            for (int k = 0; k < 20; ++k) o[(long long)k * N] = row[k];
        }
        oslot = (oslot + 1 == a.n_obs_slots) ? 0 : oslot + 1;
    }

    if (writer) {
        a.s.p[di] = d.px;
        a.s.p[N + di] = d.py;
        a.s.p[2 * N + di] = d.pz;
        a.s.q[di] = d.qw;
        a.s.q[N + di] = d.qx;
        a.s.q[2 * N + di] = d.qy;
        a.s.q[3 * N + di] = d.qz;
        a.s.v[di] = d.vx;
        a.s.v[N + di] = d.vy;
        a.s.v[2 * N + di] = d.vz;
        a.s.w[di] = d.wx;
        a.s.w[N + di] = d.wy;
        a.s.w[2 * N + di] = d.wz;
        for (int k = 0; k < 4; ++k) a.s.rpm[k * N + di] = n[k];
        if (ACT == 1) {
            for (int k = 0; k < 6; ++k) a.s.pid_int[k * N + di] = I[k];
        }
    }
}

template <uint32_t MASK, int ACT, int LPD>
hipError_t launch_u(const StepArgs &a, int unroll, int n_bins, int threads, size_t lds,
                    hipStream_t st) {
    switch (unroll) {
        case 1: hipLaunchKernelGGL((step_kernel<MASK, ACT, LPD, 1>), dim3(n_bins), dim3(threads), lds, st, a); break;
        case 2: hipLaunchKernelGGL((step_kernel<MASK, ACT, LPD, 2>), dim3(n_bins), dim3(threads), lds, st, a); break;
        case 4: hipLaunchKernelGGL((step_kernel<MASK, ACT, LPD, 4>), dim3(n_bins), dim3(threads), lds, st, a); break;
        case 8: hipLaunchKernelGGL((step_kernel<MASK, ACT, LPD, 8>), dim3(n_bins), dim3(threads), lds, st, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <uint32_t MASK, int ACT>
hipError_t launch_l(const StepArgs &a, const LaunchCfg &cfg, int n_bins, int threads, size_t lds,
                    hipStream_t st) {
    if (!(MASK & 4u)) {
        // no neighbour sweep: one lane per drone, no unrolled loop to tune
        return launch_u<MASK, ACT, 1>(a, 1, n_bins, threads, lds, st);
    }
    switch (cfg.lpd) {
        case 1: return launch_u<MASK, ACT, 1>(a, cfg.unroll, n_bins, threads, lds, st);
        case 2: return launch_u<MASK, ACT, 2>(a, cfg.unroll, n_bins, threads, lds, st);
        case 4: return launch_u<MASK, ACT, 4>(a, cfg.unroll, n_bins, threads, lds, st);
        default: return hipErrorInvalidValue;
    }
}

template <int ACT>
hipError_t launch_m(const StepArgs &a, uint32_t mask, const LaunchCfg &cfg, int n_bins,
                    int threads, size_t lds, hipStream_t st) {
    switch (mask & 7u) {
        case 0: return launch_l<0, ACT>(a, cfg, n_bins, threads, lds, st);
        case 1: return launch_l<1, ACT>(a, cfg, n_bins, threads, lds, st);
        case 2: return launch_l<2, ACT>(a, cfg, n_bins, threads, lds, st);
        case 3: return launch_l<3, ACT>(a, cfg, n_bins, threads, lds, st);
        case 4: return launch_l<4, ACT>(a, cfg, n_bins, threads, lds, st);
        case 5: return launch_l<5, ACT>(a, cfg, n_bins, threads, lds, st);
        case 6: return launch_l<6, ACT>(a, cfg, n_bins, threads, lds, st);
        default: return launch_l<7, ACT>(a, cfg, n_bins, threads, lds, st);
    }
}

}  // namespace

hipError_t launch_step(const StepArgs &a, uint32_t mask, int act, const LaunchCfg &cfg,
                       int n_bins, int slots, hipStream_t stream) {
    if (n_bins <= 0 || a.n_steps <= 0) return hipSuccess;
    const int lpd = (mask & 4u) ? cfg.lpd : 1;
    const int threads = slots * lpd;
    const size_t lds = (mask & 4u) ? sizeof(float4) * 2 * 2 * (size_t)slots : 0;
    if (act == 0) return launch_m<0>(a, mask, cfg, n_bins, threads, lds, stream);
    return launch_m<1>(a, mask, cfg, n_bins, threads, lds, stream);
}

}  // namespace md
