// md_rk4.hip -- the persistent step kernel with the classic fourth-order
// Runge-Kutta integrator (the integrator of the paper's MuJoCo physics modes,
// Table "Physics modes") in place of the semi-implicit Euler step.
//
// Per step the rotor speeds (RPM action or a controller update at the step's
// start) and with them the thrust and body torques are held; the rigid-body
// state x = (p, v, q, w) is advanced by x + dt/6 (k1 + 2 k2 + 2 k3 + k4) with
// stages at x, x + dt/2 k1, x + dt/2 k2, x + dt k3.  Every stage evaluates the
// aerodynamic terms (Eq. 4-6) at the stage state; the downwash of a stage
// needs every drone's stage position, so each stage publishes positions to
// LDS (alternating buffers, one barrier per stage).  The time derivative is
//   p' = v, v' = F / m, q' = q (x) [0, w] / 2, w' = J^-1 (tau - w x J w),
// with the rotation of a stage taken from its normalised quaternion; the
// quaternion is renormalised after the step.  One lane per drone; the
// neighbour sweep is the all-pairs or one of the pair-symmetric ones.
#include "md_sweep.h"

namespace md {
namespace {

using namespace phys;

template <uint32_t MASK, int ACT, int UNROLL, int SYM>
__global__ void __launch_bounds__(1024) rk4_kernel(StepArgs a) {
    extern __shared__ float4 lds_pos[];  // [2][2 * slots] positions; then T [slots][tstride] (SYM)
    const KConst &c = a.c;
    const int slots = blockDim.x;
    const int slot = threadIdx.x;
    const int2 tab = a.bins.slot[blockIdx.x * slots + slot];
    const int di = tab.x;
    const bool valid = di >= 0;
    const int lo = tab.y >> 16;
    const int menv = tab.y & 0xffff;
    const int mm_word = a.bins.bin_mmax[blockIdx.x];
    const int mmax = mm_word & 0xffff;
    const bool uniform = (mm_word >> 16) != 0;
    const int N = a.N;

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
        if (ACT >= 1) {
            for (int k = 0; k < 6; ++k) I[k] = a.s.pid_int[k * N + di];
        }
    } else {
        d.qw = 1.f;
    }

    float *tmat = (float *)(lds_pos + 4 * slots);
    if (SYM == 1 && (MASK & 4u) && valid) {
        // the diagonal and the padding up to the next multiple of 4 stay 0
        tmat[slot * a.tstride + (slot - lo)] = 0.f;
        for (int j = menv; j < ((menv + 3) & ~3); ++j) tmat[slot * a.tstride + j] = 0.f;
    }
    const bool held = a.act_step_stride == 0;
    constexpr int ROWS = action_rows(ACT);
    float tgt_held[ROWS];
    float sp[4] = {0.f, 0.f, 0.f, 0.f};
    for (int k = 0; k < ROWS; ++k) tgt_held[k] = 0.f;
    if (ACT >= 1 && held && valid)
        for (int k = 0; k < ROWS; ++k) tgt_held[k] = a.action[(long long)k * N + di];
    if (ACT == 4 && valid)
        for (int k = 0; k < 4; ++k) sp[k] = a.s.ctl[k * N + di];
    int phase = (ACT >= 1) ? (int)(a.step0 % (long long)c.decim) : 0;
    int oslot = 0;
    const float half_dt = 0.5f * c.dt, sixth_dt = c.dt * (1.f / 6.f);
    for (int step = 0; step < a.n_steps; ++step) {
        // ---- rotor speeds, held over the step
        const float *act = a.action + a.act_step_stride * step;
        if (ACT == 0) {
            if (valid) {
                for (int k = 0; k < 4; ++k) n[k] = clampf(act[(long long)k * N + di], 0.f, c.max_rpm);
            }
        } else {
            if (phase == 0 && valid) {
                float cmd[ROWS];
                for (int k = 0; k < ROWS; ++k) cmd[k] = held ? tgt_held[k] : act[(long long)k * N + di];
                control<ACT>(c, d, cmd, I, sp, n);
            }
            phase = (phase + 1 == c.decim) ? 0 : phase + 1;
        }
        float T, tx, ty, tz;
        motor(c, n, T, tx, ty, tz);
        // ---- four stages
        const Drone x0 = d;
        Drone ks{};  // k1 + 2 k2 + 2 k3 + k4
#pragma unroll
        for (int st = 0; st < 4; ++st) {
            float4 *buf = lds_pos + (st & 1) * (2 * slots);
            if (MASK & 4u) {
                if (SYM == 3) {
                    // interleaved uniform bins: each wave's positions twice (128 entries)
                    const int lane = slot & 63;
                    float4 *own = buf + 2 * (slot - lane) + lane;
                    own[0] = own[64] = make_float4(d.px, d.py, d.pz, 0.f);
                } else {
                    buf[slot] = make_float4(d.px, d.py, d.pz, 0.f);
                }
                __syncthreads();
            }
            const float qi = rsqrtf(d.qw * d.qw + d.qx * d.qx + d.qy * d.qy + d.qz * d.qz);
            Drone dn = d;
            dn.qw *= qi;
            dn.qx *= qi;
            dn.qy *= qi;
            dn.qz *= qi;
            const Rot R = rot_of(dn);
            float Fx = R.r02 * T, Fy = R.r12 * T, Fz = R.r22 * T - c.mg;
            if (MASK & 1u) Fz += ground_effect(c, dn, R, T);
            if (MASK & 2u) {
                float dx, dy, dz;
                drag(c, dn, R, n, dx, dy, dz);
                Fx += dx;
                Fy += dy;
                Fz += dz;
            }
            if (MASK & 4u)
                Fz -= c.K1 * dw_sum<1, UNROLL, SYM>(c, buf, tmat, a.tstride, slot, 0, lo, mmax, menv, uniform, d);
            // time derivative k of the stage
            Drone k;
            k.px = d.vx;
            k.py = d.vy;
            k.pz = d.vz;
            k.vx = Fx * c.m_inv;
            k.vy = Fy * c.m_inv;
            k.vz = Fz * c.m_inv;
            k.qw = 0.5f * (-d.qx * d.wx - d.qy * d.wy - d.qz * d.wz);
            k.qx = 0.5f * (d.qw * d.wx + d.qy * d.wz - d.qz * d.wy);
            k.qy = 0.5f * (d.qw * d.wy - d.qx * d.wz + d.qz * d.wx);
            k.qz = 0.5f * (d.qw * d.wz + d.qx * d.wy - d.qy * d.wx);
            const float Jwx = c.Jx * d.wx, Jwy = c.Jy * d.wy, Jwz = c.Jz * d.wz;
            k.wx = (tx - (d.wy * Jwz - d.wz * Jwy)) * c.Jx_inv;
            k.wy = (ty - (d.wz * Jwx - d.wx * Jwz)) * c.Jy_inv;
            k.wz = (tz - (d.wx * Jwy - d.wy * Jwx)) * c.Jz_inv;
            const float wgt = (st == 0 || st == 3) ? 1.f : 2.f;
            const float h = (st < 2) ? half_dt : c.dt;
#define MD_RK_FIELD(f)              \
    ks.f += wgt * k.f;              \
    if (st < 3) d.f = x0.f + h * k.f;
            MD_RK_FIELD(px) MD_RK_FIELD(py) MD_RK_FIELD(pz)
            MD_RK_FIELD(vx) MD_RK_FIELD(vy) MD_RK_FIELD(vz)
            MD_RK_FIELD(qw) MD_RK_FIELD(qx) MD_RK_FIELD(qy) MD_RK_FIELD(qz)
            MD_RK_FIELD(wx) MD_RK_FIELD(wy) MD_RK_FIELD(wz)
#undef MD_RK_FIELD
        }
#define MD_RK_FINAL(f) d.f = x0.f + sixth_dt * ks.f;
        MD_RK_FINAL(px) MD_RK_FINAL(py) MD_RK_FINAL(pz)
        MD_RK_FINAL(vx) MD_RK_FINAL(vy) MD_RK_FINAL(vz)
        MD_RK_FINAL(qw) MD_RK_FINAL(qx) MD_RK_FINAL(qy) MD_RK_FINAL(qz)
        MD_RK_FINAL(wx) MD_RK_FINAL(wy) MD_RK_FINAL(wz)
#undef MD_RK_FINAL
        const float qi = rsqrtf(d.qw * d.qw + d.qx * d.qx + d.qy * d.qy + d.qz * d.qz);
        d.qw *= qi;
        d.qx *= qi;
        d.qy *= qi;
        d.qz *= qi;
        // ---- KIN observation
        if (a.obs != nullptr && valid) {
            float roll, pitch, yaw;
            euler_zyx(d, roll, pitch, yaw);
            const float row[20] = {d.px, d.py, d.pz, d.qw, d.qx, d.qy, d.qz, roll, pitch, yaw,
                                   d.vx, d.vy, d.vz, d.wx, d.wy, d.wz, n[0], n[1], n[2], n[3]};
            store_obs(a.obs, oslot, N, di, row);
        }
        oslot = (oslot + 1 == a.n_obs_slots) ? 0 : oslot + 1;
    }

    if (valid) {
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
        if (ACT >= 1) {
            for (int k = 0; k < 6; ++k) a.s.pid_int[k * N + di] = I[k];
        }
        if (ACT == 4)
            for (int k = 0; k < 4; ++k) a.s.ctl[k * N + di] = sp[k];
    }
}

template <uint32_t MASK, int ACT, int SYM>
hipError_t launch_u(const StepArgs &a, int unroll, int n_bins, int threads, size_t lds, hipStream_t st) {
    switch (unroll) {
        case 1: hipLaunchKernelGGL((rk4_kernel<MASK, ACT, 1, SYM>), dim3(n_bins), dim3(threads), lds, st, a); break;
        case 2: hipLaunchKernelGGL((rk4_kernel<MASK, ACT, 2, SYM>), dim3(n_bins), dim3(threads), lds, st, a); break;
        case 4: hipLaunchKernelGGL((rk4_kernel<MASK, ACT, 4, SYM>), dim3(n_bins), dim3(threads), lds, st, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <uint32_t MASK, int ACT>
hipError_t launch_l(const StepArgs &a, const LaunchCfg &cfg, int n_bins, int threads, size_t lds,
                    hipStream_t st) {
    if (!(MASK & 4u)) {
        hipLaunchKernelGGL((rk4_kernel<MASK, ACT, 1, 0>), dim3(n_bins), dim3(threads), lds, st, a);
        return hipGetLastError();
    }
    if (cfg.lpd != 1) return hipErrorInvalidValue;
    switch (cfg.sym) {
        case 0: return launch_u<MASK, ACT, 0>(a, cfg.unroll, n_bins, threads, lds, st);
        case 1: return launch_u<MASK, ACT, 1>(a, cfg.unroll, n_bins, threads, lds, st);
        case 2:
        case 3:
            // the rotation sweep is unrolled in full, the permute sweep not at
            // all (see cfg_valid): one instantiation each
            if (cfg.unroll != 1) return hipErrorInvalidValue;
            if (cfg.sym == 3)
                hipLaunchKernelGGL((rk4_kernel<MASK, ACT, 1, 3>), dim3(n_bins), dim3(threads), lds, st, a);
            else
                hipLaunchKernelGGL((rk4_kernel<MASK, ACT, 1, 2>), dim3(n_bins), dim3(threads), lds, st, a);
            return hipGetLastError();
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

hipError_t launch_step_rk4(const StepArgs &a, uint32_t mask, int act, const LaunchCfg &cfg,
                           int n_bins, int slots, hipStream_t stream) {
    if (n_bins <= 0 || a.n_steps <= 0) return hipSuccess;
    if ((mask & 4u) && cfg.lpd != 1) return hipErrorInvalidValue;
    const int threads = slots;
    size_t lds = (mask & 4u) ? sizeof(float4) * 2 * 2 * (size_t)slots : 0;
    if ((mask & 4u) && cfg.sym == 1) lds += sizeof(float) * (size_t)slots * (size_t)a.tstride;
    switch (act) {
        case 0: return launch_m<0>(a, mask, cfg, n_bins, threads, lds, stream);
        case 1: return launch_m<1>(a, mask, cfg, n_bins, threads, lds, stream);
        case 2: return launch_m<2>(a, mask, cfg, n_bins, threads, lds, stream);
        case 3: return launch_m<3>(a, mask, cfg, n_bins, threads, lds, stream);
        default: return launch_m<4>(a, mask, cfg, n_bins, threads, lds, stream);
    }
}

}  // namespace md
