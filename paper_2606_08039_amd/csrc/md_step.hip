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
#include "md_physics.h"

namespace md {
namespace {

using namespace phys;

// This lane's share of the downwash sum over its environment's slots
// [lo, lo + mmax), in ascending order (every LPD-th slot from `sub`).  In a
// uniform bin every environment has mmax drones and the bound check is
// dropped.
template <bool DZMIN, int LPD, int UNROLL>
__device__ __forceinline__ float dw_sweep(const KConst &c, const float4 *buf, int lo, int sub, int mmax,
                                          int menv, bool uniform, const Drone &d) {
    float acc = 0.f;
    if (uniform) {
#pragma unroll UNROLL
        for (int j = sub; j < mmax; j += LPD) {
            const float4 pj = buf[lo + j];
            acc += dw_term<DZMIN>(c, pj.x - d.px, pj.y - d.py, pj.z - d.pz);
        }
    } else {
#pragma unroll UNROLL
        for (int j = sub; j < mmax; j += LPD) {
            const float4 pj = buf[lo + j];
            const float term = dw_term<DZMIN>(c, pj.x - d.px, pj.y - d.py, pj.z - d.pz);
            acc += (j < menv) ? term : 0.f;
        }
    }
    return acc;
}

// Pair-symmetric downwash sweep: each unordered pair of an environment is
// evaluated once, by lane i for partners (i + d) mod M, d = 1..(M-1)/2, plus
// d = M/2 from the lower half when M is even.  The term goes to the lower
// drone's row of the LDS matrix T (the other entry gets 0); after a barrier
// each drone sums its row in ascending order.  The term depends only on
// dxy^2 and |dz|, and fl(a - b) = -fl(b - a), so every entry and the sum are
// bitwise those of the all-pairs sweep.
template <bool DZMIN, int UNROLL>
__device__ __forceinline__ void dw_pairs(const KConst &c, const float4 *buf, float *T, int ts, int slot,
                                         int lo, int m, const Drone &d) {
    const int li = slot - lo;
    const int h = (m - 1) >> 1;
#pragma unroll UNROLL
    for (int k = 1; k <= h; ++k) {
        int lj = li + k;
        lj -= (lj >= m) ? m : 0;
        const float4 pj = buf[lo + lj];
        const float dz = pj.z - d.pz;
        const float t = dw_term<DZMIN>(c, pj.x - d.px, pj.y - d.py, fabsf(dz));
        T[slot * ts + lj] = dz > 0.f ? t : 0.f;
        T[(lo + lj) * ts + li] = dz < 0.f ? t : 0.f;
    }
    if ((m & 1) == 0 && li < (m >> 1) && m > 0) {
        const int lj = li + (m >> 1);
        const float4 pj = buf[lo + lj];
        const float dz = pj.z - d.pz;
        const float t = dw_term<DZMIN>(c, pj.x - d.px, pj.y - d.py, fabsf(dz));
        T[slot * ts + lj] = dz > 0.f ? t : 0.f;
        T[(lo + lj) * ts + li] = dz < 0.f ? t : 0.f;
    }
}

template <uint32_t MASK, int ACT, int LPD, int UNROLL, bool SYM>
__global__ void __launch_bounds__(1024) step_kernel(StepArgs a) {
    extern __shared__ float4 lds_pos[];  // [2][2 * slots] positions; then T [slots][tstride] (SYM)
    const KConst &c = a.c;
    const int slots = blockDim.x / LPD;
    const int slot = threadIdx.x / LPD;
    const int sub = threadIdx.x - slot * LPD;
    const int2 tab = a.bins.slot[blockIdx.x * slots + slot];
    const int di = tab.x;
    const bool valid = di >= 0;
    const int lo = tab.y >> 16;
    const int menv = tab.y & 0xffff;
    const int mm_word = a.bins.bin_mmax[blockIdx.x];
    const int mmax = mm_word & 0xffff;
    const bool uniform = (mm_word >> 16) != 0;
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
        if (ACT >= 1) {
            for (int k = 0; k < 6; ++k) I[k] = a.s.pid_int[k * N + di];
        }
    } else {
        d.qw = 1.f;
    }

    float *tmat = (float *)(lds_pos + 4 * slots);
    if (SYM && (MASK & 4u)) tmat[slot * a.tstride + (slot - lo)] = 0.f;  // the diagonal stays 0
    // Held waypoints (one action row for the whole launch) stay in registers:
    // re-reading them at every PID update would fetch them from HBM again,
    // since the observation stream evicts them from L2.
    const bool held = a.act_step_stride == 0;
    constexpr int ROWS = action_rows(ACT);
    float tgt_held[ROWS];
    float sp[4] = {0.f, 0.f, 0.f, 0.f};
    for (int k = 0; k < ROWS; ++k) tgt_held[k] = 0.f;
    if (ACT >= 1 && held && valid)
        for (int k = 0; k < ROWS; ++k) tgt_held[k] = a.action[(long long)k * N + di];
    if (ACT == 4 && valid)
        for (int k = 0; k < 4; ++k) sp[k] = a.s.ctl[k * N + di];
    // PID phase and observation slot advance as counters (no per-step division)
    int phase = (ACT >= 1) ? (int)(a.step0 % (long long)c.decim) : 0;
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
                float cmd[ROWS];
                for (int k = 0; k < ROWS; ++k) cmd[k] = held ? tgt_held[k] : act[(long long)k * N + di];
                control<ACT>(c, d, cmd, I, sp, n);
            }
            phase = (phase + 1 == c.decim) ? 0 : phase + 1;
        }
        // ---- motor model and mixer (Eq. 1-3)
        float T, tx, ty, tz;
        motor(c, n, T, tx, ty, tz);
        const Rot R = rot_of(d);
        float Fx = R.r02 * T, Fy = R.r12 * T, Fz = R.r22 * T - c.mg;
        // ---- ground effect (Eq. 4)
        if (MASK & 1u) Fz += ground_effect(c, d, R, T);
        // ---- blade drag (Eq. 5)
        if (MASK & 2u) {
            float dx, dy, dz;
            drag(c, d, R, n, dx, dy, dz);
            Fx += dx;
            Fy += dy;
            Fz += dz;
        }
        // ---- downwash (Eq. 6): sweep the environment in ascending order
        if (MASK & 4u) {
            float acc = 0.f;
            if (SYM) {
                if (c.dz_min > 0.f)
                    dw_pairs<true, UNROLL>(c, buf, tmat, a.tstride, slot, lo, menv, d);
                else
                    dw_pairs<false, UNROLL>(c, buf, tmat, a.tstride, slot, lo, menv, d);
                __syncthreads();
                const float *row = tmat + slot * a.tstride;
                for (int j = 0; j < menv; ++j) acc += row[j];
            } else if (c.dz_min > 0.f) {
                acc = dw_sweep<true, LPD, UNROLL>(c, buf, lo, sub, mmax, menv, uniform, d);
            } else {
                acc = dw_sweep<false, LPD, UNROLL>(c, buf, lo, sub, mmax, menv, uniform, d);
            }
            if (LPD >= 2) {
                const float o = __shfl_xor(acc, 1, 64);
                acc = (sub & 1) ? (o + acc) : (acc + o);
            }
            if (LPD >= 4) {
                const float o = __shfl_xor(acc, 2, 64);
                acc = (sub & 2) ? (o + acc) : (acc + o);
            }
            Fz -= c.K1 * acc;
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
        if (ACT >= 1) {
            for (int k = 0; k < 6; ++k) a.s.pid_int[k * N + di] = I[k];
        }
        if (ACT == 4)
            for (int k = 0; k < 4; ++k) a.s.ctl[k * N + di] = sp[k];
    }
}

template <uint32_t MASK, int ACT, int LPD, bool SYM>
hipError_t launch_u(const StepArgs &a, int unroll, int n_bins, int threads, size_t lds, hipStream_t st) {
    switch (unroll) {
        case 1: hipLaunchKernelGGL((step_kernel<MASK, ACT, LPD, 1, SYM>), dim3(n_bins), dim3(threads), lds, st, a); break;
        case 2: hipLaunchKernelGGL((step_kernel<MASK, ACT, LPD, 2, SYM>), dim3(n_bins), dim3(threads), lds, st, a); break;
        case 4: hipLaunchKernelGGL((step_kernel<MASK, ACT, LPD, 4, SYM>), dim3(n_bins), dim3(threads), lds, st, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <uint32_t MASK, int ACT>
hipError_t launch_l(const StepArgs &a, const LaunchCfg &cfg, int n_bins, int threads, size_t lds,
                    hipStream_t st) {
    if (!(MASK & 4u)) {
        // no neighbour sweep: one lane per drone, no loop to tune
        hipLaunchKernelGGL((step_kernel<MASK, ACT, 1, 1, false>), dim3(n_bins), dim3(threads), lds, st, a);
        return hipGetLastError();
    }
    if (cfg.sym) {
        if (cfg.lpd != 1) return hipErrorInvalidValue;
        return launch_u<MASK, ACT, 1, true>(a, cfg.unroll, n_bins, threads, lds, st);
    }
    switch (cfg.lpd) {
        case 1: return launch_u<MASK, ACT, 1, false>(a, cfg.unroll, n_bins, threads, lds, st);
        case 2: return launch_u<MASK, ACT, 2, false>(a, cfg.unroll, n_bins, threads, lds, st);
        case 4: return launch_u<MASK, ACT, 4, false>(a, cfg.unroll, n_bins, threads, lds, st);
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
    size_t lds = (mask & 4u) ? sizeof(float4) * 2 * 2 * (size_t)slots : 0;
    if ((mask & 4u) && cfg.sym) lds += sizeof(float) * (size_t)slots * (size_t)a.tstride;
    switch (act) {
        case 0: return launch_m<0>(a, mask, cfg, n_bins, threads, lds, stream);
        case 1: return launch_m<1>(a, mask, cfg, n_bins, threads, lds, stream);
        case 2: return launch_m<2>(a, mask, cfg, n_bins, threads, lds, stream);
        case 3: return launch_m<3>(a, mask, cfg, n_bins, threads, lds, stream);
        default: return launch_m<4>(a, mask, cfg, n_bins, threads, lds, stream);
    }
}

}  // namespace md
