// md_step_kernel.h -- the persistent, ragged-batched explicit quadrotor step
// (gfx950), instantiated without domain randomisation in md_step.hip and
// with it in md_step_dr.hip.
//
// One workgroup runs one bin: a set of whole environments packed into its
// slots.  A drone's state lives in registers for all n_steps of the launch;
// HBM sees the state once in and once out, the per-step actions (RPM mode)
// and the per-step observation rows.  Positions are published to LDS every
// step (double buffered, one barrier per step) so that each drone can sweep
// its environment for the pairwise downwash of Eq. 6 with one of the sweeps
// of md_sweep.h.
//
// Physics per step (paper: Sec. "Quadrotor Dynamics", Sec. "Physics Modes"):
//   rotor speeds   RPM action clipped to [0, MAX_RPM] or a controller (Sec. "Control")
//   motor model    F_i = kf n_i^2, X-mixer torques, yaw reaction torques     (Eq. 1-3)
//   ground effect  C_gnd T (r_p / 4 max(z, h_clip))^2 while the body z axis points up (Eq. 4)
//   drag           R (-diag(c_xy, c_xy, c_z) (sum 2 pi n_i / 60) R^T v)    (Eq. 5)
//   downwash       sum over higher drones j of -C1 (r_p/4dz)^2 exp(-(dxy/beta)^2/2) (Eq. 6)
//   integrator     semi-implicit Euler, body-rate exponential map, renormalise (Eq. 7)
//
// Disturbed instantiations: DIST = 2 domain randomisation (with or without
// wind), DIST = 1 wind alone (without the randomisation's registers),
// DIST = 0 the nominal step.
// Domain randomisation (Sec. "Domain randomization", Table
// "Recommended domain-randomization ranges"): each drone carries its own
// physical constants (mass, inertia, arm length, kf, km, drag, C_gnd, C1, g,
// MAX_RPM as factors of the nominal ones) in registers for the launch, and
// an actuator chain before the motor model: action latency through a ring of
// MD_DR_HIST past actions, per-motor bias, clip to the drone's MAX_RPM, and a
// first-order motor lag n <- n + (1 - e^{-dt/tau})(c - n).  Controllers keep
// the nominal constants.  The returned observation rows carry the sensor
// side: a sticky per-drone bias, per-step Gaussian noise and a sensor
// latency ring of MD_DR_OBS_HIST rows.  Both latency rings are read and
// written only across launch boundaries (see the step loop).  Wind (Sec.
// "Wind and turbulence"): constant-wind drag (optionally a mean wind per
// drone), gusts, Dryden turbulence and a sinusoid, with per-drone state in
// registers and Philox4x32-10 draws keyed by (drone, global step).
#pragma once

#include "md_sweep.h"

namespace md {
namespace {

using namespace phys;

// The drone's own constants: the nominal block with the randomised fields
// replaced (the others stay uniform across the wave).
__device__ __forceinline__ void dr_constants(const KConst &c, const DrPtr &dr, int N, int di, KConst &cl,
                                             float bias[4]) {
    const float sm = dr.scale[MD_DR_M * N + di], sJ = dr.scale[MD_DR_J * N + di];
    const float sg = dr.scale[MD_DR_G * N + di];
    cl.m = c.m * sm;
    cl.m_inv = 1.f / cl.m;
    cl.mg = cl.m * (c.g * sg);
    cl.Jx = c.Jx * sJ;
    cl.Jy = c.Jy * sJ;
    cl.Jz = c.Jz * sJ;
    cl.Jx_inv = 1.f / cl.Jx;
    cl.Jy_inv = 1.f / cl.Jy;
    cl.Jz_inv = 1.f / cl.Jz;
    cl.l_arm = c.l_arm * dr.scale[MD_DR_L * N + di];
    cl.kf = c.kf * dr.scale[MD_DR_KF * N + di];
    cl.km = c.km * dr.scale[MD_DR_KM * N + di];
    const float sd = dr.scale[MD_DR_DRAG * N + di];
    cl.c_xy = c.c_xy * sd;
    cl.c_z = c.c_z * sd;
    cl.K_gnd = c.K_gnd * dr.scale[MD_DR_GND * N + di];
    cl.K1 = c.K1 * dr.scale[MD_DR_C1 * N + di];
    cl.max_rpm = c.max_rpm * dr.scale[MD_DR_MAXRPM * N + di];
#pragma unroll
    for (int k = 0; k < 4; ++k) bias[k] = dr.scale[(MD_DR_BIAS + k) * N + di];
}

// Philox4x32-10 (Salmon et al., SC 2011): ten rounds of the two 32x32-bit
// products with the round multipliers, high halves xored with the other
// counter words and the round key, key bumped by the Weyl constants.  Each
// product is formed whole (one 32x32 -> 64-bit multiply-add gives both
// halves) instead of as separate high and low multiplies.
__device__ __forceinline__ uint4 philox4x32(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const unsigned long long p0 = (unsigned long long)0xD2511F53u * c.x;
        const unsigned long long p1 = (unsigned long long)0xCD9E8D57u * c.z;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

__device__ __forceinline__ float unit24(uint32_t x) { return (float)(x >> 8) * (1.f / 16777216.f); }

// sin(2 pi r) and cos(2 pi r) for r in revolutions, on the hardware units
// (they take revolutions: no range reduction for |r| <= 256).
__device__ __forceinline__ float sin_rev(float r) { return __builtin_amdgcn_sinf(r); }
__device__ __forceinline__ float cos_rev(float r) { return __builtin_amdgcn_cosf(r); }

// Box-Muller on two 24-bit uniforms: rho = sqrt(-2 ln(1 - u_a)) with the
// hardware log2 (1 - u_a >= 2^-24 is a normal number), angle 2 pi u_b.
__device__ __forceinline__ void normal_pair(uint32_t a, uint32_t b, float &n0, float &n1) {
    const float rho = fsqrt(-1.3862943611198906f * __builtin_amdgcn_logf(1.f - unit24(a)));
    const float u = unit24(b);
    n0 = rho * cos_rev(u);
    n1 = rho * sin_rev(u);
}

// 1 - e^{-2c} for c >= 0 without cancellation: its Taylor series below
// 2c = 1/16 (truncation error < 2e-8 relative), expm1 above.
__device__ __forceinline__ float one_minus_exp2c(float c) {
    const float x = 2.f * c;
    if (x < 0.0625f) return x * (1.f + x * (-0.5f + x * (1.f / 6.f + x * (-1.f / 24.f + x * (1.f / 120.f)))));
    return -expm1f(-x);
}

// World-frame wind force of one drone at global step t (pre-step state d);
// vm = its mean wind; ws = the drone's wind state (Dryden x, y, z; gust step,
// -1 idle; gust heading), updated in place.  Models as documented at
// md_set_wind.
__device__ __forceinline__ void wind_force(const WindArgs &W, float dt, long long t, int di, const float vm[3],
                                           const Drone &d, float ws[5], float &Fx, float &Fy, float &Fz) {
    Fx = Fy = Fz = 0.f;
    const uint32_t tl = (uint32_t)((unsigned long long)t & 0xffffffffull);
    const uint32_t th = (uint32_t)((unsigned long long)t >> 32);
    if (W.models & MD_WIND_CONSTANT) {
        // vm: the drone's mean wind (per-drone array or the common one),
        // read once per launch
        const float ux = vm[0] - d.vx, uy = vm[1] - d.vy, uz = vm[2] - d.vz;
        const float kn = W.kd * fsqrt(ux * ux + uy * uy + uz * uz);
        Fx += kn * ux;
        Fy += kn * uy;
        Fz += kn * uz;
    }
    if (W.models & MD_WIND_DRYDEN) {
        const uint4 r = philox4x32(make_uint4((uint32_t)di, tl, th, 0u), W.key0, W.key1);
        float xi[4];
        normal_pair(r.x, r.y, xi[0], xi[1]);
        normal_pair(r.z, r.w, xi[2], xi[3]);
        const float h = clampf(d.pz * (1.f / 0.3048f), 10.f, 1000.f);
        // (0.177 + 8.23e-4 h)^1.2 through the hardware log2 and exp2
        const float Lu = h / __builtin_amdgcn_exp2f(1.2f * __builtin_amdgcn_logf(0.177f + 8.23e-4f * h)) * 0.3048f,
                    Lw = h * 0.3048f;
        const float cu = dt * W.airspeed / Lu, cw = dt * W.airspeed / Lw;
        // alpha = e^{-c}; 1 - alpha^2 = 1 - e^{-2c} without cancellation
        const float au = __expf(-cu), aw = __expf(-cw);
        const float bu = W.sigma * fsqrt(one_minus_exp2c(cu)), bw = W.sigma * fsqrt(one_minus_exp2c(cw));
        ws[0] = au * ws[0] + bu * xi[0];
        ws[1] = au * ws[1] + bu * xi[1];
        ws[2] = aw * ws[2] + bw * xi[2];
        const float kn = W.kd * fsqrt(ws[0] * ws[0] + ws[1] * ws[1] + ws[2] * ws[2]);
        Fx += kn * ws[0];
        Fy += kn * ws[1];
        Fz += kn * ws[2];
    }
    if (W.models & MD_WIND_GUST) {
        if (ws[3] < 0.f) {
            const uint4 g = philox4x32(make_uint4((uint32_t)di, tl, th, 1u), W.key0, W.key1);
            if (unit24(g.x) < W.gust_prob) {
                ws[3] = 0.f;
                ws[4] = 6.283185307179586f * unit24(g.y);
            }
        }
        if (ws[3] >= 0.f) {
            const float env = sin_rev(0.5f * ws[3] / (float)W.gust_steps);
            const float hr = ws[4] * 0.15915494309189535f;  // heading in revolutions
            const float sh = sin_rev(hr), ch = cos_rev(hr);
            Fx += W.gust_amp * ch * env;
            Fy += W.gust_amp * sh * env;
            ws[3] += 1.f;
            if (ws[3] >= (float)W.gust_steps) ws[3] = -1.f;
        }
    }
    if (W.models & MD_WIND_SINUSOIDAL) {
        // phase reduced in double (t dt grows without bound), in revolutions
        const double ph = W.sin_wdt * (double)t * (1.0 / 6.283185307179586);
        const float rev = (float)(ph - floor(ph));
        const float s1 = sin_rev(rev), c1 = cos_rev(rev), s2 = sin_rev(2.f * rev);
        Fx += W.sin_amp * s1;
        Fy += W.sin_amp * c1;
        Fz += W.sin_amp * 0.3f * s2;
    }
}

// Sensor noise on one drone's KIN row at global step t, as documented at
// md_set_domain_randomization: Gaussian noise on position, velocity,
// roll/pitch/yaw and body rates from three Philox blocks (streams 2, 3, 4;
// Box-Muller on 24-bit uniforms).
__device__ __forceinline__ void sensor_noise(const DrPtr &dr, int di, long long t, float row[20]) {
    const uint32_t tl = (uint32_t)((unsigned long long)t & 0xffffffffull);
    const uint32_t th = (uint32_t)((unsigned long long)t >> 32);
    float xi[12];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        const uint4 r = philox4x32(make_uint4((uint32_t)di, tl, th, 2u + (uint32_t)b), dr.key0, dr.key1);
        normal_pair(r.x, r.y, xi[4 * b + 0], xi[4 * b + 1]);
        normal_pair(r.z, r.w, xi[4 * b + 2], xi[4 * b + 3]);
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        row[k] = fmaf(dr.sig[0], xi[k], row[k]);
        row[10 + k] = fmaf(dr.sig[1], xi[3 + k], row[10 + k]);
        row[7 + k] = fmaf(dr.sig[2], xi[6 + k], row[7 + k]);
        row[13 + k] = fmaf(dr.sig[3], xi[9 + k], row[13 + k]);
    }
}

// One drone's 20-row observation into slot `slot` of [slots][20][N] when the
// slot differs between lanes (64-bit per-lane addresses).
__device__ __forceinline__ void store_obs_lane(float *obs, int slot, int N, int di, const float row[20]) {
    float *b = obs + (long long)slot * 20 * N + di;
#pragma unroll
    for (int k = 0; k < 20; ++k) b[(long long)k * N] = row[k];
}

// The previous step's observation row, stored a few rows at a time after the
// segments of the rotation sweep (rows [s 20 / (H + 1), (s + 1) 20 / (H + 1))
// after segment s of H + 1).  Stored in one burst per step, the rows of every
// wave leave the vector ALU and the write stream taking turns; spread through
// the sweep they overlap.  No branch enters the sweep: the buffer range is
// the slot's 20 rows (the range check counts the scalar row offset), and an
// idle lane's offset of 20 N * 4 lies past it for every row, so the hardware
// drops its stores (the offsets stay below 2^32 for N <= 2^24).
struct RowSeg {
    __amdgpu_buffer_rsrc_t rs;
    int voff, rowbytes;
    float v[20];
    // rows [r0, r1) with their scalar offsets r * rowbytes formed by scalar
    // adds beside the stores: rowbytes is made opaque per call, so the
    // offsets are not hoisted out of the step loop (twenty of them held for
    // the whole launch overflowed the scalar registers, and the spilled ones
    // came back through the vector ALU every step)
    __device__ __forceinline__ void rows(int r0, int r1) const {
        int rb = rowbytes;
        asm volatile("" : "+s"(rb));
        int so = r0 * rb;
#pragma unroll
        for (int r = r0; r < r1; ++r) {
            __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v[r]), rs, voff, so, 0);
            so += rb;
        }
    }
    __device__ __forceinline__ void all() const { rows(0, 20); }
    template <int H>
    __device__ __forceinline__ void at(int s) const {
        const int r0 = s * 20 / (H + 1), r1 = (s + 1) * 20 / (H + 1);
        if (r1 > r0) rows(r0, r1);
    }
};

// Workgroups of up to 1024 threads, 512 with domain randomisation: its
// per-drone constants, actuator chain and sensor side need more than the 128
// registers per lane that sixteen waves per workgroup leave (they spilled to
// scratch memory, which the long launches then streamed through HBM).
template <uint32_t MASK, int ACT, int LPD, int UNROLL, int SYM, int DIST>
__global__ void __launch_bounds__(DIST == 2 ? MAX_THREADS_DR : 1024) step_kernel(StepArgs a) {
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
    // Physical constants of this drone (the nominal ones without randomisation).
    KConst cl = c;
    float bias[4] = {1.f, 1.f, 1.f, 1.f};
    float lag = 1.f;            // 1 - e^{-dt/tau}
    bool has_lag = false;
    int delay = 0, acnt0 = 0;  // action latency (steps, clamped to the ring) and ring fill at launch
    float cmdh[4] = {0.f, 0.f, 0.f, 0.f};  // controller output held between updates
    // Randomisation (the factor table, lag, latencies, the held-command block,
    // the sensor side) runs only in the DIST = 2 instantiation and when the
    // context has a factor table; otherwise the plain actuator chain runs and
    // rpm_cmd / act_hist / act_count / obs_hist / obs_count are never touched.
    const bool rnd = DIST == 2 && a.dr.scale != nullptr;
    const bool ring = rnd && a.dr.delay != nullptr;
    float ws[5] = {0.f, 0.f, 0.f, -1.f, 0.f};  // wind state
    const bool windy = DIST >= 1 && a.wind.models != 0u;
    if (windy && valid && a.s.wind != nullptr)
        for (int k = 0; k < 5; ++k) ws[k] = a.s.wind[k * N + di];
    // the drone's mean wind, held for the launch
    float vmean[3] = {a.wind.vm[0], a.wind.vm[1], a.wind.vm[2]};
    if (windy && valid && a.wind.vm_drone != nullptr)
        for (int k = 0; k < 3; ++k) vmean[k] = a.wind.vm_drone[k * N + di];
    if (rnd && valid) {
        dr_constants(c, a.dr, N, di, cl, bias);
        const float tau = a.dr.tau_mot ? a.dr.tau_mot[di] : 0.f;
        has_lag = tau > 0.f;
        lag = has_lag ? 1.f - expf(-c.dt / tau) : 1.f;
        if (ring) {
            delay = min(max(a.dr.delay[di], 0), MD_DR_HIST - 1);
            acnt0 = min(max(a.s.act_count[di], 0), MD_DR_HIST);
        }
        if (ACT >= 1)
            for (int k = 0; k < 4; ++k) cmdh[k] = a.s.rpm_cmd[k * N + di];
    }
    // Sensor noise and latency act on the returned rows only.  The latency
    // rings (actions and rows) are kept in HBM across launches only: the
    // value used at global step t is the one entered at step
    // r = t - min(delay, fill at launch + steps so far) (the oldest one while
    // the ring fills), read from this launch's own inputs or rows when
    // r >= step0 and from the ring otherwise; each launch enters only its
    // last MD_DR_HIST actions and MD_DR_OBS_HIST rows, which is all a later
    // launch can reach.
    const bool oring = rnd && a.dr.obs_delay != nullptr;
    const bool noisy = rnd && a.dr.noisy;
    int odelay = 0, ocnt0 = 0;
    if (oring && valid) {
        odelay = min(max(a.dr.obs_delay[di], 0), MD_DR_OBS_HIST - 1);
        ocnt0 = min(max(a.s.obs_count[di], 0), MD_DR_OBS_HIST);
    }
    int osl = oring ? (int)(a.step0 % (long long)MD_DR_OBS_HIST) : 0;
    // the sticky observation bias (position, velocity, angles, rates), held
    // for the launch
    float obias[12];
    for (int b = 0; b < 12; ++b) obias[b] = 0.f;
    const bool biased = rnd && a.dr.obs_bias != nullptr;
    if (biased && valid)
        for (int b = 0; b < 12; ++b) obias[b] = a.dr.obs_bias[(long long)b * N + di];

    float *tmat = (float *)(lds_pos + 4 * slots);
    if (SYM == 1 && (MASK & 4u) && valid) {
        // the diagonal and the padding up to the next multiple of 4 stay 0
        tmat[slot * a.tstride + (slot - lo)] = 0.f;
        for (int j = menv; j < ((menv + 3) & ~3); ++j) tmat[slot * a.tstride + j] = 0.f;
    }
    // Held waypoints (one action row for the whole launch) stay in registers:
    // re-reading them at every controller update would fetch them from HBM
    // again, since the observation stream evicts them from L2.
    const bool held = a.act_step_stride == 0;
    constexpr int ROWS = action_rows(ACT);
    float tgt_held[ROWS];
    float sp[4] = {0.f, 0.f, 0.f, 0.f};
    for (int k = 0; k < ROWS; ++k) tgt_held[k] = 0.f;
    if (ACT >= 1 && held && valid)
        for (int k = 0; k < ROWS; ++k) tgt_held[k] = a.action[(long long)k * N + di];
    if (ACT == 4 && valid)
        for (int k = 0; k < 4; ++k) sp[k] = a.s.ctl[k * N + di];
    // Per-step rotor-speed actions are read one step ahead: the row of step
    // k + 1 is requested during step k, so its memory latency overlaps the
    // step instead of opening the next one (short launches of small layouts
    // are latency-bound).  The read is unconditional (the last step reads
    // its own row again; idle lanes read drone 0's row and keep zero rotor
    // speeds): a read under a condition leaves the loaded value to be merged
    // into the loop's register right after the load, which waits for it.
    const int da = valid ? di : 0;
    float nact[4] = {0.f, 0.f, 0.f, 0.f};
    if (ACT == 0 && !rnd && a.n_steps > 0)
        for (int k = 0; k < 4; ++k) nact[k] = a.action[(long long)k * N + da];
    // controller phase, observation slot and ring slot advance as counters
    int phase = (ACT >= 1) ? (int)(a.step0 % (long long)c.decim) : 0;
    int oslot = 0;
    int hslot = (int)(a.step0 % (long long)MD_DR_HIST);
    // Nominal step with the rotation sweep: each observation row is stored
    // during the next step between the sweep's segments (RowSeg); the state
    // is still that row until the integration, its angles are formed at the
    // start of the next step (from the rotation entries that step's
    // controller also reads; the same expressions as euler_zyx), its rotor
    // speeds are kept in nprev, and the launch's last row is stored after
    // the loop.
    constexpr bool seg_obs = DIST == 0 && SYM == 3 && (MASK & 4u) && LPD == 1;
    const bool seg_on = seg_obs && a.obs != nullptr && N <= (1 << 24);  // uniform
    float nprev[4] = {0.f, 0.f, 0.f, 0.f};
    float rpy[3] = {0.f, 0.f, 0.f};  // the previous row's angles
    int pslot = 0;
    for (int step = 0; step < a.n_steps; ++step) {
        float4 *buf = lds_pos + (step & 1) * (2 * slots);
        if (MASK & 4u) {
            if (SYM == 3) {
                // interleaved uniform bins: each wave's positions twice (128 entries)
                const int lane = slot & 63;
                float4 *own = buf + 2 * (slot - lane) + lane;
                own[0] = own[64] = make_float4(d.px, d.py, d.pz, 0.f);
            } else if (sub == 0) {
                buf[slot] = make_float4(d.px, d.py, d.pz, 0.f);
            }
            __syncthreads();
        }
        // the rotation sweep's instantiation forms the attitude angles once:
        // for the previous row's observation and for this step's controller
        RotZYX ez{};
        float att[3] = {0.f, 0.f, 0.f};
        if constexpr (seg_obs) {
            ez = rot_zyx(d);
            if ((seg_on && step > 0) || (ACT >= 1 && phase == 0)) euler_of(ez, att[0], att[1], att[2]);
            for (int k = 0; k < 3; ++k) rpy[k] = att[k];
        }
        // ---- rotor speeds
        const float *act = a.action + a.act_step_stride * step;
        if (!rnd) {
            if (ACT == 0) {
                for (int k = 0; k < 4; ++k) n[k] = valid ? clampf(nact[k], 0.f, c.max_rpm) : 0.f;
                const float *nx = (step + 1 < a.n_steps) ? act + a.act_step_stride : act;
                for (int k = 0; k < 4; ++k) nact[k] = nx[(long long)k * N + da];
            } else {
                if (phase == 0 && valid) {
                    float cmd[ROWS];
                    for (int k = 0; k < ROWS; ++k) cmd[k] = held ? tgt_held[k] : act[(long long)k * N + di];
                    if constexpr (seg_obs)
                        control_rpy<ACT>(c, d, ez, att[0], att[1], att[2], cmd, I, sp, n);
                    else
                        control<ACT>(c, d, cmd, I, sp, n);
                }
                phase = (phase + 1 == c.decim) ? 0 : phase + 1;
            }
        } else {
            // action rows of this step, delayed by the drone's latency
            const bool need = (ACT == 0) || (phase == 0);
            float row[ROWS];
            if (valid && need) {
                const int back = ring ? min(delay, acnt0 + step) : 0;
                if (back <= step) {
                    const float *ar = act - a.act_step_stride * back;
                    for (int k = 0; k < ROWS; ++k)
                        row[k] = (ACT >= 1 && held) ? tgt_held[k] : ar[(long long)k * N + di];
                } else {
                    const float *h = a.s.act_hist;
                    const int from = hslot - back + (hslot < back ? MD_DR_HIST : 0);
                    for (int k = 0; k < ROWS; ++k) row[k] = h[((long long)from * ROWS + k) * N + di];
                }
            }
            float cmd4[4];
            if (ACT == 0) {
                for (int k = 0; k < 4; ++k) cmd4[k] = row[k];
            } else {
                if (phase == 0 && valid) control<ACT>(c, d, row, I, sp, cmdh);
                phase = (phase + 1 == c.decim) ? 0 : phase + 1;
                for (int k = 0; k < 4; ++k) cmd4[k] = cmdh[k];
            }
            if (valid) {
                for (int k = 0; k < 4; ++k) {
                    const float cc = clampf(bias[k] * cmd4[k], 0.f, cl.max_rpm);
                    n[k] = has_lag ? n[k] + lag * (cc - n[k]) : cc;
                }
            }
            hslot = (hslot + 1 == MD_DR_HIST) ? 0 : hslot + 1;
        }
        // ---- motor model and mixer (Eq. 1-3)
        float T, tx, ty, tz;
        motor(cl, n, T, tx, ty, tz);
        const Rot R = rot_of(d);
        float Fx = R.r02 * T, Fy = R.r12 * T, Fz = R.r22 * T - cl.mg;
        // ---- ground effect (Eq. 4)
        if (MASK & 1u) Fz += ground_effect(cl, d, R, T);
        // ---- blade drag (Eq. 5)
        if (MASK & 2u) {
            float dx, dy, dz;
            drag(cl, d, R, n, dx, dy, dz);
            Fx += dx;
            Fy += dy;
            Fz += dz;
        }
        // ---- downwash (Eq. 6): sweep the environment in ascending order
        if (MASK & 4u) {
            float acc;
            if (seg_obs) {
                const int lane = slot & 63;
                const float4 *own = buf + 2 * (slot - lane) + lane;
                if (seg_on && step > 0) {
                    const RowSeg seg{__builtin_amdgcn_make_buffer_rsrc(a.obs + (long long)pslot * 20 * N, (short)0,
                                                                       20 * N * 4, 0x00020000),
                                     writer ? di * 4 : 20 * N * 4, N * 4,
                                     {d.px, d.py, d.pz, d.qw, d.qx, d.qy, d.qz, rpy[0], rpy[1], rpy[2],
                                      d.vx, d.vy, d.vz, d.wx, d.wy, d.wz, nprev[0], nprev[1], nprev[2], nprev[3]}};
                    acc = c.dz_min > 0.f ? dw_rot<true>(c, own, lane, mmax, d, seg)
                                         : dw_rot<false>(c, own, lane, mmax, d, seg);
                } else {
                    acc = c.dz_min > 0.f ? dw_rot<true>(c, own, lane, mmax, d) : dw_rot<false>(c, own, lane, mmax, d);
                }
            } else {
                acc = dw_sum<LPD, UNROLL, SYM>(c, buf, tmat, a.tstride, slot, sub, lo, mmax, menv, uniform, d);
            }
            Fz -= cl.K1 * acc;
        }
        // ---- wind
        if (windy && valid) {
            float wx, wy, wz;
            wind_force(a.wind, c.dt, a.step0 + step, di, vmean, d, ws, wx, wy, wz);
            Fx += wx;
            Fy += wy;
            Fz += wz;
        }
        // ---- Newton-Euler + exponential map (Eq. 7)
        integrate(cl, d, Fx, Fy, Fz, tx, ty, tz);
        // ---- KIN observation
        const bool otail = oring && step >= a.n_steps - MD_DR_OBS_HIST;
        if (seg_on) {
            for (int k = 0; k < 4; ++k) nprev[k] = n[k];
            pslot = oslot;
        } else if ((a.obs != nullptr || otail) && writer) {
            float roll, pitch, yaw;
            euler_zyx(d, roll, pitch, yaw);
            float orow[20] = {d.px, d.py, d.pz, d.qw, d.qx, d.qy, d.qz, roll, pitch, yaw,
                              d.vx, d.vy, d.vz, d.wx, d.wy, d.wz, n[0], n[1], n[2], n[3]};
            if (biased) {
#pragma unroll
                for (int b = 0; b < 12; ++b) orow[b < 3 ? b : (b < 6 ? b + 7 : (b < 9 ? b + 1 : b + 4))] += obias[b];
            }
            if (noisy) sensor_noise(a.dr, di, a.step0 + step, orow);
            if (!oring) {
                store_obs(a.obs, oslot, N, di, orow);
            } else {
                float *h = a.s.obs_hist;
                if (otail) {
#pragma unroll
                    for (int k = 0; k < 20; ++k) h[((long long)osl * 20 + k) * N + di] = orow[k];
                }
                if (a.obs != nullptr) {
                    const int S = a.n_obs_slots, n_st = a.n_steps;
                    // this step returns a row entered before the launch
                    const int back = min(odelay, ocnt0 + step);
                    if (back > step && step >= n_st - S) {
                        const int from = osl - back + (osl < back ? MD_DR_OBS_HIST : 0);
                        float old[20];
#pragma unroll
                        for (int k = 0; k < 20; ++k) old[k] = h[((long long)from * 20 + k) * N + di];
                        store_obs(a.obs, oslot, N, di, old);
                    }
                    // the steps that return this row: step + delay, and every
                    // step up to it when the ring starts empty here
                    const int k_hi = min(step + odelay, n_st - 1);
                    const int k_lo = max((ocnt0 == 0 && step == 0) ? 0 : step + odelay, n_st - S);
                    for (int kk = k_lo; kk <= k_hi; ++kk) {
                        int sl = oslot + (kk - step);
                        while (sl >= S) sl -= S;
                        store_obs_lane(a.obs, sl, N, di, orow);
                    }
                }
            }
        }
        oslot = (oslot + 1 == a.n_obs_slots) ? 0 : oslot + 1;
        if (oring) osl = (osl + 1 == MD_DR_OBS_HIST) ? 0 : osl + 1;
    }
    if (seg_on && writer && a.n_steps > 0) {
        euler_zyx(d, rpy[0], rpy[1], rpy[2]);
        const float orow[20] = {d.px, d.py, d.pz, d.qw, d.qx, d.qy, d.qz, rpy[0], rpy[1], rpy[2],
                                d.vx, d.vy, d.vz, d.wx, d.wy, d.wz, n[0], n[1], n[2], n[3]};
        store_obs(a.obs, pslot, N, di, orow);
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
        if (rnd && ACT >= 1)
            for (int k = 0; k < 4; ++k) a.s.rpm_cmd[k * N + di] = cmdh[k];
        if (ring) {
            // enter this launch's last MD_DR_HIST action rows
            const int j0 = max(a.n_steps - MD_DR_HIST, 0);
            int sl = (int)((a.step0 + j0) % (long long)MD_DR_HIST);
            for (int j = j0; j < a.n_steps; ++j) {
                const float *ar = a.action + a.act_step_stride * j;
                for (int k = 0; k < ROWS; ++k)
                    a.s.act_hist[((long long)sl * ROWS + k) * N + di] =
                        (ACT >= 1 && held) ? tgt_held[k] : ar[(long long)k * N + di];
                sl = (sl + 1 == MD_DR_HIST) ? 0 : sl + 1;
            }
            a.s.act_count[di] = (int)min((long long)acnt0 + a.n_steps, (long long)MD_DR_HIST);
        }
        if (oring) a.s.obs_count[di] = (int)min((long long)ocnt0 + a.n_steps, (long long)MD_DR_OBS_HIST);
        if (windy && a.s.wind != nullptr)
            for (int k = 0; k < 5; ++k) a.s.wind[k * N + di] = ws[k];
    }
}

template <uint32_t MASK, int ACT, int LPD, int SYM, int DIST>
hipError_t launch_u(const StepArgs &a, int unroll, int n_bins, int threads, size_t lds, hipStream_t st) {
    switch (unroll) {
        case 1: hipLaunchKernelGGL((step_kernel<MASK, ACT, LPD, 1, SYM, DIST>), dim3(n_bins), dim3(threads), lds, st, a); break;
        case 2: hipLaunchKernelGGL((step_kernel<MASK, ACT, LPD, 2, SYM, DIST>), dim3(n_bins), dim3(threads), lds, st, a); break;
        case 4: hipLaunchKernelGGL((step_kernel<MASK, ACT, LPD, 4, SYM, DIST>), dim3(n_bins), dim3(threads), lds, st, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <uint32_t MASK, int ACT, int DIST>
hipError_t launch_l(const StepArgs &a, const LaunchCfg &cfg, int n_bins, int threads, size_t lds,
                    hipStream_t st) {
    if (!(MASK & 4u)) {
        // no neighbour sweep: one lane per drone, no loop to tune
        hipLaunchKernelGGL((step_kernel<MASK, ACT, 1, 1, 0, DIST>), dim3(n_bins), dim3(threads), lds, st, a);
        return hipGetLastError();
    }
    if (cfg.sym) {
        if (cfg.lpd != 1) return hipErrorInvalidValue;
        if (cfg.sym >= 2) {
            // the rotation sweep is unrolled in full, the permute sweep not at
            // all (see cfg_valid): one instantiation each
            if (cfg.unroll != 1) return hipErrorInvalidValue;
            if (cfg.sym == 3)
                hipLaunchKernelGGL((step_kernel<MASK, ACT, 1, 1, 3, DIST>), dim3(n_bins), dim3(threads), lds, st, a);
            else
                hipLaunchKernelGGL((step_kernel<MASK, ACT, 1, 1, 2, DIST>), dim3(n_bins), dim3(threads), lds, st, a);
            return hipGetLastError();
        }
        return launch_u<MASK, ACT, 1, 1, DIST>(a, cfg.unroll, n_bins, threads, lds, st);
    }
    switch (cfg.lpd) {
        case 1: return launch_u<MASK, ACT, 1, 0, DIST>(a, cfg.unroll, n_bins, threads, lds, st);
        case 2: return launch_u<MASK, ACT, 2, 0, DIST>(a, cfg.unroll, n_bins, threads, lds, st);
        case 4: return launch_u<MASK, ACT, 4, 0, DIST>(a, cfg.unroll, n_bins, threads, lds, st);
        default: return hipErrorInvalidValue;
    }
}

template <int ACT, int DIST>
hipError_t launch_m(const StepArgs &a, uint32_t mask, const LaunchCfg &cfg, int n_bins,
                    int threads, size_t lds, hipStream_t st) {
    switch (mask & 7u) {
        case 0: return launch_l<0, ACT, DIST>(a, cfg, n_bins, threads, lds, st);
        case 1: return launch_l<1, ACT, DIST>(a, cfg, n_bins, threads, lds, st);
        case 2: return launch_l<2, ACT, DIST>(a, cfg, n_bins, threads, lds, st);
        case 3: return launch_l<3, ACT, DIST>(a, cfg, n_bins, threads, lds, st);
        case 4: return launch_l<4, ACT, DIST>(a, cfg, n_bins, threads, lds, st);
        case 5: return launch_l<5, ACT, DIST>(a, cfg, n_bins, threads, lds, st);
        case 6: return launch_l<6, ACT, DIST>(a, cfg, n_bins, threads, lds, st);
        default: return launch_l<7, ACT, DIST>(a, cfg, n_bins, threads, lds, st);
    }
}

template <int DIST>
hipError_t launch_step_t(const StepArgs &a, uint32_t mask, int act, const LaunchCfg &cfg, int n_bins,
                         int slots, hipStream_t stream) {
    if (n_bins <= 0 || a.n_steps <= 0) return hipSuccess;
    const int lpd = (mask & 4u) ? cfg.lpd : 1;
    const int threads = slots * lpd;
    size_t lds = (mask & 4u) ? sizeof(float4) * 2 * 2 * (size_t)slots : 0;
    if ((mask & 4u) && cfg.sym == 1) lds += sizeof(float) * (size_t)slots * (size_t)a.tstride;
    switch (act) {
        case 0: return launch_m<0, DIST>(a, mask, cfg, n_bins, threads, lds, stream);
        case 1: return launch_m<1, DIST>(a, mask, cfg, n_bins, threads, lds, stream);
        case 2: return launch_m<2, DIST>(a, mask, cfg, n_bins, threads, lds, stream);
        case 3: return launch_m<3, DIST>(a, mask, cfg, n_bins, threads, lds, stream);
        default: return launch_m<4, DIST>(a, mask, cfg, n_bins, threads, lds, stream);
    }
}

}  // namespace
}  // namespace md
