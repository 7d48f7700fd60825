// md_internal.h -- shared between the host API (md_api.cpp) and the HIP
// kernels of libmd.  Not installed; the public ABI is include/md.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "md.h"

namespace md {

// Per-context float32 constants, precomputed on the host in double and passed
// to the kernels by value.
struct KConst {
    float dt, m, m_inv, g, mg;
    float kf, km, l_arm;                  // l_arm = L / sqrt(2)   (Eq. 2-3)
    float Jx, Jy, Jz, Jx_inv, Jy_inv, Jz_inv;
    float max_rpm, h_clip, K_gnd;         // K_gnd = C_gnd r_p^2 / 16   (Eq. 4)
    float drag_s, c_xy, c_z;              // drag_s = 2 pi / 60         (Eq. 5)
    float K1, C2, C3, dz_min;             // K1 = C1 r_p^2 / 16         (Eq. 6)
    float C2s, C3s;                       // sqrt(2 ln 2) C2, sqrt(2 ln 2) C3
    float pkp[3], pki[3], pkd[3], p_clamp;
    float akp[3], aki[3], akd[3], a_clamp;
    float dsl_pkp[3], dsl_pki[3], dsl_pkd[3], dsl_p_clamp;
    float dsl_akp[3], dsl_aki[3], dsl_akd[3], dsl_a_clamp;
    float dsl_step, dsl_ystep;  // setpoint limits per controller update (m, rad)
    float dt_c, g_inv, l_inv, kappa_inv, fmax, kf_inv;
    float hover_inv;                      // 1 / HOVER_RPM (surrogate inputs)
    int decim;
};

// SoA device pointers of md_state.
struct StatePtr {
    float *p, *q, *v, *w, *pid_int, *rpm, *ctl;
    float *rpm_cmd, *act_hist;  // domain randomisation: held command, action ring
    int32_t *act_count;         // domain randomisation: ring fill per drone
    float *wind;                // wind: [5][N] Dryden velocity, gust step, gust heading
    float *obs_hist;            // sensor latency: [MD_DR_OBS_HIST][20][N] ring of rows
    int32_t *obs_count;         // sensor latency: ring fill per drone
};

// Wind parameters (md_wind) prepared on the host.
struct WindArgs {
    uint32_t models;            // MD_WIND_* bits, 0 = off
    float vm[3];                // mean wind, m/s
    float kd;                   // rho CdA / 2
    float gust_prob, gust_amp;  // per-step trigger probability, N
    int gust_steps;             // round(duration / dt), >= 1
    float sigma, airspeed;      // Dryden sigma (m/s) and V (m/s)
    float sin_amp;              // N
    double sin_wdt;             // sinusoid phase per step, omega dt (rad)
    uint32_t key0, key1;        // Philox key (seed)
    const float *vm_drone;      // [3][N] per-drone mean wind or null
};

// Domain randomisation inputs (md_dr), device pointers.
struct DrPtr {
    const float *scale;      // [MD_DR_NSCALE][N]
    const float *tau_mot;    // [N] or null
    const int32_t *delay;    // [N] or null
    float sig[4];            // sensor noise sigma: position, velocity, roll/pitch/yaw, body rates
    bool noisy;              // any sigma > 0
    uint32_t key0, key1;     // Philox key of the sensor noise (seed)
    const int32_t *obs_delay;  // [N] or null
    const float *obs_bias;     // [12][N] or null
};

// Action rows per action type (MD_ACT_DSL carries a feed-forward acceleration).
__host__ __device__ constexpr int action_rows(int act) { return act == 4 ? 7 : 4; }

// One bin = one workgroup.  Per slot (drone slot inside the bin):
//   x = global drone index or -1 for an idle slot,
//   y = (first slot of the drone's environment inside the bin) << 16 | M_env.
// Per bin: the largest environment it holds (the uniform neighbour-loop
// bound) in the low 16 bits, and bit 16 set when every environment in the
// bin has that size (no per-lane bound check needed).
struct BinTables {
    const int2 *slot;      // [n_bins * slots]
    const int *bin_mmax;   // [n_bins]
};

struct StepArgs {
    KConst c;
    StatePtr s;
    const float *action;
    long long act_step_stride;  // 0 (held) or 4 * N
    float *obs;
    int n_obs_slots;
    int n_steps;
    long long step0;
    int N;
    BinTables bins;
    int tstride;  // row stride (floats) of the pair-term matrix in LDS (sym sweep)
    DrPtr dr;       // domain randomisation (used by the disturbed instantiation only)
    WindArgs wind;  // wind (disturbed instantiation only)
};

// Row stride (floats) of the pair-term matrix of the pair-symmetric sweep: a
// multiple of 4 (rows are summed with 16-byte LDS reads) that holds the
// largest environment; the odd lane stride ts + 1 of its row and column
// writes spreads a wave over the LDS banks.
__host__ __device__ constexpr int pair_stride(int max_m) { return ((max_m + 3) / 4) * 4 > 0 ? ((max_m + 3) / 4) * 4 : 4; }

// Largest workgroup of the step kernel with domain randomisation (threads).
constexpr int MAX_THREADS_DR = 512;

// Launch configuration chosen per (shape, mask) by the autotuner.
struct LaunchCfg {
    int lpd;     // lanes per drone in the neighbour sweep: 1, 2 or 4
    int unroll;  // neighbour-loop unroll: 1, 2, 4 or 8
    int waves;   // waves per workgroup (bin size 64 * waves / lpd slots)
    int sym;     // pair-symmetric sweep (lpd must be 1): 1 LDS term matrix, 2 wave permutes,
                 // 3 whole-wave rotation on interleaved uniform bins
};

hipError_t launch_step(const StepArgs &a, uint32_t mask, int act, const LaunchCfg &cfg,
                       int n_bins, int slots, hipStream_t stream);
// Same contract with per-drone domain randomisation (a.dr).
hipError_t launch_step_dr(const StepArgs &a, uint32_t mask, int act, const LaunchCfg &cfg,
                          int n_bins, int slots, hipStream_t stream);
hipError_t launch_step_wind(const StepArgs &a, uint32_t mask, int act, const LaunchCfg &cfg,
                          int n_bins, int slots, hipStream_t stream);
// Same contract with the classic Runge-Kutta integrator (lanes per drone 1).
hipError_t launch_step_rk4(const StepArgs &a, uint32_t mask, int act, const LaunchCfg &cfg,
                           int n_bins, int slots, hipStream_t stream);

}  // namespace md
