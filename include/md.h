/*
 * md.h -- C ABI of libmd, the MI355X (gfx950) batched explicit quadrotor step.
 *
 * The library advances many independent environments of Crazyflie-class
 * quadrotors by the explicit dynamics of MuJoCo-Drones-Gym (Sec. "Quadrotor
 * Dynamics", Sec. "Physics Modes"): rotor speeds -> thrust and torques
 * (Eq. 1-3), optional ground effect (Eq. 4), blade drag (Eq. 5) and pairwise
 * downwash (Eq. 6), then Newton-Euler with the quaternion exponential map
 * (Eq. 7).  Actions are raw rotor speeds or PID waypoints (Table "Action
 * types", Sec. "Control").  An optional learned surrogate replaces Eq. 4-6.
 *
 * Conventions for every entry point:
 *   - Pointers named d_* are DEVICE pointers (hipMalloc'ed or from a
 *     framework allocator) on the context's device; h_* are host pointers.
 *   - The caller owns every buffer it passes; the library never frees or
 *     retains caller memory beyond the call (asynchronous calls read and write
 *     it on the given stream until that stream reaches the enqueued work).
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *   - Every function returns md_status: 0 on success, a negative MD_E_* code
 *     otherwise; no C++ exception crosses the ABI.  md_last_error(ctx) then
 *     holds a message (per context, valid until the next call on it).
 *   - Device faults of asynchronous work surface at the next synchronising
 *     call on the stream (hipStreamSynchronize or md_* calls that read back).
 *   - One context may be used from one host thread at a time.
 *
 * Device state is float32, structure-of-arrays, component-major: component c
 * of drone i lives at ptr[c * n_drones + i].  Drones of one environment are
 * contiguous; environment e holds drones [off[e], off[e+1]).
 */
#ifndef MD_H
#define MD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t md_status;
#define MD_OK 0
#define MD_E_INVALID_ARG (-1) /* a null pointer, a negative size, an unknown enum */
#define MD_E_HIP (-2)         /* a HIP runtime call failed (message has the HIP error) */
#define MD_E_OOM (-3)         /* the library could not allocate its own device memory */
#define MD_E_UNSUPPORTED (-4) /* a valid request the library does not implement */
#define MD_E_LAYOUT (-5)      /* no layout bound, layout sizes disagree, or a stale captured rollout */

/* Aerodynamic terms (Table "Physics modes" toggles), OR-able. */
#define MD_AERO_GND 1u       /* ground effect, Eq. 4 */
#define MD_AERO_DRAG 2u      /* blade drag, Eq. 5 */
#define MD_AERO_DW 4u        /* pairwise downwash within an environment, Eq. 6 */
#define MD_AERO_SURROGATE 8u /* learned residual replaces GND|DRAG|DW (exclusive with them) */

/* Action types (Table "Action types"; controllers of Sec. "Control").  The
 * controllers run every ctrl_decim steps and hold their rotor speeds. */
#define MD_ACT_RPM 0      /* action[4][N]: rotor speeds in rev/min, clipped to [0, MAX_RPM] */
#define MD_ACT_PID 1      /* action[4][N]: waypoint x, y, z (m), yaw (rad), cascaded PID */
#define MD_ACT_VEL 2      /* action[4][N]: heading-frame velocity vx, vy, vz (m/s), yaw rate (rad/s) */
#define MD_ACT_ATTITUDE 3 /* action[4][N]: collective thrust (N), roll, pitch (rad), yaw rate (rad/s) */
#define MD_ACT_DSL 4      /* action[7][N]: waypoint x, y, z, yaw, feed-forward acceleration ax, ay, az;
                             DSL-style PID with rate-limited setpoint (state block ctl) */

/* Physical and controller constants, SI units, rotor speed in rev/min.
 * m mass; L arm length; kf, km thrust and reaction-torque coefficients per
 * RPM^2 (Eq. 1); Ixx, Iyy, Izz principal inertia; thrust2weight sets MAX_RPM;
 * r_p propeller radius; g gravity; C_gnd ground-effect coefficient (Eq. 4);
 * c_xy, c_z drag coefficients (Eq. 5); C1, C2, C3 downwash coefficients
 * (Eq. 6); dw_dz_min optional lower bound on the downwash vertical gap
 * (0 = the literal equation); PID gains and symmetric integral clamps
 * (Table "Default PIDControl gains"). */
typedef struct md_params {
    double m, L, kf, km, Ixx, Iyy, Izz, thrust2weight, r_p, g;
    double C_gnd, c_xy, c_z, C1, C2, C3, dw_dz_min;
    double pos_kp[3], pos_ki[3], pos_kd[3], pos_i_clamp;
    double att_kp[3], att_ki[3], att_kd[3], att_i_clamp;
    /* DSL-style PID: own gains and integral clamps, setpoint rate limits
     * (m/s, rad/s) */
    double dsl_pos_kp[3], dsl_pos_ki[3], dsl_pos_kd[3], dsl_pos_i_clamp;
    double dsl_att_kp[3], dsl_att_ki[3], dsl_att_kd[3], dsl_att_i_clamp;
    double dsl_max_speed, dsl_max_yaw_rate;
} md_params;

/* Quantities derived from md_params (Sec. "Drone Models"; h_clip under Eq. 4). */
typedef struct md_derived {
    double hover_rpm, max_rpm, max_thrust, h_clip;
} md_derived;

/* Device state of n_drones drones, each pointer [rows][n_drones] float32:
 * p[3] world position; q[4] body->world unit quaternion (w,x,y,z);
 * v[3] world velocity; w[3] body angular velocity; pid_int[6] PID integral
 * sums (position xyz, then roll/pitch/yaw; only read/written in PID mode,
 * may be NULL for RPM actions); rpm[4] rotor speeds applied in the last
 * step (the held command between controller updates); ctl[4] the DSL
 * controller's rate-limited setpoint x, y, z, yaw (MD_ACT_DSL only, may be
 * NULL otherwise; initialise it to the drone's position and yaw).
 * With domain randomisation (md_set_domain_randomization) three more blocks:
 * rpm_cmd[4] the controller output held between updates (controller actions
 * only; rpm then holds the lagged actual speeds), act_hist
 * [MD_DR_HIST][rows][n_drones] the action-latency ring and act_count
 * (int32 [n_drones]) the number of actions entered into it, saturating at
 * MD_DR_HIST (both only with per-drone delays; zero act_count to start an
 * episode).  They may be NULL otherwise.  With per-drone sensor latency
 * (md_dr.obs_delay) obs_hist [MD_DR_OBS_HIST][20][n_drones] float32 is the
 * ring of observation rows and obs_count (int32 [n_drones]) the number of
 * rows entered into it, saturating at MD_DR_OBS_HIST (zero it to start an
 * episode); NULL otherwise. */
typedef struct md_state {
    float *p, *q, *v, *w, *pid_int, *rpm, *ctl;
    float *rpm_cmd, *act_hist;
    int32_t *act_count;
    float *wind; /* [5][n_drones] with wind gusts or turbulence, see md_set_wind */
    float *obs_hist;
    int32_t *obs_count;
} md_state;

typedef struct md_ctx md_ctx;

/* Library version string (static storage). */
const char *md_version(void);

/* Fill *out with the CF2X constants (Table "Drone model parameters",
 * Eq. 6 coefficients, Table "Default PIDControl gains"; g = 9.81 and the
 * ground-effect / drag coefficients of the predecessor simulator). */
md_status md_default_params_cf2x(md_params *out);

/* Derived constants of *p (HOVER_RPM, MAX_RPM, MAX_THRUST, h_clip). */
md_status md_derive(const md_params *p, md_derived *out);

/* Create a context on the current HIP device.  dt > 0 (s); aero_mask is an OR
 * of MD_AERO_*; act_type one of MD_ACT_RPM, MD_ACT_PID, MD_ACT_VEL,
 * MD_ACT_ATTITUDE, MD_ACT_DSL; ctrl_decim >= 1 is the number of physics steps
 * per controller update (zero-order hold in between; unused with MD_ACT_RPM).
 * MD_AERO_SURROGATE needs weights loaded by md_load_surrogate before stepping. */
md_status md_create(const md_params *p, float dt, uint32_t aero_mask, int act_type,
                    int ctrl_decim, md_ctx **out);

/* Destroy a context and free everything the library allocated for it.
 * Waits for the context's device work to finish.  NULL is ignored. */
void md_destroy(md_ctx *ctx);

/* Message of the last failed call on ctx (or of the last failed md_create
 * when ctx is NULL).  Never NULL. */
const char *md_last_error(const md_ctx *ctx);

/* Bind the ragged environment layout: h_env_offsets[n_envs + 1] (host,
 * int32, non-decreasing, off[0] = 0, off[n_envs] = n_drones).  Each
 * environment may hold 0..1024 drones, a context up to 2^25 drones
 * (MD_E_UNSUPPORTED beyond).  The library packs environments into
 * wavefront bins and uploads its lane tables (synchronously).  The offsets
 * are a host array because the packing runs on the host.  Re-binding
 * replaces the previous layout, frees the previous lane tables and makes the
 * context's captured rollouts stale (md_graph_launch refuses them). */
md_status md_bind_layout(md_ctx *ctx, const int32_t *h_env_offsets, int n_envs, int n_drones);

/* Advance every drone n_steps physics steps of dt, asynchronously on stream.
 *   s: device state, updated in place (read once, written once per call);
 *   d_action: [n_act][rows][N] with rows as listed for the action type (4, or
 *     7 for MD_ACT_DSL); n_act = n_steps if action_per_step else 1;
 *   d_obs: NULL, or [n_obs_slots][20][N] KIN observations: after step k the
 *     row block k mod n_obs_slots receives p[3], q[4], roll/pitch/yaw[3]
 *     (Z-Y-X), v[3], w[3], applied rotor speeds[4];
 *   step0: global index of the first step; controller updates run at steps
 *     with (step0 + k) mod ctrl_decim == 0.
 * Each drone's downwash terms are summed in an order fixed by the launch
 * configuration and the drone's place in its environment (ascending drone
 * order for lanes_per_drone 1 with pair_symmetric 0 or 1; see
 * md_launch_config), so results do not depend on how environments are packed
 * or on how a rollout is split into launches.  Errors: MD_E_LAYOUT if no
 * layout is bound, MD_E_INVALID_ARG for null required pointers or
 * n_steps < 0. */
md_status md_step(md_ctx *ctx, const md_state *s, const float *d_action, int action_per_step,
                  float *d_obs, int n_obs_slots, int n_steps, int64_t step0, void *stream);

/* Domain randomisation (Sec. "Domain randomization", Table "Recommended
 * domain-randomization ranges"), per drone, for the semi-implicit Euler step.
 *   scale [MD_DR_NSCALE][n_drones] factors on the nominal constants: mass,
 *     inertia (all three moments), arm length, kf, km, drag (c_xy and c_z),
 *     C_gnd, C1 (the downwash a drone receives), MAX_RPM, g, and four
 *     per-motor bias factors on the commanded rotor speeds;
 *   tau_mot [n_drones] motor time constant in s (0: no lag), nullable;
 *   delay [n_drones] action latency in steps, 0..MD_DR_HIST-1 (values
 *     outside are clamped to that range), nullable.
 * Per step k and drone: the action rows used are those of step
 * k - min(delay, act_count - 1), act_count counting the actions of the
 * episode up to step k and saturating at MD_DR_HIST; the command (the RPM action, or
 * the controller's output at controller steps, held in rpm_cmd) is
 * multiplied by the bias, clipped to [0, factor x MAX_RPM] and passed
 * through the lag n <- n + (1 - e^{-dt/tau})(c - n) (n = c for tau = 0);
 * Eq. 1-7 then use the drone's constants.  Controllers keep the nominal
 * constants; h_clip stays nominal.  All factors 1, tau 0 and delay 0
 * reproduce the plain step.
 * Sensor side (same table: observation noise and sensor latency), applied
 * to the KIN row of every step, which the controllers never see:
 *   noise_p, noise_v, noise_rpy, noise_w standard deviations (m, m/s, rad,
 *     rad/s) of zero-mean Gaussian noise added to position, velocity,
 *     roll/pitch/yaw and body rates (quaternion and rotor rows exact); the
 *     twelve normals of drone i at global step t are Box-Muller pairs of the
 *     24-bit uniforms of Philox4x32-10 blocks with counter (i, t low word,
 *     t high word, 2 + b), b = 0, 1, 2, key = seed (low word, high word), in
 *     the order p xyz, v xyz, rpy, w xyz;
 *   obs_bias [12][n_drones] a constant per-drone bias (the sticky
 *     per-episode observation bias recommended with the table) on the
 *     position, velocity, roll/pitch/yaw and body-rate rows, in that order,
 *     added before the noise, nullable;
 *   obs_delay [n_drones] sensor latency in steps, 0..MD_DR_OBS_HIST-1
 *     (clamped), nullable: the row returned at step k is the (noisy) row of
 *     step k - min(obs_delay, obs_count - 1), obs_count counting the rows of
 *     the episode up to step k and saturating at MD_DR_OBS_HIST; rows are
 *     counted whether or not the launch returns observations.
 * Both rings carry the latency across launches: at its end a launch leaves
 * its last MD_DR_HIST action rows in act_hist and its last MD_DR_OBS_HIST
 * rows in obs_hist, at slot (global step) mod the ring size, which is
 * exactly what the next launch can reach (earlier slots keep older entries).
 * Within a launch the delayed values come from the launch's own inputs and
 * rows, not from the rings.
 * The arrays are device memory owned by the caller and read by every later
 * md_step until the next call; NULL turns randomisation off.  Errors:
 * MD_E_INVALID_ARG for a null scale or a negative or non-finite noise level,
 * MD_E_UNSUPPORTED with MD_AERO_SURROGATE or MD_INTEG_RK4, or for a layout
 * with an environment of more than 512 drones (workgroups of the randomised
 * step hold at most 512 threads: waves_per_group <= 8; a launch
 * configuration beyond that is reset to the default). */
#define MD_DR_M 0
#define MD_DR_J 1
#define MD_DR_L 2
#define MD_DR_KF 3
#define MD_DR_KM 4
#define MD_DR_DRAG 5
#define MD_DR_GND 6
#define MD_DR_C1 7
#define MD_DR_MAXRPM 8
#define MD_DR_G 9
#define MD_DR_BIAS 10 /* rows 10..13: motors 0..3 */
#define MD_DR_NSCALE 14
#define MD_DR_HIST 32
#define MD_DR_OBS_HIST 8
typedef struct md_dr {
    const float *scale;
    const float *tau_mot;
    const int32_t *delay;
    float noise_p, noise_v, noise_rpy, noise_w;
    uint64_t seed;
    const int32_t *obs_delay;
    const float *obs_bias;
} md_dr;
md_status md_set_domain_randomization(md_ctx *ctx, const md_dr *dr);

/* Wind (Sec. "Wind and turbulence"): a world-frame force at the centre of
 * mass of every drone, added to the semi-implicit Euler step (with or without
 * domain randomisation), evaluated at the pre-step state of global step
 * t = step0 + k.  Models (OR of bits; all four = COMBINED, their sum):
 *   CONSTANT    F = 1/2 rho CdA |u| u, u = v_mean - v (air relative to drone);
 *   GUST        an idle drone starts a gust when a uniform draw is below
 *               gust_prob; heading uniform in [0, 2 pi); it lasts
 *               n_g = max(1, round(gust_duration / dt)) steps with force
 *               gust_amp (cos h, sin h, 0) sin(pi k / n_g) at its k-th step;
 *   DRYDEN      per-drone turbulence velocity x, per axis
 *               x <- alpha x + sigma sqrt(1 - alpha^2) xi, alpha = e^{-dt V/L},
 *               L_u = L_v = h / (0.177 + 8.23e-4 h)^1.2, L_w = h, h the height
 *               in feet clamped to [10, 1000] (MIL-F-8785C low altitude),
 *               V = dryden_airspeed; then F = 1/2 rho CdA |x| x;
 *   SINUSOIDAL  F = sin_amp [sin w t dt, cos w t dt, 0.3 sin 2 w t dt].
 * Random draws: Philox4x32-10 keyed by seed, counter (drone index, t low,
 * t high, stream): stream 0 gives the Dryden normals (Box-Muller), stream 1
 * the gust trigger and heading; uniforms are the top 24 bits x 2^-24.  State:
 * md_state.wind [5][N] = Dryden x, y, z (m/s), gust step (-1 idle), gust
 * heading (rad), caller-owned, required with GUST or DRYDEN (start it at
 * 0, 0, 0, -1, 0).  v_mean_drone: nullable device array [3][n_drones] of
 * per-drone mean winds replacing v_mean (the per-episode wind magnitude of
 * Table "Recommended domain-randomization ranges"), owned by the caller and
 * read by every later md_step.  NULL or models 0 turns wind off.  Errors:
 * MD_E_INVALID_ARG for unknown bits or negative parameters, MD_E_UNSUPPORTED
 * with MD_AERO_SURROGATE or MD_INTEG_RK4. */
#define MD_WIND_CONSTANT 1u
#define MD_WIND_GUST 2u
#define MD_WIND_DRYDEN 4u
#define MD_WIND_SINUSOIDAL 8u
#define MD_WIND_COMBINED 15u
typedef struct md_wind {
    uint32_t models;
    float v_mean[3];
    float rho, cd_area;
    float gust_prob, gust_duration, gust_amp;
    float dryden_sigma, dryden_airspeed;
    float sin_amp, sin_omega;
    uint64_t seed;
    const float *v_mean_drone;
} md_wind;
md_status md_set_wind(md_ctx *ctx, const md_wind *w);

/* Integrator of md_step (default MD_INTEG_EULER).  MD_INTEG_RK4 is the
 * classic fourth-order Runge-Kutta step, the integrator of the paper's MuJoCo
 * physics modes (Table "Physics modes"): rotor speeds, thrust and torques are
 * held over the step; the rigid-body state x = (p, v, q, w) with
 * p' = v, v' = F(x) / m, q' = q (x) [0, w] / 2, w' = J^-1 (tau - w x J w)
 * advances by dt/6 (k1 + 2 k2 + 2 k3 + k4); the aerodynamic terms of Eq. 4-6
 * are evaluated at every stage (the downwash from every drone's stage
 * position), rotations from the normalised stage quaternion, and the
 * quaternion is renormalised after the step.  Observations, controllers and
 * all other arguments of md_step behave as with MD_INTEG_EULER.  Errors:
 * MD_E_INVALID_ARG for an unknown value, MD_E_UNSUPPORTED with
 * MD_AERO_SURROGATE, domain randomisation or wind.  Switching to MD_INTEG_RK4 resets a launch
 * configuration with lanes_per_drone > 1 to the default. */
#define MD_INTEG_EULER 0
#define MD_INTEG_RK4 1
md_status md_set_integrator(md_ctx *ctx, int integrator);
md_status md_get_integrator(const md_ctx *ctx, int *out);

/* ------------------------------------------------------------------------
 * Launch configuration, autotuning and captured rollouts.
 * ---------------------------------------------------------------------- */

/* How md_step maps drones to the GPU.  Every valid configuration computes
 * the same physics: lanes_per_drone 1 with pair_symmetric 0 or 1 and any
 * waves_per_group give bitwise identical results; lanes_per_drone 2 or 4
 * split each neighbour sum into interleaved partial sums, and
 * pair_symmetric 2 and 3 sum each drone's terms shift by shift (different but
 * fixed summation orders, independent of how environments are packed; 2 and
 * 3 are bitwise identical). */
typedef struct md_launch_config {
    int lanes_per_drone; /* 1, 2 or 4 lanes share one drone's neighbour sweep */
    int unroll;          /* neighbour-loop unroll: 1, 2 or 4 (1 for pair_symmetric 2 and 3) */
    int waves_per_group; /* 1, 2, 4, 8 or 16 wave64s per workgroup (bin of 64*w/lpd slots) */
    int pair_symmetric;  /* 0: all ordered pairs; 1: each unordered pair once, terms routed
                            through an LDS matrix; 2: each unordered pair once, terms routed
                            between lanes by wave permutes (environments of at most 64
                            drones, packed so that none crosses a wavefront; unroll 1); 3: the
                            pairs of 2 as rotations of the whole wave, for layouts whose
                            non-empty environments all have one power-of-two size 2..64
                            (environments interleaved in their wave; unroll 1, the sweep
                            is unrolled in full).  1, 2 and 3 need lanes_per_drone 1. */
} md_launch_config;

md_status md_get_launch_config(const md_ctx *ctx, md_launch_config *out);
/* MD_E_INVALID_ARG if the configuration cannot hold the bound layout's
 * largest environment or its LDS need exceeds 64 KB, if lanes_per_drone
 * is not 1 for MD_INTEG_RK4 with the downwash term, or if pair_symmetric 3
 * does not fit the layout. */
md_status md_set_launch_config(md_ctx *ctx, md_launch_config *cfg);

/* Time every valid launch configuration for the bound layout on scratch
 * copies of s (s itself is not modified) over n_steps steps of d_action,
 * and select the fastest: the candidates run round robin, one warm-up round
 * and three timed ones, each scored by its median; the three best are timed
 * again as runs of six consecutive launches (the sustained load of a
 * rollout), which decide.  The choice is remembered in the JSON file
 * cache_path (NULL: the MD_AUTOTUNE_CACHE environment variable; empty: no
 * cache) under a signature of the layout, mask, action type and integrator; a cached
 * choice is reused unless force is non-zero.  Synchronous; allocates two
 * temporary state copies.  With the environment variable
 * MD_AUTOTUNE_VERBOSE=1 every candidate's time is printed to stderr. */
md_status md_autotune(md_ctx *ctx, const md_state *s, const float *d_action, int action_per_step,
                      int n_steps, int64_t step0, void *stream, const char *cache_path, int force);

/* md_autotune for callers that write the KIN-20 observation every step
 * (Sec. 3 observation spaces): every candidate also writes its rows into
 * d_obs (device, [n_obs_slots][20][n_drones] as for md_step, slot of step k
 * as md_step places it), so that the choice includes the cost of that write
 * stream, which some configurations overlap with the compute better than
 * others.  The contents of d_obs afterwards are unspecified; the caller's
 * state is not modified.  The choice is cached under the md_autotune
 * signature with an observation mark.  MD_E_INVALID_ARG for a null d_obs or
 * n_obs_slots < 1; otherwise as md_autotune. */
md_status md_autotune_obs(md_ctx *ctx, const md_state *s, const float *d_action, int action_per_step,
                          float *d_obs, int n_obs_slots, int n_steps, int64_t step0, void *stream,
                          const char *cache_path, int force);

/* A rollout of n_launches consecutive md_step launches of steps_per_launch
 * steps each (step0 advancing by steps_per_launch; per-step actions and, when
 * n_obs_slots >= steps_per_launch * n_launches, observation slots advance
 * with it), captured once into a HIP graph.  md_graph_launch replays the
 * whole rollout on a stream with the same pointers and step indices: keep
 * steps_per_launch * n_launches a multiple of ctrl_decim for replays to keep
 * the PID phase.  The captured kernels hold the context's lane tables and
 * settings as they were at capture, so the graph goes stale at the next call
 * that changes the context's layout (md_bind_layout), launch configuration
 * (md_set_launch_config, or md_autotune / md_autotune_obs choosing another),
 * integrator, domain randomisation, wind or surrogate (md_load_surrogate*,
 * md_set_surrogate_ood), and when the context is destroyed: md_graph_launch
 * then returns MD_E_LAYOUT and launches nothing (the message, while the
 * context lives, is in md_last_error).  Capture again after such a change.
 * md_graph_destroy is valid on a stale graph, also after md_destroy of its
 * context. */
typedef struct md_graph md_graph;
md_status md_rollout_graph_create(md_ctx *ctx, const md_state *s, const float *d_action,
                                  int action_per_step, float *d_obs, int n_obs_slots,
                                  int steps_per_launch, int n_launches, int64_t step0,
                                  void *stream, md_graph **out);
md_status md_graph_launch(md_graph *g, void *stream);
void md_graph_destroy(md_graph *g);

/* ------------------------------------------------------------------------
 * Learned aerodynamic residual (surrogate for Eq. 4-6).
 *
 * Network: 64 inputs (60 features, zero padded) -> 128 -> 128 -> 128 -> 6,
 * SiLU on the hidden layers; bfloat16 operands with fp32 accumulation (the
 * matrix products run on MFMA).  Inputs are standardised in fp32,
 * x' = (x - x_mean) * x_inv_std, then rounded to bfloat16; the 6 outputs are
 * standardised targets, y = y' * y_std + y_mean (body-frame force, N, and
 * torque, N m).  Parameters are one flat fp32 vector of MD_MLP_NPARAMS:
 * W1[128][64], b1[128], W2[128][128], b2[128], W3[128][128], b3[128],
 * W4[6][128], b4[6] (W row-major [out][in]).  The normalisation vector has
 * MD_MLP_NORM floats: x_mean[64], x_inv_std[64], y_mean[6], y_std[6].
 * ---------------------------------------------------------------------- */
#define MD_MLP_IN 64
#define MD_MLP_HIDDEN 128
#define MD_MLP_OUT 6
#define MD_MLP_NPARAMS 42118
#define MD_MLP_NORM 140

typedef struct md_mlp md_mlp;

/* A trainable network on the current device with buffers for batches of up
 * to max_batch samples.  Parameters start at zero; set them with
 * md_mlp_set_params. */
md_status md_mlp_create(int max_batch, md_mlp **out);
void md_mlp_destroy(md_mlp *m);
const char *md_mlp_last_error(const md_mlp *m);

/* Host <-> device copies of the flat fp32 parameters (synchronous).
 * set_params also resets the Adam moments and step count. */
md_status md_mlp_set_params(md_mlp *m, const float *h_params);
md_status md_mlp_get_params(const md_mlp *m, float *h_params);
/* Input / output standardisation (MD_MLP_NORM floats, synchronous). */
md_status md_mlp_set_norm(md_mlp *m, const float *h_norm);
md_status md_mlp_get_norm(const md_mlp *m, float *h_norm);

/* Forward pass of B <= max_batch samples: d_X [B][64] raw features (fp32,
 * device).  Keeps the activations for md_mlp_backward.  d_Y (nullable):
 * [B][6] de-standardised outputs (fp32, device).  Asynchronous on stream. */
md_status md_mlp_forward(md_mlp *m, const float *d_X, int B, float *d_Y, void *stream);

/* md_mlp_forward for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * The de-standardised outputs of B <= MD_MLP_NOALLOC_MAX_BATCH samples d_X
 * [B][64] (raw fp32 features, device) go to d_Y [B][6] (fp32, device,
 * required), computed by the same kernels as md_mlp_forward (bitwise the
 * same outputs), with every intermediate (standardised input, hidden
 * activations, standardised outputs) in a static device buffer of the
 * library instead of m's buffers: 2.6 MiB per GPU, taken on each GPU the
 * library runs on and held until the process ends; its address on m's device
 * is resolved by md_mlp_create.  Calls no allocator.  The activations are
 * not kept: md_mlp_backward still refers to the last md_mlp_forward.  Every
 * call on one GPU shares that buffer, so calls that overlap in time on one GPU
 * (other streams, other host threads) race; calls in order on one stream do
 * not.  Asynchronous on stream (a stream of m's device).  MD_E_INVALID_ARG
 * for a null pointer, B < 0 or B > MD_MLP_NOALLOC_MAX_BATCH; MD_E_HIP if
 * the buffer's address could not be resolved at md_mlp_create. */
#define MD_MLP_NOALLOC_MAX_BATCH 4096
md_status md_mlp_forward_noalloc(md_mlp *m, const float *d_X, int B, float *d_Y, void *stream);

/* Gradient of the mean squared error between the standardised outputs of
 * the last forward pass and the standardised targets d_T [B][6] (raw fp32,
 * device) with respect to every parameter, written to the network's gradient
 * buffer.  Deterministic (fixed reduction order).  Asynchronous. */
md_status md_mlp_backward(md_mlp *m, const float *d_T, int B, void *stream);
/* The gradient vector (synchronous copy) and the last backward's loss. */
md_status md_mlp_get_grads(const md_mlp *m, float *h_grads);
md_status md_mlp_loss(const md_mlp *m, double *out);

/* One Adam step (Kingma and Ba) on the fp32 parameters with the current
 * gradients: lr, beta1, beta2 in [0, 1), eps > 0.  Asynchronous. */
md_status md_mlp_adam(md_mlp *m, float lr, float beta1, float beta2, float eps, void *stream);

/* ------------------------------------------------------------------------
 * Surrogate inside the step, training data, and its judge.
 * ---------------------------------------------------------------------- */

/* Load trained parameters (h_params[MD_MLP_NPARAMS], h_norm[MD_MLP_NORM],
 * host fp32, layouts as for md_mlp_set_params / md_mlp_set_norm) into a
 * context created with MD_AERO_SURROGATE.  The library keeps bfloat16
 * copies on the device (about 85 KB).  Fallback: a drone with a same-env
 * neighbour among its 8 laterally nearest that sits above it by less than dz_ood
 * metres (0 < dz < dz_ood, where Eq. 6 is singular) takes the plain ground
 * effect + drag + downwash for that step.  Judge: every judge_stride-th
 * drone-step (a power of two; 0 = off) also evaluates the plain terms and
 * accumulates the surrogate's force error (md_judge_stats).  Synchronous. */
md_status md_load_surrogate(md_ctx *ctx, const float *h_params, const float *h_norm, float dz_ood,
                            int judge_stride);
/* Same, reading the parameters and normalisation of a trained md_mlp. */
md_status md_load_surrogate_mlp(md_ctx *ctx, const md_mlp *m, float dz_ood, int judge_stride);

/* Out-of-distribution fallback of the loaded surrogate (each bound 0 = that
 * check off; loading a network turns all three off): a drone with a world
 * velocity component beyond max_speed (m/s), a neighbour among its 8 whose
 * velocity differs from its own by more than max_rel_speed along an axis,
 * or a tilt beyond max_tilt (rad; qx^2 + qy^2 > sin^2(max_tilt / 2), formed
 * with rounded operations) takes the plain Eq. 4-6 terms for that step, as
 * at the downwash singularity.  The network is valid only where it was
 * trained.  MD_E_INVALID_ARG without a loaded surrogate or for a negative
 * bound. */
md_status md_set_surrogate_ood(md_ctx *ctx, float max_speed, float max_rel_speed, float max_tilt);

/* Training samples at the current state (bound layout, current device):
 * d_X [N][64] fp32 raw surrogate inputs (v_body[3], world up axis in the
 * body frame[3], rpm/HOVER_RPM[4], for the 8 nearest same-environment
 * neighbours by horizontal distance (ascending, ties to the lower index,
 * zeros when missing) p_j - p_i[3] and v_j - v_i[3], z[1], ground proximity
 * (h_clip / max(z, h_clip))^2 [1], zeros[4]);
 * d_Y [N][6] fp32: the aerodynamic force of the effects in aero_mask (a
 * subset of GND|DRAG|DW) in the body frame, then the torque (identically 0
 * for these centre-of-mass forces); d_nbr (nullable) [N][8] int32 neighbour
 * drone indices or -1.  Rotor speeds are the state's rpm.  Asynchronous. */
md_status md_datagen(md_ctx *ctx, const md_state *s, uint32_t aero_mask, float *d_X, float *d_Y,
                     int32_t *d_nbr, void *stream);

/* Judge statistics accumulated since the last reset (synchronous):
 * n_judged judged drone-steps; force_err2 = sum |F_surrogate - F_plain|^2;
 * force_ref2 = sum |F_plain|^2; torque_err2 = sum |tau_surrogate|^2 (plain
 * torque is 0); n_fallback drone-steps that took the plain terms;
 * n_drone_steps all drone-steps stepped; force_rel_err = sqrt(err2 / ref2)
 * (NaN when nothing was judged); n_nonfinite judged drone-steps whose
 * surrogate or plain force was not finite (left out of the sums and of
 * n_judged); n_knn_full drone-steps that ranked their whole environment for
 * the nearest neighbours (the others ranked their candidate list, see
 * md_set_surrogate_knn_reuse).  The plain terms of judged and fallback
 * drones are evaluated by the whole wave, one such drone at a time; their
 * downwash sum is added in a fixed order that depends only on the drone's
 * place in its environment. */
typedef struct md_judge {
    double n_judged, force_err2, force_ref2, torque_err2, n_fallback, n_drone_steps;
    double force_rel_err, n_nonfinite;
    double n_knn_full;
} md_judge;
md_status md_judge_stats(md_ctx *ctx, md_judge *out);
/* Zero the judge statistics (synchronous; a no-op without a loaded
 * surrogate).  MD_E_INVALID_ARG for a null context, MD_E_HIP if the device
 * reports an error. */
md_status md_judge_reset(md_ctx *ctx);

/* Region fallback of the loaded surrogate (each bound 0 = that check off;
 * loading a network turns both off): a drone with a neighbour among its 8
 * nearest inside the cylinder |dz| < near_dz, horizontal distance < near_r
 * (above or below: a near neighbour where Eq. 6 grows without bound and the
 * network has seen no samples), or farther than far_dz vertically, takes the
 * plain Eq. 4-6 terms for that step.  dz is the difference of the stored
 * heights and the squared horizontal distance is formed as for the neighbour
 * ranking (dx*dx + dy*dy, each operation rounded), compared with the float
 * of near_r^2.  MD_E_INVALID_ARG without a loaded surrogate or for a
 * negative bound. */
md_status md_set_surrogate_region(md_ctx *ctx, float near_dz, float near_r, float far_dz);

/* Neighbour candidate lists of the surrogate step (on after
 * md_load_surrogate*).  In bins whose largest environment has at least 14
 * drones, each drone ranks its whole environment only at a rebuild, keeps
 * its 12 laterally nearest and, until the next rebuild, ranks only those: a
 * bin rebuilds at the first step of every launch and whenever its largest
 * lateral displacement since the last rebuild reaches a quarter of its
 * smallest gap between a drone's 12th and 8th nearest distances (margins
 * shrunk against float32 rounding), which guarantees the same 8 neighbours
 * in the same order as ranking the whole environment.  Results are bitwise
 * those of reuse 0, which ranks every drone every step.  MD_E_INVALID_ARG
 * without a loaded surrogate. */
md_status md_set_surrogate_knn_reuse(md_ctx *ctx, int reuse);

#ifdef __cplusplus
}
#endif
#endif /* MD_H */
