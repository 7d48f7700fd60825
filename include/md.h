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
#define MD_E_UNSUPPORTED (-4) /* a valid request this build does not implement */
#define MD_E_LAYOUT (-5)      /* no layout bound, or state/layout sizes disagree */

/* Aerodynamic terms (Table "Physics modes" toggles), OR-able. */
#define MD_AERO_GND 1u       /* ground effect, Eq. 4 */
#define MD_AERO_DRAG 2u      /* blade drag, Eq. 5 */
#define MD_AERO_DW 4u        /* pairwise downwash within an environment, Eq. 6 */
#define MD_AERO_SURROGATE 8u /* learned residual replaces GND|DRAG|DW (exclusive with them) */

/* Action types (Table "Action types"). */
#define MD_ACT_RPM 0 /* action[4][N]: rotor speeds in rev/min, clipped to [0, MAX_RPM] */
#define MD_ACT_PID 1 /* action[4][N]: waypoint x, y, z (m), yaw (rad) for the cascaded PID */

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
} md_params;

/* Quantities derived from md_params (Sec. "Drone Models"; h_clip under Eq. 4). */
typedef struct md_derived {
    double hover_rpm, max_rpm, max_thrust, h_clip;
} md_derived;

/* Device state of n_drones drones, each pointer [rows][n_drones] float32:
 * p[3] world position; q[4] body->world unit quaternion (w,x,y,z);
 * v[3] world velocity; w[3] body angular velocity; pid_int[6] PID integral
 * sums (position xyz, then roll/pitch/yaw; only read/written in PID mode,
 * may be NULL otherwise); rpm[4] rotor speeds applied in the last step
 * (the held command between PID updates). */
typedef struct md_state {
    float *p, *q, *v, *w, *pid_int, *rpm;
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
 * of MD_AERO_*; act_type MD_ACT_RPM or MD_ACT_PID; ctrl_decim >= 1 is the
 * number of physics steps per PID update (zero-order hold in between).
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
 * environment may hold 0..1024 drones.  The library packs environments into
 * wavefront bins and uploads its lane tables (synchronously).  Re-binding
 * replaces the previous layout and invalidates captured graphs. */
md_status md_bind_layout(md_ctx *ctx, const int32_t *h_env_offsets, int n_envs, int n_drones);

/* Advance every drone n_steps physics steps of dt, asynchronously on stream.
 *   s: device state, updated in place (read once, written once per call);
 *   d_action: RPM mode -> [n_act][4][N] rotor speeds; PID mode -> [n_act][4][N]
 *     waypoints (x, y, z, yaw); n_act = n_steps if action_per_step else 1;
 *   d_obs: NULL, or [n_obs_slots][20][N] KIN observations: after step k the
 *     row block k mod n_obs_slots receives p[3], q[4], roll/pitch/yaw[3]
 *     (Z-Y-X), v[3], w[3], applied rotor speeds[4];
 *   step0: global index of the first step; PID updates run at steps with
 *     (step0 + k) mod ctrl_decim == 0.
 * Sums over neighbours run in ascending drone order, so results do not depend
 * on how environments are packed.  Errors: MD_E_LAYOUT if no layout is bound,
 * MD_E_INVALID_ARG for null required pointers or n_steps < 0. */
md_status md_step(md_ctx *ctx, const md_state *s, const float *d_action, int action_per_step,
                  float *d_obs, int n_obs_slots, int n_steps, int64_t step0, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* MD_H */
