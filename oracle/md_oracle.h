/*
 * md_oracle.h -- FP64 CPU oracle for the batched explicit quadrotor step.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, obviously-correct
 * reference of what the GPU path computes.  Only the test-suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load it.  It shares no
 * code, header, table or helper with the HIP library and never calls it.
 *
 * Every routine follows the paper (MuJoCo-Drones-Gym) step by step:
 *   - motor model and X mixer            : Sec. "Quadrotor Dynamics", Eq. (1)-(3)
 *   - ground effect                      : Sec. "Aerodynamic effects", Eq. (4)
 *   - blade drag                         : Sec. "Aerodynamic effects", Eq. (5)
 *   - downwash                           : Sec. "Aerodynamic effects", Eq. (6)
 *   - explicit integrator + exp map      : Sec. "Physics Modes", Eq. (7)
 *   - HOVER_RPM / MAX_RPM                : Sec. "Drone Models", Table "Drone model parameters"
 *   - cascaded PID                       : Sec. "Control", Eq. (9), Table "Default PIDControl gains"
 *   - KIN observation                    : Sec. "Observation types"
 *   - VEL / ATTITUDE / DSL-style PID     : Table "Action types", Sec. "Control"
 *   - classic RK4 variant                : Table "Physics modes"
 *   - domain randomisation               : Sec. "Domain randomization",
 *                                          Table "Recommended domain-randomization ranges"
 * Readings of silent / ambiguous passages are noted at each routine.
 *
 * Parity status: every routine is pinned by CPU tests (closed forms,
 * invariants, library routines, brute force) except the physical values of
 * C_gnd, c_xy, c_z and the h_clip rule (not printed in the paper) and the
 * PID allocation in saturated cases: "parity unpinned" for those.
 */
#ifndef MD_ORACLE_H
#define MD_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc_params {
    double m, L, kf, km, Ixx, Iyy, Izz, thrust2weight, r_p, g;
    double C_gnd, c_xy, c_z, C1, C2, C3, dw_dz_min;
    double pos_kp[3], pos_ki[3], pos_kd[3], pos_i_clamp;
    double att_kp[3], att_ki[3], att_kd[3], att_i_clamp;
    /* DSL-style PID: own gains and clamps, setpoint rate limits */
    double dsl_pos_kp[3], dsl_pos_ki[3], dsl_pos_kd[3], dsl_pos_i_clamp;
    double dsl_att_kp[3], dsl_att_ki[3], dsl_att_kd[3], dsl_att_i_clamp;
    double dsl_max_speed, dsl_max_yaw_rate;
} orc_params;

typedef struct orc_derived {
    double hover_rpm, max_rpm, max_thrust, h_clip;
} orc_derived;

/* SoA state, component-major: p[c*n + i]. */
typedef struct orc_state {
    double *p;       /* [3][n] world position, m                         */
    double *q;       /* [4][n] body->world quaternion, w,x,y,z            */
    double *v;       /* [3][n] world linear velocity, m/s                 */
    double *w;       /* [3][n] body angular velocity, rad/s               */
    double *pid_int; /* [6][n] position (0..2) and attitude (3..5) sums   */
    double *rpm;     /* [4][n] rotor speeds applied in the last step, RPM */
    double *ctl;     /* [4][n] DSL rate-limited setpoint x, y, z, yaw (DSL only) */
    /* domain randomisation only (orc_step_dr): */
    double *rpm_cmd;    /* [4][n] controller output held between updates (controller actions) */
    double *act_hist;   /* [ORC_DR_HIST][rows][n] action ring (with action latency) */
    int32_t *act_count; /* [n] actions entered since the ring was cleared (with latency) */
    /* wind only: [5][n] Dryden velocity x, y, z (m/s), gust step (-1 idle), gust heading (rad) */
    double *wind;
    /* sensor latency only: [ORC_DR_OBS_HIST][20][n] ring of noisy KIN rows, and
     * [n] rows entered since the ring was cleared */
    double *obs_hist;
    int32_t *obs_count;
} orc_state;

/* Wind (Sec. "Wind and turbulence"); readings at wind_force in md_oracle.c. */
enum { ORC_WIND_CONSTANT = 1, ORC_WIND_GUST = 2, ORC_WIND_DRYDEN = 4, ORC_WIND_SINUSOIDAL = 8 };
typedef struct orc_wind {
    uint32_t models;          /* OR of ORC_WIND_*; all four = COMBINED */
    double v_mean[3];         /* mean wind, world frame, m/s */
    double rho, cd_area;      /* air density (kg/m^3) and drag area C_d A (m^2) */
    double gust_prob;         /* per-step trigger probability of an idle drone */
    double gust_duration;     /* s */
    double gust_amp;          /* N */
    double dryden_sigma;      /* m/s */
    double dryden_airspeed;   /* V in alpha = exp(-dt V / L), m/s */
    double sin_amp, sin_omega;/* N, rad/s */
    uint64_t seed;            /* Philox key */
    const int32_t *drone_id;  /* [n] first Philox counter word of each drone
                               * (nullable: the drone's index), so that a
                               * sub-batch keeps the streams of its drones */
    const double *v_mean_drone; /* [3][n] per-drone mean wind (nullable:
                                 * v_mean for every drone) */
} orc_wind;
void orc_philox4x32(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Domain randomisation (Table "Recommended domain-randomization ranges"):
 * per-drone multiplicative factors, motor lag and action latency. */
enum {
    ORC_DR_M, ORC_DR_J, ORC_DR_L, ORC_DR_KF, ORC_DR_KM, ORC_DR_DRAG, ORC_DR_GND, ORC_DR_C1,
    ORC_DR_MAXRPM, ORC_DR_G, ORC_DR_BIAS, /* 4 rows: per-motor bias */
    ORC_DR_NSCALE = ORC_DR_BIAS + 4
};
#define ORC_DR_HIST 32
#define ORC_DR_OBS_HIST 8
typedef struct orc_dr {
    const double *scale;   /* [ORC_DR_NSCALE][n] */
    const double *tau_mot; /* [n] motor time constant, s (0 = no lag); nullable */
    const int32_t *delay;  /* [n] action latency in steps, 0..ORC_DR_HIST-1; nullable */
    /* sensor side: per-step Gaussian noise on the KIN rows (standard deviations
     * of position m, velocity m/s, roll/pitch/yaw rad, body rate rad/s; 0 =
     * off), Philox key, and sensor latency in steps 0..ORC_DR_OBS_HIST-1
     * (nullable) */
    double noise_p, noise_v, noise_rpy, noise_w;
    uint64_t seed;
    const int32_t *obs_delay;
    const int32_t *drone_id; /* [n] first Philox counter word (nullable: index) */
    const double *obs_bias;  /* [12][n] sticky bias on the position, velocity,
                              * roll/pitch/yaw and body-rate rows (nullable) */
} orc_dr;

enum { ORC_AERO_GND = 1, ORC_AERO_DRAG = 2, ORC_AERO_DW = 4, ORC_AERO_SURROGATE = 8 };
enum { ORC_ACT_RPM = 0, ORC_ACT_PID = 1, ORC_ACT_VEL = 2, ORC_ACT_ATTITUDE = 3, ORC_ACT_DSL = 4 };

void orc_params_cf2x(orc_params *P);
void orc_derive(const orc_params *P, orc_derived *D);

void orc_quat_to_rot(const double q[4], double R[9]);
void orc_quat_mul(const double a[4], const double b[4], double out[4]);
void orc_euler_zyx(const double q[4], double rpy[3]);

void orc_motor(const orc_params *P, const double n[4], double F[4], double *T, double tau[3]);
double orc_ground_effect(const orc_params *P, const orc_derived *D, const double n[4],
                         double pz, const double q[4]);
void orc_drag(const orc_params *P, const double n[4], const double q[4], const double v[3],
              double Fw[3]);
double orc_downwash_pair(const orc_params *P, const double p_low[3], const double p_other[3]);
void orc_pid(const orc_params *P, const orc_derived *D, double dt_c, const double p[3],
             const double q[4], const double v[3], const double w[3], const double target[4],
             double integ[6], double n_out[4]);
void orc_vel_ctrl(const orc_params *P, const orc_derived *D, double dt_c, const double q[4],
                  const double v[3], const double w[3], const double cmd[4], double integ[6],
                  double n_out[4]);
void orc_att_ctrl(const orc_params *P, const orc_derived *D, double dt_c, const double q[4],
                  const double w[3], const double cmd[4], double integ[6], double n_out[4]);
void orc_dsl_pid(const orc_params *P, const orc_derived *D, double dt_c, const double p[3],
                 const double q[4], const double v[3], const double w[3], const double cmd[7],
                 double integ[6], double sp[4], double n_out[4]);
int orc_action_rows(int act_type);
void orc_integrate(const orc_params *P, double dt, const double Fw[3], const double tau[3],
                   double p[3], double q[4], double v[3], double w[3]);

int orc_step(const orc_params *P, double dt, uint32_t aero_mask, int act_type, int ctrl_decim,
             int n_envs, const int32_t *env_offsets, int n_drones, orc_state *s,
             const double *action, int action_per_step, double *obs, int n_obs_slots,
             int n_steps, int64_t step0, int n_threads);

int orc_step_dr(const orc_params *P, double dt, uint32_t aero_mask, int act_type, int ctrl_decim,
                int n_envs, const int32_t *env_offsets, int n_drones, orc_state *s,
                const double *action, int action_per_step, double *obs, int n_obs_slots,
                int n_steps, int64_t step0, int n_threads, const orc_dr *dr);

/* orc_step with optional domain randomisation and optional wind (either may
 * be NULL). */
int orc_step_disturbed(const orc_params *P, double dt, uint32_t aero_mask, int act_type, int ctrl_decim,
                       int n_envs, const int32_t *env_offsets, int n_drones, orc_state *s,
                       const double *action, int action_per_step, double *obs, int n_obs_slots,
                       int n_steps, int64_t step0, int n_threads, const orc_dr *dr, const orc_wind *wind);

int orc_step_rk4(const orc_params *P, double dt, uint32_t aero_mask, int act_type, int ctrl_decim,
                 int n_envs, const int32_t *env_offsets, int n_drones, orc_state *s,
                 const double *action, int action_per_step, double *obs, int n_obs_slots,
                 int n_steps, int64_t step0, int n_threads);

/* ---- surrogate support ------------------------------------------------ */
int orc_knn(int n_envs, const int32_t *env_offsets, int n_drones, const double *p, int k,
            int32_t *nbr);
int orc_features(const orc_params *P, int n_envs, const int32_t *env_offsets, int n_drones,
                 const orc_state *s, const int32_t *nbr, int k, int n_feat, double *X);
int orc_aero_residual(const orc_params *P, uint32_t aero_mask, int n_envs,
                      const int32_t *env_offsets, int n_drones, const orc_state *s,
                      const double *rpm, double *Y);
int orc_mlp_forward(int n_layers, const int32_t *dims, const double *const *W,
                    const double *const *b, int B, const double *X, double *Y, double *acts,
                    int bf16_acts);
int orc_mlp_backward(int n_layers, const int32_t *dims, const double *const *W,
                     const double *const *b, int B, const double *X, const double *acts,
                     const double *dY, double *const *dW, double *const *db, double *dX);
void orc_adam(int n, double *param, const double *grad, double *m1, double *m2, double lr,
              double beta1, double beta2, double eps, int64_t t);
double orc_bf16_round(double x);

/* The trained surrogate as the oracle evaluates it (see orc_step_surrogate). */
typedef struct orc_net {
    const double *W[4]; /* [128][64], [128][128], [128][128], [6][128], bfloat16 values */
    const double *b[4]; /* [128], [128], [128], [6] */
    const double *norm; /* x_mean[64], x_inv_std[64], y_mean[6], y_std[6] */
    double dz_ood;
    /* out-of-distribution fallback (0 = that check off): own world speed
     * component above ood_speed, a neighbour's relative speed component
     * above ood_rel_speed, tilt above ood_tilt (rad) */
    double ood_speed, ood_rel_speed, ood_tilt;
    /* region fallback (0 = off): a neighbour among the 8 inside the cylinder
     * |dz| < near_dz, horizontal distance < near_r, or with |dz| > far_dz */
    double near_dz, near_r, far_dz;
} orc_net;

int orc_step_surrogate(const orc_params *P, double dt, int act_type, int ctrl_decim, int n_envs,
                       const int32_t *env_offsets, int n_drones, orc_state *s,
                       const double *action, int action_per_step, double *obs, int n_obs_slots,
                       int n_steps, int64_t step0, const orc_net *net, double *aero_out,
                       int32_t *fallback_out, int n_threads);

#ifdef __cplusplus
}
#endif
#endif
