/*
 * md_oracle.c -- FP64 CPU oracle for the batched explicit quadrotor step.
 *
 * TEST INFRASTRUCTURE ONLY (tests, the smoke check and the benchmark's CPU
 * baseline leg).  Plain loops in double precision, written from the paper's
 * equations in the paper's order.  No blocking, fusion or reordering; the
 * only parallelism is an OpenMP loop over independent environments, which
 * does not change any drone's arithmetic.  Shares nothing with the HIP path.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fPIC -shared (see build_oracle.py)
 */
#include "md_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------------ */
/* Constants.                                                                */
/* ------------------------------------------------------------------------ */

/* Table "Drone model parameters" (CF2X column), the downwash coefficients
 * printed with Eq. (6), and Table "Default PIDControl gains".
 * Readings (not printed in the paper):
 *   g = 9.81 m/s^2 (MuJoCo's default gravity);
 *   C_gnd, c_xy, c_z: the paper states its aerodynamic formulae and drone
 *   parameters are identical to its predecessor's; these are that simulator's
 *   CF2X values -- their physical values are "parity unpinned".
 *   Units: n in rev/min and kf, km per RPM^2 (the table's rad/s units are
 *   inconsistent with hover at ~14.5k RPM and with Eq. (5)'s 2*pi*n/60). */
void orc_params_cf2x(orc_params *P)
{
    memset(P, 0, sizeof *P);
    P->m = 0.027;
    P->L = 0.0397;
    P->thrust2weight = 2.25;
    P->Ixx = 1.4e-5;
    P->Iyy = 1.4e-5;
    P->Izz = 2.17e-5;
    P->kf = 3.16e-10;
    P->km = 7.94e-12;
    P->r_p = 0.02325;
    P->g = 9.81;
    P->C_gnd = 11.36359;
    P->c_xy = 9.1785e-7;
    P->c_z = 10.311e-7;
    P->C1 = 2267.18;
    P->C2 = 0.16;
    P->C3 = -0.11;
    P->dw_dz_min = 0.0;
    const double pkp[3] = {0.4, 0.4, 1.0}, pki[3] = {0.01, 0.01, 0.01}, pkd[3] = {0.9, 0.9, 2.0};
    const double akp[3] = {2e-3, 2e-3, 1e-3}, aki[3] = {0.0, 0.0, 1e-4}, akd[3] = {5e-4, 5e-4, 2e-4};
    for (int c = 0; c < 3; ++c) {
        P->pos_kp[c] = pkp[c];
        P->pos_ki[c] = pki[c];
        P->pos_kd[c] = pkd[c];
        P->att_kp[c] = akp[c];
        P->att_ki[c] = aki[c];
        P->att_kd[c] = akd[c];
    }
    P->pos_i_clamp = 2.0;
    P->att_i_clamp = 0.5;
    /* Sec. "Control", DSLPIDControl: halved integral clamps and setpoint rate
     * limits of 2.0 m/s and pi rad/s.  Reading: its retuned gains are not
     * printed; the defaults repeat the PIDControl gains (parity unpinned for
     * any other tuning). */
    for (int c = 0; c < 3; ++c) {
        P->dsl_pos_kp[c] = pkp[c];
        P->dsl_pos_ki[c] = pki[c];
        P->dsl_pos_kd[c] = pkd[c];
        P->dsl_att_kp[c] = akp[c];
        P->dsl_att_ki[c] = aki[c];
        P->dsl_att_kd[c] = akd[c];
    }
    P->dsl_pos_i_clamp = 1.0;
    P->dsl_att_i_clamp = 0.25;
    P->dsl_max_speed = 2.0;
    P->dsl_max_yaw_rate = M_PI;
}

/* Sec. "Drone Models": HOVER_RPM = sqrt(m g / (4 kf)); MAX_RPM from
 * (m, g, kf, T/W): the speed at which four rotors give T/W times the weight.
 * Reading for h_clip (Sec. "Aerodynamic effects", Eq. (4); the text ties the
 * clip height to r_p and MAX_THRUST without a formula): the height at which
 * one rotor's ground-effect force at MAX_RPM equals MAX_THRUST/15. */
void orc_derive(const orc_params *P, orc_derived *D)
{
    D->hover_rpm = sqrt(P->m * P->g / (4.0 * P->kf));
    D->max_rpm = sqrt(P->thrust2weight * P->m * P->g / (4.0 * P->kf));
    D->max_thrust = 4.0 * P->kf * D->max_rpm * D->max_rpm;
    D->h_clip = 0.25 * P->r_p *
                sqrt(15.0 * P->C_gnd * P->kf * D->max_rpm * D->max_rpm / D->max_thrust);
}

/* ------------------------------------------------------------------------ */
/* Quaternion helpers, [w, x, y, z] body->world (Sec. "Notation").           */
/* ------------------------------------------------------------------------ */

void orc_quat_to_rot(const double q[4], double R[9])
{
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1.0 - 2.0 * (y * y + z * z);
    R[1] = 2.0 * (x * y - w * z);
    R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z);
    R[4] = 1.0 - 2.0 * (x * x + z * z);
    R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y);
    R[7] = 2.0 * (y * z + w * x);
    R[8] = 1.0 - 2.0 * (x * x + y * y);
}

/* Hamilton product a (x) b. */
void orc_quat_mul(const double a[4], const double b[4], double o[4])
{
    o[0] = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
    o[1] = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
    o[2] = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
    o[3] = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
}

/* Roll, pitch, yaw of the KIN observation (Sec. "Observation types").
 * Reading: intrinsic Z-Y-X (yaw, pitch, roll). */
void orc_euler_zyx(const double q[4], double rpy[3])
{
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    double sp = 2.0 * (w * y - z * x);
    if (sp > 1.0) sp = 1.0;
    if (sp < -1.0) sp = -1.0;
    rpy[0] = atan2(2.0 * (w * x + y * z), 1.0 - 2.0 * (x * x + y * y));
    rpy[1] = asin(sp);
    rpy[2] = atan2(2.0 * (w * z + x * y), 1.0 - 2.0 * (y * y + z * z));
}

/* ------------------------------------------------------------------------ */
/* Forces.                                                                   */
/* ------------------------------------------------------------------------ */

/* Eq. (1)-(3): F_i = kf n_i^2, tau_z,i = (-1)^{m_i} km n_i^2, X-config roll
 * and pitch torques with lever L/sqrt(2), collective thrust T = sum F_i.
 * Reading of the alternating sign: m = (1, 0, 1, 0), i.e. yaw signs
 * (-, +, -, +) for motors 0..3. */
void orc_motor(const orc_params *P, const double n[4], double F[4], double *T, double tau[3])
{
    static const int m_sign[4] = {1, 0, 1, 0};
    double tz = 0.0, Tsum = 0.0;
    for (int i = 0; i < 4; ++i) {
        F[i] = P->kf * n[i] * n[i];
        Tsum += F[i];
        const double s = (m_sign[i] ? -1.0 : 1.0);
        tz += s * P->km * n[i] * n[i];
    }
    const double l = P->L / sqrt(2.0);
    tau[0] = l * (F[0] + F[1] - F[2] - F[3]);
    tau[1] = l * (-F[0] + F[1] + F[2] - F[3]);
    tau[2] = tz;
    *T = Tsum;
}

/* Eq. (4): extra vertical force C_gnd * sum(kf n_i^2) * (r_p / (4 h))^2,
 * h = max(p_z, h_clip), applied only while |roll| and |pitch| < pi/2.
 * Reading: one h taken at the body's centre, force along world +z. */
double orc_ground_effect(const orc_params *P, const orc_derived *D, const double n[4],
                         double pz, const double q[4])
{
    double rpy[3];
    orc_euler_zyx(q, rpy);
    if (!(fabs(rpy[0]) < 0.5 * M_PI && fabs(rpy[1]) < 0.5 * M_PI)) return 0.0;
    const double h = (pz > D->h_clip) ? pz : D->h_clip;
    double s = 0.0;
    for (int i = 0; i < 4; ++i) s += P->kf * n[i] * n[i];
    const double r = P->r_p / (4.0 * h);
    return P->C_gnd * s * r * r;
}

/* Eq. (5): body-frame drag -diag(c_xy, c_xy, c_z) * (sum 2 pi n_i / 60) * v_body,
 * rotated back to the world frame: F_w = R * f_body with v_body = R^T v. */
void orc_drag(const orc_params *P, const double n[4], const double q[4], const double v[3],
              double Fw[3])
{
    double R[9];
    orc_quat_to_rot(q, R);
    double vb[3];
    for (int a = 0; a < 3; ++a) vb[a] = R[0 * 3 + a] * v[0] + R[1 * 3 + a] * v[1] + R[2 * 3 + a] * v[2];
    double S = 0.0;
    for (int i = 0; i < 4; ++i) S += 2.0 * M_PI * n[i] / 60.0;
    const double c[3] = {P->c_xy, P->c_xy, P->c_z};
    double fb[3];
    for (int a = 0; a < 3; ++a) fb[a] = -c[a] * S * vb[a];
    for (int a = 0; a < 3; ++a) Fw[a] = R[a * 3 + 0] * fb[0] + R[a * 3 + 1] * fb[1] + R[a * 3 + 2] * fb[2];
}

/* Eq. (6): the drone at p_low receives -alpha exp(-(dxy/beta)^2 / 2) along
 * world z from a drone at p_other above it (dz = z_other - z_low > 0) with
 * lateral distance dxy < 10 m; alpha = C1 (r_p / (4 dz))^2, beta = C2 dz + C3.
 * Readings: strict dz > 0; beta enters only squared, and for beta = 0 the
 * Gaussian is 1 at dxy = 0 and 0 elsewhere (its limit); the optional floor
 * dw_dz_min (0 = off, the literal equation) bounds dz from below. */
double orc_downwash_pair(const orc_params *P, const double p_low[3], const double p_other[3])
{
    const double dz = p_other[2] - p_low[2];
    const double dx = p_other[0] - p_low[0];
    const double dy = p_other[1] - p_low[1];
    const double dxy = sqrt(dx * dx + dy * dy);
    if (!(dz > 0.0 && dxy < 10.0)) return 0.0;
    double dze = dz;
    if (P->dw_dz_min > 0.0 && dze < P->dw_dz_min) dze = P->dw_dz_min;
    const double r = P->r_p / (4.0 * dze);
    const double alpha = P->C1 * r * r;
    const double beta = P->C2 * dze + P->C3;
    double gauss;
    if (beta == 0.0) {
        gauss = (dxy == 0.0) ? 1.0 : 0.0;
    } else {
        const double t = dxy / beta;
        gauss = exp(-0.5 * t * t);
    }
    return -alpha * gauss;
}

/* ------------------------------------------------------------------------ */
/* Cascaded PID (Sec. "Control", Eq. (9), Table "Default PIDControl gains"). */
/* ------------------------------------------------------------------------ */

static double wrap_pi(double a)
{
    /* into [-pi, pi) */
    return a - 2.0 * M_PI * floor((a + M_PI) / (2.0 * M_PI));
}

static double clampd(double x, double lo, double hi)
{
    return x < lo ? lo : (x > hi ? hi : x);
}

/* Attitude PID and allocation shared by the controllers.  Attitude error
 * e = (roll* - roll, pitch* - pitch, e_yaw); I += e dt_c clamped to +-clamp;
 * tau = Kp e + Ki I + Kd (w*_z z_hat - w) where the yaw-rate target w*_z is 0
 * for the waypoint controllers; then the exact allocation inverse (rows of
 * the mixer are orthogonal), rotor forces clipped to [0, kf MAX_RPM^2]. */
static void attitude_allocate(const orc_params *P, const orc_derived *D, double dt_c,
                              const double rpy[3], const double w[3], double T, double roll_t,
                              double pitch_t, double e_yaw, double wz_t, const double kp[3],
                              const double ki[3], const double kd[3], double clamp,
                              double integ_att[3], double n_out[4])
{
    const double ea[3] = {roll_t - rpy[0], pitch_t - rpy[1], e_yaw};
    const double wt[3] = {0.0, 0.0, wz_t};
    double tau[3];
    for (int c = 0; c < 3; ++c) {
        integ_att[c] = clampd(integ_att[c] + ea[c] * dt_c, -clamp, clamp);
        tau[c] = kp[c] * ea[c] + ki[c] * integ_att[c] + kd[c] * (wt[c] - w[c]);
    }
    const double l = P->L / sqrt(2.0), kap = P->km / P->kf;
    static const double sx[4] = {1, 1, -1, -1}, sy[4] = {-1, 1, 1, -1}, sz[4] = {-1, 1, -1, 1};
    const double fmax = P->kf * D->max_rpm * D->max_rpm;
    for (int i = 0; i < 4; ++i) {
        double F = 0.25 * (T + sx[i] * tau[0] / l + sy[i] * tau[1] / l + sz[i] * tau[2] / kap);
        F = clampd(F, 0.0, fmax);
        n_out[i] = sqrt(F / P->kf);
    }
}

/* Thrust and small-angle attitude target from a desired acceleration a*
 * (gravity included): T = m |a*|, roll* = (a_x sin psi - a_y cos psi) / g,
 * pitch* = (a_x cos psi + a_y sin psi) / g at the current yaw psi. */
static void thrust_direction(const orc_params *P, const double acc[3], double yaw, double *T,
                             double *roll_t, double *pitch_t)
{
    *T = P->m * sqrt(acc[0] * acc[0] + acc[1] * acc[1] + acc[2] * acc[2]);
    const double sps = sin(yaw), cps = cos(yaw);
    *roll_t = (acc[0] * sps - acc[1] * cps) / P->g;
    *pitch_t = (acc[0] * cps + acc[1] * sps) / P->g;
}

/* Position loop: a* = Kp e + Ki int(e) + Kd (v* - v) + g z_hat with v* = 0;
 * T = m |a*|.  Readings: the integrals advance by e * dt_c and are clamped
 * before use; the small-angle attitude target is the near-hover inversion of
 * the thrust direction at the current yaw (thrust_direction); the attitude
 * PID acts on (roll*-roll, pitch*-pitch, wrap(yaw*-yaw)) with derivative
 * term Kd (0 - omega); the allocation T,tau = M [kf n_i^2] is inverted exactly
 * and each rotor force is clipped to [0, kf MAX_RPM^2] (parity unpinned when
 * saturated). */
void orc_pid(const orc_params *P, const orc_derived *D, double dt_c, const double p[3],
             const double q[4], const double v[3], const double w[3], const double target[4],
             double integ[6], double n_out[4])
{
    double e[3], acc[3];
    for (int c = 0; c < 3; ++c) {
        e[c] = target[c] - p[c];
        integ[c] = clampd(integ[c] + e[c] * dt_c, -P->pos_i_clamp, P->pos_i_clamp);
        acc[c] = P->pos_kp[c] * e[c] + P->pos_ki[c] * integ[c] + P->pos_kd[c] * (0.0 - v[c]);
    }
    acc[2] += P->g;
    double rpy[3], T, rt, pt;
    orc_euler_zyx(q, rpy);
    thrust_direction(P, acc, rpy[2], &T, &rt, &pt);
    attitude_allocate(P, D, dt_c, rpy, w, T, rt, pt, wrap_pi(target[3] - rpy[2]), 0.0, P->att_kp,
                      P->att_ki, P->att_kd, P->att_i_clamp, integ + 3, n_out);
}

/* VEL action (Table "Action types": body-frame [v_x, v_y, v_z, w_z], PID inner
 * loop).  Readings: the velocity is given in the heading frame (yaw-only
 * rotation of the world frame), v* = R_z(psi) (v_x, v_y, v_z); the position
 * loop is bypassed, a* = Kd (v* - v) + g z_hat (its position integrals are
 * left unchanged); the yaw channel tracks the rate, e_yaw = 0 and w*_z = w_z
 * command; roll and pitch as in the PID. */
void orc_vel_ctrl(const orc_params *P, const orc_derived *D, double dt_c, const double q[4],
                  const double v[3], const double w[3], const double cmd[4], double integ[6],
                  double n_out[4])
{
    double rpy[3];
    orc_euler_zyx(q, rpy);
    const double c = cos(rpy[2]), s = sin(rpy[2]);
    const double vt[3] = {c * cmd[0] - s * cmd[1], s * cmd[0] + c * cmd[1], cmd[2]};
    double acc[3];
    for (int k = 0; k < 3; ++k) acc[k] = P->pos_kd[k] * (vt[k] - v[k]);
    acc[2] += P->g;
    double T, rt, pt;
    thrust_direction(P, acc, rpy[2], &T, &rt, &pt);
    attitude_allocate(P, D, dt_c, rpy, w, T, rt, pt, 0.0, cmd[3], P->att_kp, P->att_ki,
                      P->att_kd, P->att_i_clamp, integ + 3, n_out);
}

/* ATTITUDE action (Table "Action types": thrust + roll + pitch + yaw-rate,
 * mixer to RPM).  Readings: thrust is the collective thrust in newtons, roll
 * and pitch are Z-Y-X angle targets in radians, the yaw channel tracks the
 * rate (e_yaw = 0, w*_z = command); the attitude PID and allocation as in
 * the PID. */
void orc_att_ctrl(const orc_params *P, const orc_derived *D, double dt_c, const double q[4],
                  const double w[3], const double cmd[4], double integ[6], double n_out[4])
{
    double rpy[3];
    orc_euler_zyx(q, rpy);
    attitude_allocate(P, D, dt_c, rpy, w, cmd[0], cmd[1], cmd[2], 0.0, cmd[3], P->att_kp,
                      P->att_ki, P->att_kd, P->att_i_clamp, integ + 3, n_out);
}

/* DSL-style PID (Sec. "Control", DSLPIDControl): the waypoint controller
 * with its own gains, halved integral clamps, a position setpoint that moves
 * toward the waypoint by at most dsl_max_speed * dt_c (in norm) per update, a
 * yaw setpoint that turns toward the waypoint yaw by at most
 * dsl_max_yaw_rate * dt_c, and a feed-forward acceleration added to the
 * position-loop output before the thrust direction.  cmd = (x, y, z, yaw,
 * a_ff x, y, z); sp holds the setpoint (x, y, z, yaw) between updates.
 * Reading: v* = 0, as in the PID. */
void orc_dsl_pid(const orc_params *P, const orc_derived *D, double dt_c, const double p[3],
                 const double q[4], const double v[3], const double w[3], const double cmd[7],
                 double integ[6], double sp[4], double n_out[4])
{
    double d[3], dn = 0.0;
    for (int c = 0; c < 3; ++c) {
        d[c] = cmd[c] - sp[c];
        dn += d[c] * d[c];
    }
    dn = sqrt(dn);
    const double step = P->dsl_max_speed * dt_c;
    const double sc = (dn > step) ? step / dn : 1.0;
    for (int c = 0; c < 3; ++c) sp[c] += sc * d[c];
    const double ymax = P->dsl_max_yaw_rate * dt_c;
    sp[3] = wrap_pi(sp[3] + clampd(wrap_pi(cmd[3] - sp[3]), -ymax, ymax));
    double e[3], acc[3];
    for (int c = 0; c < 3; ++c) {
        e[c] = sp[c] - p[c];
        integ[c] = clampd(integ[c] + e[c] * dt_c, -P->dsl_pos_i_clamp, P->dsl_pos_i_clamp);
        acc[c] = P->dsl_pos_kp[c] * e[c] + P->dsl_pos_ki[c] * integ[c] +
                 P->dsl_pos_kd[c] * (0.0 - v[c]) + cmd[4 + c];
    }
    acc[2] += P->g;
    double rpy[3], T, rt, pt;
    orc_euler_zyx(q, rpy);
    thrust_direction(P, acc, rpy[2], &T, &rt, &pt);
    attitude_allocate(P, D, dt_c, rpy, w, T, rt, pt, wrap_pi(sp[3] - rpy[2]), 0.0, P->dsl_att_kp,
                      P->dsl_att_ki, P->dsl_att_kd, P->dsl_att_i_clamp, integ + 3, n_out);
}

int orc_action_rows(int act_type) { return act_type == ORC_ACT_DSL ? 7 : 4; }

/* One controller update of drone i for the non-RPM action types. */
static void controller(const orc_params *P, const orc_derived *D, int act_type, double dt_c, int N,
                       int i, const double cmd[7], const double p[3], const double q[4],
                       const double v[3], const double w[3], orc_state *s, double n[4])
{
    double integ[6], sp[4];
    for (int c = 0; c < 6; ++c) integ[c] = s->pid_int[c * N + i];
    if (act_type == ORC_ACT_PID) {
        orc_pid(P, D, dt_c, p, q, v, w, cmd, integ, n);
    } else if (act_type == ORC_ACT_VEL) {
        orc_vel_ctrl(P, D, dt_c, q, v, w, cmd, integ, n);
    } else if (act_type == ORC_ACT_ATTITUDE) {
        orc_att_ctrl(P, D, dt_c, q, w, cmd, integ, n);
    } else {
        for (int c = 0; c < 4; ++c) sp[c] = s->ctl[c * N + i];
        orc_dsl_pid(P, D, dt_c, p, q, v, w, cmd, integ, sp, n);
        for (int c = 0; c < 4; ++c) s->ctl[c * N + i] = sp[c];
    }
    for (int c = 0; c < 6; ++c) s->pid_int[c * N + i] = integ[c];
}

/* ------------------------------------------------------------------------ */
/* Integrator (Sec. "Physics Modes", Eq. (7)).                                */
/* ------------------------------------------------------------------------ */

/* Newton-Euler with a = F_w / m and omega_dot = J^-1 (tau - omega x J omega).
 * Readings: semi-implicit Euler (v and omega first; p uses the new v; q uses
 * the new omega), omega in the body frame; the exponential map of Eq. (7),
 * with Lambda(omega) the quaternion-product matrix that carries the 1/2 of
 * q_dot = Lambda q, equals q <- q (x) [cos th, sin th omega/|omega|] with
 * th = |omega| dt / 2; q is renormalised every step. */
void orc_integrate(const orc_params *P, double dt, const double Fw[3], const double tau[3],
                   double p[3], double q[4], double v[3], double w[3])
{
    const double J[3] = {P->Ixx, P->Iyy, P->Izz};
    double Jw[3] = {J[0] * w[0], J[1] * w[1], J[2] * w[2]};
    double cr[3] = {w[1] * Jw[2] - w[2] * Jw[1], w[2] * Jw[0] - w[0] * Jw[2],
                    w[0] * Jw[1] - w[1] * Jw[0]};
    double wd[3];
    for (int c = 0; c < 3; ++c) wd[c] = (tau[c] - cr[c]) / J[c];
    for (int c = 0; c < 3; ++c) {
        v[c] += dt * (Fw[c] / P->m);
        w[c] += dt * wd[c];
    }
    for (int c = 0; c < 3; ++c) p[c] += dt * v[c];
    const double nw = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    if (nw > 0.0) {
        const double th = 0.5 * nw * dt;
        const double s = sin(th) / nw;
        const double r[4] = {cos(th), s * w[0], s * w[1], s * w[2]};
        double o[4];
        orc_quat_mul(q, r, o);
        memcpy(q, o, sizeof o);
    }
    const double nq = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    for (int c = 0; c < 4; ++c) q[c] /= nq;
}

/* ------------------------------------------------------------------------ */
/* Whole batched step.                                                       */
/* ------------------------------------------------------------------------ */

/* ------------------------------------------------------------------------ */
/* Wind (Sec. "Wind and turbulence").                                        */
/* ------------------------------------------------------------------------ */

/* Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC 2011): ten rounds of two 32x32 -> 64-bit products of
 * counter words with the round multipliers, the high halves xored with the
 * other counter words and the round key, the key bumped by the Weyl
 * constants between rounds. */
void orc_philox4x32(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

/* A 24-bit uniform in [0, 1) from the top bits of a 32-bit word (exact in
 * binary32 and binary64). */
static double unit24(uint32_t x) { return (double)(x >> 8) * (1.0 / 16777216.0); }

/* The random words of drone i at global step t: stream 0 feeds the Dryden
 * normals, stream 1 the gust trigger and heading. */
static void wind_words(const orc_wind *W, int32_t i, int64_t t, uint32_t stream, uint32_t out[4])
{
    const uint32_t ctr[4] = {(uint32_t)i, (uint32_t)((uint64_t)t & 0xffffffffu), (uint32_t)((uint64_t)t >> 32),
                             stream};
    const uint32_t key[2] = {(uint32_t)(W->seed & 0xffffffffu), (uint32_t)(W->seed >> 32)};
    orc_philox4x32(ctr, key, out);
}

/* World-frame wind force on drone i at global step t (pre-step position p and
 * velocity v); ws = the drone's wind state (Dryden velocity x, y, z in m/s;
 * gust step counter, -1 when idle; gust heading in rad), updated in place.
 * Readings (the paper gives the model forms, not their constants or units):
 *   CONSTANT   F = 1/2 rho CdA |u| u with u = v_mean - v, the air velocity
 *              relative to the drone;
 *   DRYDEN     per axis x <- alpha x + sigma sqrt(1 - alpha^2) xi, alpha =
 *              exp(-dt V / L), L_u = L_v = h / (0.177 + 8.23e-4 h)^1.2 and
 *              L_w = h with h the height in feet (the MIL-F-8785C low-altitude
 *              scales) clamped to [10, 1000] ft, lengths back in metres; the
 *              state is advanced first, then its drag 1/2 rho CdA |x| x acts;
 *              xi from Box-Muller on Philox words;
 *   GUST       an idle drone starts a gust when a uniform is below gust_prob,
 *              heading uniform in [0, 2 pi); a gust lasts n_g = round(T / dt)
 *              steps (at least 1) and pushes with gust_amp (cos h, sin h, 0)
 *              sin(pi k / n_g) at its k-th step;
 *   SINUSOIDAL F = A [sin w tau, cos w tau, 0.3 sin 2 w tau], tau = t dt;
 *   COMBINED   the sum of the selected models. */
static void wind_force(const orc_wind *W, double dt, int64_t t, int32_t i, int32_t li, const double p[3],
                       const double v[3], double *ws, int N, double F[3])
{
    F[0] = F[1] = F[2] = 0.0;
    const double k = 0.5 * W->rho * W->cd_area;
    if (W->models & ORC_WIND_CONSTANT) {
        double vm[3];
        for (int c = 0; c < 3; ++c) vm[c] = W->v_mean_drone ? W->v_mean_drone[(size_t)c * N + li] : W->v_mean[c];
        const double u[3] = {vm[0] - v[0], vm[1] - v[1], vm[2] - v[2]};
        const double un = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
        for (int c = 0; c < 3; ++c) F[c] += k * un * u[c];
    }
    if (W->models & ORC_WIND_DRYDEN) {
        uint32_t r[4];
        wind_words(W, i, t, 0u, r);
        const double rad0 = sqrt(-2.0 * log(1.0 - unit24(r[0])));
        const double rad1 = sqrt(-2.0 * log(1.0 - unit24(r[2])));
        const double xi[3] = {rad0 * cos(2.0 * M_PI * unit24(r[1])), rad0 * sin(2.0 * M_PI * unit24(r[1])),
                              rad1 * cos(2.0 * M_PI * unit24(r[3]))};
        double h = p[2] / 0.3048;
        h = h < 10.0 ? 10.0 : (h > 1000.0 ? 1000.0 : h);
        const double Lu = h / pow(0.177 + 8.23e-4 * h, 1.2) * 0.3048, Lw = h * 0.3048;
        const double au = exp(-dt * W->dryden_airspeed / Lu), aw = exp(-dt * W->dryden_airspeed / Lw);
        const double a[3] = {au, au, aw};
        double x[3];
        for (int c = 0; c < 3; ++c) {
            x[c] = a[c] * ws[c * N] + W->dryden_sigma * sqrt(1.0 - a[c] * a[c]) * xi[c];
            ws[c * N] = x[c];
        }
        const double xn = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
        for (int c = 0; c < 3; ++c) F[c] += k * xn * x[c];
    }
    if (W->models & ORC_WIND_GUST) {
        long ng = lround(W->gust_duration / dt);
        if (ng < 1) ng = 1;
        if (ws[3 * N] < 0.0) {
            uint32_t g[4];
            wind_words(W, i, t, 1u, g);
            if (unit24(g[0]) < (double)(float)W->gust_prob) {
                ws[3 * N] = 0.0;
                ws[4 * N] = 2.0 * M_PI * unit24(g[1]);
            }
        }
        if (ws[3 * N] >= 0.0) {
            const double env = sin(M_PI * ws[3 * N] / (double)ng);
            F[0] += W->gust_amp * cos(ws[4 * N]) * env;
            F[1] += W->gust_amp * sin(ws[4 * N]) * env;
            ws[3 * N] += 1.0;
            if (ws[3 * N] >= (double)ng) ws[3 * N] = -1.0;
        }
    }
    if (W->models & ORC_WIND_SINUSOIDAL) {
        const double tau = (double)t * dt, wt = W->sin_omega * tau;
        F[0] += W->sin_amp * sin(wt);
        F[1] += W->sin_amp * cos(wt);
        F[2] += W->sin_amp * 0.3 * sin(2.0 * wt);
    }
}

/* The KIN row the sensors deliver under domain randomisation (Table
 * "Recommended domain-randomization ranges", sensors, and the sticky
 * per-episode observation bias recommended beside it): the drone's constant
 * bias, then per-step Gaussian
 * noise added to position, roll/pitch/yaw, velocity and body rates (the
 * quaternion and rotor-speed rows stay exact), twelve normals from Philox
 * streams 2-4 of (drone, global step) by Box-Muller; then the sensor latency:
 * the noisy row enters a ring of ORC_DR_OBS_HIST slots indexed by the global
 * step and the row delivered is the one entered min(obs_delay, entered - 1)
 * steps earlier.  Readings: noise and latency act on the returned
 * observation only (the controllers fly on the simulator's state); the ring
 * is advanced every step whether or not observations are requested. */
static void sensor_row(const orc_dr *dr, int64_t t, int32_t i, int N, orc_state *s, double row[20])
{
    if (dr->obs_bias) {
        static const int rows[12] = {0, 1, 2, 10, 11, 12, 7, 8, 9, 13, 14, 15};
        for (int b = 0; b < 12; ++b) row[rows[b]] += dr->obs_bias[(size_t)b * N + i];
    }
    if (dr->noise_p > 0.0 || dr->noise_v > 0.0 || dr->noise_rpy > 0.0 || dr->noise_w > 0.0) {
        const orc_wind key = {.seed = dr->seed};
        double xi[12];
        for (uint32_t st = 0; st < 3; ++st) {
            uint32_t r[4];
            wind_words(&key, dr->drone_id ? dr->drone_id[i] : i, t, 2u + st, r);
            const double rad0 = sqrt(-2.0 * log(1.0 - unit24(r[0])));
            const double rad1 = sqrt(-2.0 * log(1.0 - unit24(r[2])));
            xi[4 * st + 0] = rad0 * cos(2.0 * M_PI * unit24(r[1]));
            xi[4 * st + 1] = rad0 * sin(2.0 * M_PI * unit24(r[1]));
            xi[4 * st + 2] = rad1 * cos(2.0 * M_PI * unit24(r[3]));
            xi[4 * st + 3] = rad1 * sin(2.0 * M_PI * unit24(r[3]));
        }
        for (int c = 0; c < 3; ++c) {
            row[c] += dr->noise_p * xi[c];
            row[7 + c] += dr->noise_rpy * xi[6 + c];
            row[10 + c] += dr->noise_v * xi[3 + c];
            row[13 + c] += dr->noise_w * xi[9 + c];
        }
    }
    if (dr->obs_delay) {
        const int64_t slot = t % ORC_DR_OBS_HIST;
        for (int c = 0; c < 20; ++c) s->obs_hist[((size_t)slot * 20 + c) * N + i] = row[c];
        int32_t cnt = s->obs_count[i] + 1;
        if (cnt > ORC_DR_OBS_HIST) cnt = ORC_DR_OBS_HIST;
        s->obs_count[i] = cnt;
        int32_t d = dr->obs_delay[i];
        if (d > cnt - 1) d = cnt - 1;
        const int64_t from = (slot - d + ORC_DR_OBS_HIST) % ORC_DR_OBS_HIST;
        for (int c = 0; c < 20; ++c) row[c] = s->obs_hist[((size_t)from * 20 + c) * N + i];
    }
}

/* One drone's physical parameter block under domain randomisation (Table
 * "Recommended domain-randomization ranges"): the nominal block with mass,
 * inertia (one factor for the three principal moments), arm length, kf, km,
 * drag (one factor for c_xy and c_z), C_gnd, C1 and g multiplied by the
 * drone's factors, and MAX_RPM = factor x the nominal MAX_RPM.  Readings:
 * the controllers keep the nominal constants (the randomised dynamics are
 * what they must be robust to); h_clip stays nominal; the downwash on a drone
 * uses that drone's C1. */
static void dr_params(const orc_params *P, const orc_derived *D, const orc_dr *dr, int N, int i,
                      orc_params *Pi, double *max_rpm_i)
{
    *Pi = *P;
    *max_rpm_i = D->max_rpm;
    if (!dr) return;
    const double *s = dr->scale;
    Pi->m *= s[ORC_DR_M * N + i];
    Pi->Ixx *= s[ORC_DR_J * N + i];
    Pi->Iyy *= s[ORC_DR_J * N + i];
    Pi->Izz *= s[ORC_DR_J * N + i];
    Pi->L *= s[ORC_DR_L * N + i];
    Pi->kf *= s[ORC_DR_KF * N + i];
    Pi->km *= s[ORC_DR_KM * N + i];
    Pi->c_xy *= s[ORC_DR_DRAG * N + i];
    Pi->c_z *= s[ORC_DR_DRAG * N + i];
    Pi->C_gnd *= s[ORC_DR_GND * N + i];
    Pi->C1 *= s[ORC_DR_C1 * N + i];
    Pi->g *= s[ORC_DR_G * N + i];
    *max_rpm_i = D->max_rpm * s[ORC_DR_MAXRPM * N + i];
}

/* Semi-implicit Euler step shared by orc_step (dr = NULL) and orc_step_dr.
 *
 * Actuator chain under domain randomisation, per step and drone:
 *   1. action latency: the step's action rows enter a ring of ORC_DR_HIST
 *      slots indexed by the global step; the rows used are those issued
 *      min(delay, issued - 1) steps earlier, issued counting the actions
 *      entered since the ring was cleared (so a fresh episode uses its first
 *      action until the delay has elapsed);
 *   2. command: the RPM action, or the controller's output at controller
 *      steps (held in rpm_cmd in between);
 *   3. per-motor bias b_k and clip: c_k = clip(b_k cmd_k, 0, MAX_RPM_i);
 *   4. first-order motor lag with time constant tau (zero-order hold of c
 *      over the step, exact discretisation): n <- n + (1 - e^{-dt/tau})(c - n),
 *      or n = c for tau = 0;
 *   5. the drone's own parameter block for Eq. 1-7.
 * With all factors 1, tau = 0 and no delay the step equals orc_step. */
static int step_impl(const orc_params *P, double dt, uint32_t aero_mask, int act_type, int ctrl_decim,
                     int n_envs, const int32_t *env_offsets, int n_drones, orc_state *s,
                     const double *action, int action_per_step, double *obs, int n_obs_slots,
                     int n_steps, int64_t step0, int n_threads, const orc_dr *dr, const orc_wind *wind)
{
    if (n_drones < 0 || n_envs < 0 || n_steps < 0 || ctrl_decim < 1) return -1;
    if (env_offsets[0] != 0 || env_offsets[n_envs] != n_drones) return -1;
    if (aero_mask & ORC_AERO_SURROGATE) return -1; /* handled by the surrogate oracle */
    if (act_type < ORC_ACT_RPM || act_type > ORC_ACT_DSL || (act_type == ORC_ACT_DSL && !s->ctl)) return -1;
    if (dr && (!dr->scale || (act_type != ORC_ACT_RPM && !s->rpm_cmd) ||
               (dr->delay && (!s->act_hist || !s->act_count))))
        return -1;
    if (wind && (wind->models & (ORC_WIND_DRYDEN | ORC_WIND_GUST)) && !s->wind) return -1;
    if (dr && dr->obs_delay && (!s->obs_hist || !s->obs_count)) return -1;
    orc_derived D;
    orc_derive(P, &D);
    const int N = n_drones;
    const int rows = orc_action_rows(act_type);
    double *p_pre = (double *)malloc(sizeof(double) * 3 * (size_t)(N > 0 ? N : 1));
    if (!p_pre) return -2;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
    for (int k = 0; k < n_steps; ++k) {
        memcpy(p_pre, s->p, sizeof(double) * 3 * (size_t)N);
        const double *act = action + (action_per_step ? (size_t)k * rows * N : 0);
        const int do_pid = (act_type != ORC_ACT_RPM) && (((step0 + k) % ctrl_decim) == 0);
        const int64_t slot = (step0 + k) % ORC_DR_HIST;
#pragma omp parallel for schedule(dynamic, 16)
        for (int e = 0; e < n_envs; ++e) {
            for (int i = env_offsets[e]; i < env_offsets[e + 1]; ++i) {
                orc_params Pi;
                double max_rpm_i;
                dr_params(P, &D, dr, N, i, &Pi, &max_rpm_i);
                double p[3], q[4], v[3], w[3], n[4], a[7];
                for (int c = 0; c < 3; ++c) {
                    p[c] = s->p[c * N + i];
                    v[c] = s->v[c * N + i];
                    w[c] = s->w[c * N + i];
                }
                for (int c = 0; c < 4; ++c) q[c] = s->q[c * N + i];
                for (int c = 0; c < rows; ++c) a[c] = act[c * N + i];
                if (dr && dr->delay) {
                    for (int c = 0; c < rows; ++c) s->act_hist[((size_t)slot * rows + c) * N + i] = a[c];
                    int32_t cnt = s->act_count[i] + 1;
                    if (cnt > ORC_DR_HIST) cnt = ORC_DR_HIST;
                    s->act_count[i] = cnt;
                    int32_t d = dr->delay[i];
                    if (d > cnt - 1) d = cnt - 1;
                    const int64_t from = (slot - d + ORC_DR_HIST) % ORC_DR_HIST;
                    for (int c = 0; c < rows; ++c) a[c] = s->act_hist[((size_t)from * rows + c) * N + i];
                }

                double cmd[4];
                if (act_type == ORC_ACT_RPM) {
                    for (int c = 0; c < 4; ++c) cmd[c] = a[c];
                } else if (do_pid) {
                    controller(P, &D, act_type, dt * ctrl_decim, N, i, a, p, q, v, w, s, cmd);
                    if (dr)
                        for (int c = 0; c < 4; ++c) s->rpm_cmd[c * N + i] = cmd[c];
                } else {
                    for (int c = 0; c < 4; ++c) cmd[c] = dr ? s->rpm_cmd[c * N + i] : s->rpm[c * N + i];
                }
                if (!dr) {
                    for (int c = 0; c < 4; ++c)
                        n[c] = (act_type == ORC_ACT_RPM) ? clampd(cmd[c], 0.0, D.max_rpm) : cmd[c];
                } else {
                    const double tau_m = dr->tau_mot ? dr->tau_mot[i] : 0.0;
                    const double alpha = tau_m > 0.0 ? 1.0 - exp(-dt / tau_m) : 1.0;
                    for (int c = 0; c < 4; ++c) {
                        const double cc = clampd(dr->scale[(ORC_DR_BIAS + c) * N + i] * cmd[c], 0.0, max_rpm_i);
                        const double n0 = s->rpm[c * N + i];
                        n[c] = tau_m > 0.0 ? n0 + alpha * (cc - n0) : cc;
                    }
                }
                for (int c = 0; c < 4; ++c) s->rpm[c * N + i] = n[c];

                double F[4], T, tau[3], R[9];
                orc_motor(&Pi, n, F, &T, tau);
                orc_quat_to_rot(q, R);
                double Fw[3] = {R[2] * T, R[5] * T, R[8] * T - Pi.m * Pi.g};
                if (aero_mask & ORC_AERO_GND) Fw[2] += orc_ground_effect(&Pi, &D, n, p[2], q);
                if (aero_mask & ORC_AERO_DRAG) {
                    double Fd[3];
                    orc_drag(&Pi, n, q, v, Fd);
                    for (int c = 0; c < 3; ++c) Fw[c] += Fd[c];
                }
                if (aero_mask & ORC_AERO_DW) {
                    const double pi_[3] = {p_pre[0 * N + i], p_pre[1 * N + i], p_pre[2 * N + i]};
                    for (int j = env_offsets[e]; j < env_offsets[e + 1]; ++j) {
                        if (j == i) continue;
                        const double pj[3] = {p_pre[0 * N + j], p_pre[1 * N + j], p_pre[2 * N + j]};
                        Fw[2] += orc_downwash_pair(&Pi, pi_, pj);
                    }
                }
                if (wind && wind->models) {
                    double Fwind[3];
                    wind_force(wind, dt, step0 + k, wind->drone_id ? wind->drone_id[i] : i, i, p, v,
                               s->wind ? s->wind + i : NULL, N, Fwind);
                    for (int c = 0; c < 3; ++c) Fw[c] += Fwind[c];
                }
                orc_integrate(&Pi, dt, Fw, tau, p, q, v, w);
                for (int c = 0; c < 3; ++c) {
                    s->p[c * N + i] = p[c];
                    s->v[c * N + i] = v[c];
                    s->w[c * N + i] = w[c];
                }
                for (int c = 0; c < 4; ++c) s->q[c * N + i] = q[c];

                const int sensors = dr && (dr->obs_delay || dr->obs_bias || dr->noise_p > 0.0 || dr->noise_v > 0.0 ||
                                            dr->noise_rpy > 0.0 || dr->noise_w > 0.0);
                if ((obs && n_obs_slots > 0) || sensors) {
                    double rpy[3];
                    orc_euler_zyx(q, rpy);
                    double row[20] = {p[0], p[1], p[2], q[0], q[1], q[2], q[3],
                                      rpy[0], rpy[1], rpy[2], v[0], v[1], v[2],
                                      w[0], w[1], w[2], n[0], n[1], n[2], n[3]};
                    if (sensors) sensor_row(dr, step0 + k, i, N, s, row);
                    if (obs && n_obs_slots > 0) {
                        double *o = obs + (size_t)(k % n_obs_slots) * 20 * N;
                        for (int c = 0; c < 20; ++c) o[(size_t)c * N + i] = row[c];
                    }
                }
            }
        }
    }
    free(p_pre);
    return 0;
}

/* One call advances every drone n_steps times.  Per step (all drones use the
 * pre-step positions of the others for the downwash, i.e. synchronously):
 *   rotor speeds (RPM action clipped to [0, MAX_RPM], or the PID every
 *   ctrl_decim steps with phase (step0 + k) mod ctrl_decim = 0, held between),
 *   motor model, F_w = R (0,0,T) - m g z_hat, optional ground effect, drag and
 *   downwash (each env's drones in ascending index), Newton-Euler, exp map,
 *   optional KIN observation [p, q, roll/pitch/yaw, v, omega, n] to slot
 *   k mod n_obs_slots.  Layouts: action [n_act][4][N] with n_act = n_steps
 *   when action_per_step else 1; obs [slot][20][N]. */
int orc_step(const orc_params *P, double dt, uint32_t aero_mask, int act_type, int ctrl_decim,
             int n_envs, const int32_t *env_offsets, int n_drones, orc_state *s,
             const double *action, int action_per_step, double *obs, int n_obs_slots,
             int n_steps, int64_t step0, int n_threads)
{
    return step_impl(P, dt, aero_mask, act_type, ctrl_decim, n_envs, env_offsets, n_drones, s, action,
                     action_per_step, obs, n_obs_slots, n_steps, step0, n_threads, NULL, NULL);
}

int orc_step_dr(const orc_params *P, double dt, uint32_t aero_mask, int act_type, int ctrl_decim,
                int n_envs, const int32_t *env_offsets, int n_drones, orc_state *s,
                const double *action, int action_per_step, double *obs, int n_obs_slots,
                int n_steps, int64_t step0, int n_threads, const orc_dr *dr)
{
    if (!dr) return -1;
    return step_impl(P, dt, aero_mask, act_type, ctrl_decim, n_envs, env_offsets, n_drones, s, action,
                     action_per_step, obs, n_obs_slots, n_steps, step0, n_threads, dr, NULL);
}

int orc_step_disturbed(const orc_params *P, double dt, uint32_t aero_mask, int act_type, int ctrl_decim,
                       int n_envs, const int32_t *env_offsets, int n_drones, orc_state *s,
                       const double *action, int action_per_step, double *obs, int n_obs_slots,
                       int n_steps, int64_t step0, int n_threads, const orc_dr *dr, const orc_wind *wind)
{
    return step_impl(P, dt, aero_mask, act_type, ctrl_decim, n_envs, env_offsets, n_drones, s, action,
                     action_per_step, obs, n_obs_slots, n_steps, step0, n_threads, dr, wind);
}

/* ------------------------------------------------------------------------ */
/* Classic Runge-Kutta variant of the step.                                  */
/* ------------------------------------------------------------------------ */

/* Time derivative of one drone's rigid-body state x = (p, v, q, w) with the
 * rotor thrust T and body torque tau held over the step (zero-order hold of
 * the rotor speeds n): p' = v, v' = F_w / m, q' = q (x) [0, w] / 2,
 * w' = J^-1 (tau - w x J w), F_w = R (0,0,T) - m g z_hat plus the selected
 * aerodynamic terms at this state.  p_all holds the same stage's positions
 * of every drone (for the downwash of Eq. (6)).  Reading: R is taken from
 * the normalised stage quaternion. */
static void rk_deriv(const orc_params *P, const orc_derived *D, uint32_t mask, int N, int i, int e0,
                     int e1, const double *p_all, const double x[13], const double n[4], double T,
                     const double tau[3], double k[13])
{
    const double *p = x, *v = x + 3, *qr = x + 6, *w = x + 10;
    const double nq = sqrt(qr[0] * qr[0] + qr[1] * qr[1] + qr[2] * qr[2] + qr[3] * qr[3]);
    const double q[4] = {qr[0] / nq, qr[1] / nq, qr[2] / nq, qr[3] / nq};
    double R[9];
    orc_quat_to_rot(q, R);
    double Fw[3] = {R[2] * T, R[5] * T, R[8] * T - P->m * P->g};
    if (mask & ORC_AERO_GND) Fw[2] += orc_ground_effect(P, D, n, p[2], q);
    if (mask & ORC_AERO_DRAG) {
        double Fd[3];
        orc_drag(P, n, q, v, Fd);
        for (int c = 0; c < 3; ++c) Fw[c] += Fd[c];
    }
    if (mask & ORC_AERO_DW) {
        for (int j = e0; j < e1; ++j) {
            if (j == i) continue;
            const double pj[3] = {p_all[0 * N + j], p_all[1 * N + j], p_all[2 * N + j]};
            Fw[2] += orc_downwash_pair(P, p, pj);
        }
    }
    for (int c = 0; c < 3; ++c) {
        k[c] = v[c];
        k[3 + c] = Fw[c] / P->m;
    }
    const double wq[4] = {0.0, w[0], w[1], w[2]};
    double qd[4];
    orc_quat_mul(qr, wq, qd);
    for (int c = 0; c < 4; ++c) k[6 + c] = 0.5 * qd[c];
    const double J[3] = {P->Ixx, P->Iyy, P->Izz};
    const double Jw[3] = {J[0] * w[0], J[1] * w[1], J[2] * w[2]};
    const double cr[3] = {w[1] * Jw[2] - w[2] * Jw[1], w[2] * Jw[0] - w[0] * Jw[2],
                          w[0] * Jw[1] - w[1] * Jw[0]};
    for (int c = 0; c < 3; ++c) k[10 + c] = (tau[c] - cr[c]) / J[c];
}

/* orc_step with the classic fourth-order Runge-Kutta integrator (the MuJoCo
 * modes' integrator, Table "Physics modes") in place of the semi-implicit
 * Euler step: rotor speeds, controllers and observations as in orc_step; per
 * step x_{k+1} = x + dt/6 (k1 + 2 k2 + 2 k3 + k4) with stages at x,
 * x + dt/2 k1, x + dt/2 k2, x + dt k3 evaluated synchronously for all drones
 * (the downwash of each stage uses every drone's stage position); the
 * quaternion is renormalised after the step. */
int orc_step_rk4(const orc_params *P, double dt, uint32_t aero_mask, int act_type, int ctrl_decim,
                 int n_envs, const int32_t *env_offsets, int n_drones, orc_state *s,
                 const double *action, int action_per_step, double *obs, int n_obs_slots,
                 int n_steps, int64_t step0, int n_threads)
{
    if (n_drones < 0 || n_envs < 0 || n_steps < 0 || ctrl_decim < 1) return -1;
    if (env_offsets[0] != 0 || env_offsets[n_envs] != n_drones) return -1;
    if (aero_mask & ORC_AERO_SURROGATE) return -1;
    if (act_type < ORC_ACT_RPM || act_type > ORC_ACT_DSL || (act_type == ORC_ACT_DSL && !s->ctl)) return -1;
    orc_derived D;
    orc_derive(P, &D);
    const int N = n_drones;
    const size_t n1 = (size_t)(N > 0 ? N : 1);
    double *X0 = (double *)malloc(sizeof(double) * 13 * n1);   /* state at the step start */
    double *Xs = (double *)malloc(sizeof(double) * 13 * n1);   /* current stage state */
    double *Ks = (double *)malloc(sizeof(double) * 13 * n1);   /* sum k1 + 2k2 + 2k3 + k4 */
    double *Kc = (double *)malloc(sizeof(double) * 13 * n1);   /* current stage derivative */
    double *ps = (double *)malloc(sizeof(double) * 3 * n1);    /* stage positions [3][N] */
    double *nn = (double *)malloc(sizeof(double) * 4 * n1);
    double *TT = (double *)malloc(sizeof(double) * 4 * n1);    /* T, tau per drone */
    if (!X0 || !Xs || !Ks || !Kc || !ps || !nn || !TT) {
        free(X0); free(Xs); free(Ks); free(Kc); free(ps); free(nn); free(TT);
        return -2;
    }
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
    static const double stage_w[4] = {1.0, 2.0, 2.0, 1.0};
    for (int k = 0; k < n_steps; ++k) {
        const int rows = orc_action_rows(act_type);
        const double *act = action + (action_per_step ? (size_t)k * rows * N : 0);
        const int do_pid = (act_type != ORC_ACT_RPM) && (((step0 + k) % ctrl_decim) == 0);
        /* rotor speeds, motor model; x0 */
#pragma omp parallel for schedule(static)
        for (int i = 0; i < N; ++i) {
            double p[3], q[4], v[3], w[3], n[4];
            for (int c = 0; c < 3; ++c) {
                p[c] = s->p[c * N + i];
                v[c] = s->v[c * N + i];
                w[c] = s->w[c * N + i];
            }
            for (int c = 0; c < 4; ++c) q[c] = s->q[c * N + i];
            if (act_type == ORC_ACT_RPM) {
                for (int c = 0; c < 4; ++c) n[c] = clampd(act[c * N + i], 0.0, D.max_rpm);
            } else if (do_pid) {
                double cmd[7];
                for (int c = 0; c < rows; ++c) cmd[c] = act[c * N + i];
                controller(P, &D, act_type, dt * ctrl_decim, N, i, cmd, p, q, v, w, s, n);
            } else {
                for (int c = 0; c < 4; ++c) n[c] = s->rpm[c * N + i];
            }
            for (int c = 0; c < 4; ++c) {
                s->rpm[c * N + i] = n[c];
                nn[(size_t)i * 4 + c] = n[c];
            }
            double F[4], T, tau[3];
            orc_motor(P, n, F, &T, tau);
            TT[(size_t)i * 4 + 0] = T;
            for (int c = 0; c < 3; ++c) TT[(size_t)i * 4 + 1 + c] = tau[c];
            double *x = X0 + (size_t)i * 13;
            for (int c = 0; c < 3; ++c) {
                x[c] = p[c];
                x[3 + c] = v[c];
                x[10 + c] = w[c];
            }
            for (int c = 0; c < 4; ++c) x[6 + c] = q[c];
            for (int c = 0; c < 13; ++c) {
                Xs[(size_t)i * 13 + c] = x[c];
                Ks[(size_t)i * 13 + c] = 0.0;
            }
        }
        for (int st = 0; st < 4; ++st) {
            for (int i = 0; i < N; ++i)
                for (int c = 0; c < 3; ++c) ps[c * N + i] = Xs[(size_t)i * 13 + c];
#pragma omp parallel for schedule(dynamic, 16)
            for (int e = 0; e < n_envs; ++e)
                for (int i = env_offsets[e]; i < env_offsets[e + 1]; ++i)
                    rk_deriv(P, &D, aero_mask, N, i, env_offsets[e], env_offsets[e + 1], ps,
                             Xs + (size_t)i * 13, nn + (size_t)i * 4, TT[(size_t)i * 4],
                             TT + (size_t)i * 4 + 1, Kc + (size_t)i * 13);
            const double h = (st < 2) ? 0.5 * dt : dt;
#pragma omp parallel for schedule(static)
            for (int i = 0; i < N; ++i)
                for (int c = 0; c < 13; ++c) {
                    Ks[(size_t)i * 13 + c] += stage_w[st] * Kc[(size_t)i * 13 + c];
                    if (st < 3) Xs[(size_t)i * 13 + c] = X0[(size_t)i * 13 + c] + h * Kc[(size_t)i * 13 + c];
                }
        }
#pragma omp parallel for schedule(static)
        for (int i = 0; i < N; ++i) {
            double x[13];
            for (int c = 0; c < 13; ++c) x[c] = X0[(size_t)i * 13 + c] + dt / 6.0 * Ks[(size_t)i * 13 + c];
            const double nq = sqrt(x[6] * x[6] + x[7] * x[7] + x[8] * x[8] + x[9] * x[9]);
            for (int c = 0; c < 4; ++c) x[6 + c] /= nq;
            for (int c = 0; c < 3; ++c) {
                s->p[c * N + i] = x[c];
                s->v[c * N + i] = x[3 + c];
                s->w[c * N + i] = x[10 + c];
            }
            for (int c = 0; c < 4; ++c) s->q[c * N + i] = x[6 + c];
            if (obs && n_obs_slots > 0) {
                double *o = obs + (size_t)(k % n_obs_slots) * 20 * N;
                double rpy[3];
                orc_euler_zyx(x + 6, rpy);
                const double *n = nn + (size_t)i * 4;
                const double row[20] = {x[0], x[1], x[2], x[6], x[7], x[8], x[9],
                                        rpy[0], rpy[1], rpy[2], x[3], x[4], x[5],
                                        x[10], x[11], x[12], n[0], n[1], n[2], n[3]};
                for (int c = 0; c < 20; ++c) o[(size_t)c * N + i] = row[c];
            }
        }
    }
    free(X0); free(Xs); free(Ks); free(Kc); free(ps); free(nn); free(TT);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Surrogate support: neighbours, features, residual targets, MLP, Adam.     */
/* ------------------------------------------------------------------------ */

/* k nearest same-environment neighbours by horizontal distance, ascending,
 * ties to the lower index, padded with -1.  Reading: the metric is the
 * lateral one because the only pairwise term, the downwash of Eq. (6),
 * varies with the lateral offset on the scale of beta (centimetres) and with
 * the vertical one on the scale of metres, so the neighbours that matter are
 * the laterally closest; this also puts a drone's column partner in the same
 * input slot for every sample.  The squared distance that decides the order
 * is formed in binary32 exactly as the GPU forms it (dx*dx + dy*dy, each
 * operation rounded), so both sides take the same integer decision. */
typedef struct { float d2; int32_t j; } orc_cand;

static int cand_cmp(const void *a, const void *b)
{
    const orc_cand *x = (const orc_cand *)a, *y = (const orc_cand *)b;
    if (x->d2 < y->d2) return -1;
    if (x->d2 > y->d2) return 1;
    return (x->j < y->j) ? -1 : (x->j > y->j);
}

int orc_knn(int n_envs, const int32_t *env_offsets, int n_drones, const double *p, int k,
            int32_t *nbr)
{
    const int N = n_drones;
    int maxm = 0;
    for (int e = 0; e < n_envs; ++e) {
        const int m = env_offsets[e + 1] - env_offsets[e];
        if (m > maxm) maxm = m;
    }
    int rc = 0;
#pragma omp parallel
    {
        orc_cand *c = (orc_cand *)malloc(sizeof(orc_cand) * (size_t)(maxm > 0 ? maxm : 1));
        if (!c) {
#pragma omp atomic write
            rc = -2;
        }
#pragma omp for schedule(dynamic, 16)
        for (int e = 0; e < n_envs; ++e) {
            if (!c) continue;
            for (int i = env_offsets[e]; i < env_offsets[e + 1]; ++i) {
                int nc = 0;
                const float xi = (float)p[0 * N + i], yi = (float)p[1 * N + i];
                for (int j = env_offsets[e]; j < env_offsets[e + 1]; ++j) {
                    if (j == i) continue;
                    volatile float dx = (float)p[0 * N + j] - xi;
                    volatile float dy = (float)p[1 * N + j] - yi;
                    volatile float a = dx * dx;
                    volatile float b = dy * dy;
                    volatile float d2 = a + b;
                    c[nc].d2 = d2;
                    c[nc].j = j;
                    ++nc;
                }
                qsort(c, (size_t)nc, sizeof *c, cand_cmp);
                for (int t = 0; t < k; ++t) nbr[(size_t)i * k + t] = (t < nc) ? c[t].j : -1;
            }
        }
        free(c);
    }
    return rc;
}

/* Surrogate inputs of drone i from pre-step positions / velocities and this
 * step's rotor speeds n (layout as in orc_features). */
static void features_one(const orc_derived *D, int N, int i, const double *p_pre,
                         const double *v_pre, const double q[4], const double n[4],
                         const int32_t *nbr, int k, double *x)
{
    double R[9];
    orc_quat_to_rot(q, R);
    for (int f = 0; f < 64; ++f) x[f] = 0.0;
    const double v[3] = {v_pre[0 * N + i], v_pre[1 * N + i], v_pre[2 * N + i]};
    for (int a = 0; a < 3; ++a) x[a] = R[0 * 3 + a] * v[0] + R[1 * 3 + a] * v[1] + R[2 * 3 + a] * v[2];
    for (int a = 0; a < 3; ++a) x[3 + a] = R[2 * 3 + a];
    for (int c = 0; c < 4; ++c) x[6 + c] = n[c] / D->hover_rpm;
    for (int t = 0; t < k; ++t) {
        const int j = nbr[t];
        if (j < 0) continue;
        for (int c = 0; c < 3; ++c) {
            x[10 + 6 * t + c] = p_pre[c * N + j] - p_pre[c * N + i];
            x[10 + 6 * t + 3 + c] = v_pre[c * N + j] - v_pre[c * N + i];
        }
    }
    const double z = p_pre[2 * N + i];
    const double g = D->h_clip / (z > D->h_clip ? z : D->h_clip);
    x[10 + 6 * k] = z;
    x[11 + 6 * k] = g * g;
}

/* Surrogate inputs of one drone (raw, before any scaling), n_feat = 64:
 *   [0..2]  v_body = R^T v
 *   [3..5]  world up axis in the body frame, R^T z_hat
 *   [6..9]  n_i / HOVER_RPM
 *   [10..57] for each of the k = 8 nearest neighbours: p_j - p_i, v_j - v_i
 *            (world frame), zeros for a missing neighbour
 *   [58]    p_z
 *   [59]    ground proximity (h_clip / max(p_z, h_clip))^2, in (0, 1]
 *   [60..]  zero padding.
 * Rotor speeds are the state's rpm. */
int orc_features(const orc_params *P, int n_envs, const int32_t *env_offsets, int n_drones,
                 const orc_state *s, const int32_t *nbr, int k, int n_feat, double *X)
{
    (void)n_envs;
    (void)env_offsets;
    if (n_feat != 64 || 10 + 6 * k + 1 > n_feat) return -1;
    orc_derived D;
    orc_derive(P, &D);
    const int N = n_drones;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < N; ++i) {
        double q[4], n[4];
        for (int c = 0; c < 4; ++c) {
            q[c] = s->q[c * N + i];
            n[c] = s->rpm[c * N + i];
        }
        features_one(&D, N, i, s->p, s->v, q, n, nbr + (size_t)i * k, k, X + (size_t)i * n_feat);
    }
    return 0;
}

/* Residual the surrogate learns: the aerodynamic wrench of Eq. (4)-(6) that
 * the selected effects add to the rotor wrench, in the body frame:
 * Y[i] = (R^T F_aero_w, tau_aero_body).  With the centre-of-mass readings of
 * Eq. (4)-(6) the aerodynamic torque is identically zero. */
int orc_aero_residual(const orc_params *P, uint32_t aero_mask, int n_envs,
                      const int32_t *env_offsets, int n_drones, const orc_state *s,
                      const double *rpm, double *Y)
{
    orc_derived D;
    orc_derive(P, &D);
    const int N = n_drones;
#pragma omp parallel for schedule(dynamic, 16)
    for (int e = 0; e < n_envs; ++e) {
        for (int i = env_offsets[e]; i < env_offsets[e + 1]; ++i) {
            double p[3], q[4], v[3], n[4], R[9];
            for (int c = 0; c < 3; ++c) {
                p[c] = s->p[c * N + i];
                v[c] = s->v[c * N + i];
            }
            for (int c = 0; c < 4; ++c) {
                q[c] = s->q[c * N + i];
                n[c] = rpm[c * N + i];
            }
            double Fa[3] = {0.0, 0.0, 0.0};
            if (aero_mask & ORC_AERO_GND) Fa[2] += orc_ground_effect(P, &D, n, p[2], q);
            if (aero_mask & ORC_AERO_DRAG) {
                double Fd[3];
                orc_drag(P, n, q, v, Fd);
                for (int c = 0; c < 3; ++c) Fa[c] += Fd[c];
            }
            if (aero_mask & ORC_AERO_DW) {
                for (int j = env_offsets[e]; j < env_offsets[e + 1]; ++j) {
                    if (j == i) continue;
                    const double pj[3] = {s->p[0 * N + j], s->p[1 * N + j], s->p[2 * N + j]};
                    Fa[2] += orc_downwash_pair(P, p, pj);
                }
            }
            orc_quat_to_rot(q, R);
            double *y = Y + (size_t)i * 6;
            for (int a = 0; a < 3; ++a) y[a] = R[0 * 3 + a] * Fa[0] + R[1 * 3 + a] * Fa[1] + R[2 * 3 + a] * Fa[2];
            y[3] = y[4] = y[5] = 0.0;
        }
    }
    return 0;
}

/* Round to the nearest bfloat16 value (8 significant bits), ties to even. */
double orc_bf16_round(double x)
{
    if (x == 0.0 || !isfinite(x)) return x;
    int e;
    const double m = frexp(x, &e);
    return ldexp(nearbyint(ldexp(m, 8)), e - 8);
}

static double silu(double z) { return z / (1.0 + exp(-z)); }

static double silu_grad(double z)
{
    const double sg = 1.0 / (1.0 + exp(-z));
    return sg * (1.0 + z * (1.0 - sg));
}

/* Multilayer perceptron y = W_L h_{L-1} + b_L, h_l = SiLU(W_l h_{l-1} + b_l),
 * h_0 = x.  W[l] is [dims[l+1]][dims[l]] row-major.  acts receives, per layer,
 * the pre-activation z_l [B][dims[l+1]] followed by the output h_l
 * [B][dims[l+1]] (h = z for the last layer).  With bf16_acts the input and
 * every hidden output are rounded to bfloat16, the precision the in-step
 * network stores them in; sums stay in double. */
int orc_mlp_forward(int n_layers, const int32_t *dims, const double *const *W,
                    const double *const *b, int B, const double *X, double *Y, double *acts,
                    int bf16_acts)
{
    size_t off = 0;
    const double *hin = X;
    double *xr = NULL;
    if (bf16_acts) {
        xr = (double *)malloc(sizeof(double) * (size_t)B * dims[0]);
        if (!xr) return -2;
        for (size_t t = 0; t < (size_t)B * dims[0]; ++t) xr[t] = orc_bf16_round(X[t]);
        hin = xr;
    }
    for (int l = 0; l < n_layers; ++l) {
        const int din = dims[l], dout = dims[l + 1];
        double *z = acts + off;
        double *h = acts + off + (size_t)B * dout;
        off += 2 * (size_t)B * dout;
#pragma omp parallel for schedule(static)
        for (int r = 0; r < B; ++r) {
            for (int o = 0; o < dout; ++o) {
                double sacc = b[l][o];
                for (int c = 0; c < din; ++c) sacc += W[l][(size_t)o * din + c] * hin[(size_t)r * din + c];
                z[(size_t)r * dout + o] = sacc;
                double hv = (l < n_layers - 1) ? silu(sacc) : sacc;
                if (bf16_acts && l < n_layers - 1) hv = orc_bf16_round(hv);
                h[(size_t)r * dout + o] = hv;
            }
        }
        hin = h;
    }
    memcpy(Y, hin, sizeof(double) * (size_t)B * dims[n_layers]);
    free(xr);
    return 0;
}

/* Reverse-mode gradient of the network above for upstream gradient dY
 * [B][dims[L]]: dW[l] = sum_r g_l[r] h_{l-1}[r]^T, db[l] = sum_r g_l[r],
 * g_{l-1} = (W_l^T g_l) * SiLU'(z_{l-1}); dX = W_0^T g_0 (may be NULL).
 * X must be the input exactly as the forward pass used it. */
int orc_mlp_backward(int n_layers, const int32_t *dims, const double *const *W,
                     const double *const *b, int B, const double *X, const double *acts,
                     const double *dY, double *const *dW, double *const *db, double *dX)
{
    (void)b;
    size_t *offs = (size_t *)malloc(sizeof(size_t) * (size_t)n_layers);
    int maxd = 0;
    for (int l = 0; l <= n_layers; ++l)
        if (dims[l] > maxd) maxd = dims[l];
    double *g = (double *)malloc(sizeof(double) * (size_t)B * maxd);
    double *gn = (double *)malloc(sizeof(double) * (size_t)B * maxd);
    if (!offs || !g || !gn) {
        free(offs);
        free(g);
        free(gn);
        return -2;
    }
    size_t off = 0;
    for (int l = 0; l < n_layers; ++l) {
        offs[l] = off;
        off += 2 * (size_t)B * dims[l + 1];
    }
    memcpy(g, dY, sizeof(double) * (size_t)B * dims[n_layers]);
    for (int l = n_layers - 1; l >= 0; --l) {
        const int din = dims[l], dout = dims[l + 1];
        const double *hin = (l == 0) ? X : acts + offs[l - 1] + (size_t)B * dims[l];
#pragma omp parallel for schedule(static)
        for (int o = 0; o < dout; ++o) {
            double sb = 0.0;
            for (int r = 0; r < B; ++r) sb += g[(size_t)r * dout + o];
            db[l][o] = sb;
            for (int c = 0; c < din; ++c) {
                double sw = 0.0;
                for (int r = 0; r < B; ++r) sw += g[(size_t)r * dout + o] * hin[(size_t)r * din + c];
                dW[l][(size_t)o * din + c] = sw;
            }
        }
        if (l == 0 && !dX) break;
#pragma omp parallel for schedule(static)
        for (int r = 0; r < B; ++r) {
            for (int c = 0; c < din; ++c) {
                double sacc = 0.0;
                for (int o = 0; o < dout; ++o) sacc += W[l][(size_t)o * din + c] * g[(size_t)r * dout + o];
                if (l > 0) {
                    const double zp = acts[offs[l - 1] + (size_t)r * din + c];
                    gn[(size_t)r * din + c] = sacc * silu_grad(zp);
                } else {
                    dX[(size_t)r * din + c] = sacc;
                }
            }
        }
        if (l > 0) {
            double *t = g;
            g = gn;
            gn = t;
        }
    }
    free(offs);
    free(g);
    free(gn);
    return 0;
}

/* Adam (Kingma and Ba): m <- b1 m + (1-b1) g, v <- b2 v + (1-b2) g^2,
 * param -= lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps), t >= 1. */
void orc_adam(int n, double *param, const double *grad, double *m1, double *m2, double lr,
              double beta1, double beta2, double eps, int64_t t)
{
    const double bc1 = 1.0 - pow(beta1, (double)t), bc2 = 1.0 - pow(beta2, (double)t);
    for (int i = 0; i < n; ++i) {
        m1[i] = beta1 * m1[i] + (1.0 - beta1) * grad[i];
        m2[i] = beta2 * m2[i] + (1.0 - beta2) * grad[i] * grad[i];
        const double mh = m1[i] / bc1, vh = m2[i] / bc2;
        param[i] -= lr * mh / (sqrt(vh) + eps);
    }
}

/* ------------------------------------------------------------------------ */
/* Step with the learned residual in place of Eq. (4)-(6).                   */
/* ------------------------------------------------------------------------ */

/* Per drone and step: rotor speeds and motor model as in orc_step; the 8
 * nearest neighbours (binary32 decisions, see orc_knn) and the raw inputs;
 * fallback -> the plain Eq. (4)-(6) force when a neighbour is above by less
 * than dz_ood, or (each check optional) when the drone leaves the region the
 * network was trained on: a neighbour inside the cylinder |dz| < near_dz,
 * horizontal distance < near_r, or beyond |dz| > far_dz, a world velocity
 * component beyond ood_speed, a
 * neighbour's relative velocity component beyond ood_rel_speed, or a tilt
 * beyond ood_tilt (qx^2 + qy^2 > sin^2(ood_tilt / 2)).  Every fallback
 * decision is taken in binary32 on quantities the GPU forms exactly the same
 * way (differences of stored values; qx*qx + qy*qy with rounded operations);
 * otherwise inputs standardised x' = (x - mean) * inv_std, rounded to
 * bfloat16, the network (W already rounded to bfloat16 by the caller; hidden
 * outputs rounded to bfloat16, sums in double), y = y' * y_std + y_mean,
 * body-frame force y[0..2] rotated to the world frame and body torque
 * y[3..5] added.  aero_out [N][6] (nullable) receives the body-frame
 * residual used in the last step, fallback_out [N] whether it was plain. */
int orc_step_surrogate(const orc_params *P, double dt, int act_type, int ctrl_decim, int n_envs,
                       const int32_t *env_offsets, int n_drones, orc_state *s,
                       const double *action, int action_per_step, double *obs, int n_obs_slots,
                       int n_steps, int64_t step0, const orc_net *net, double *aero_out,
                       int32_t *fallback_out, int n_threads)
{
    if (n_drones < 0 || n_envs < 0 || n_steps < 0 || ctrl_decim < 1) return -1;
    if (env_offsets[0] != 0 || env_offsets[n_envs] != n_drones) return -1;
    orc_derived D;
    orc_derive(P, &D);
    const int N = n_drones;
    const int K = 8;
    const int32_t dims[5] = {64, 128, 128, 128, 6};
    double *p_pre = (double *)malloc(sizeof(double) * 3 * (size_t)(N > 0 ? N : 1));
    double *v_pre = (double *)malloc(sizeof(double) * 3 * (size_t)(N > 0 ? N : 1));
    int32_t *nbr = (int32_t *)malloc(sizeof(int32_t) * K * (size_t)(N > 0 ? N : 1));
    if (!p_pre || !v_pre || !nbr) {
        free(p_pre);
        free(v_pre);
        free(nbr);
        return -2;
    }
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
    int rc = 0;
    for (int k = 0; k < n_steps; ++k) {
        memcpy(p_pre, s->p, sizeof(double) * 3 * (size_t)N);
        memcpy(v_pre, s->v, sizeof(double) * 3 * (size_t)N);
        if (orc_knn(n_envs, env_offsets, N, p_pre, K, nbr) != 0) {
            rc = -2;
            break;
        }
        const int rows = orc_action_rows(act_type);
        const double *act = action + (action_per_step ? (size_t)k * rows * N : 0);
        const int do_pid = (act_type != ORC_ACT_RPM) && (((step0 + k) % ctrl_decim) == 0);
#pragma omp parallel for schedule(dynamic, 16)
        for (int e = 0; e < n_envs; ++e) {
            double acts[2 * (128 + 128 + 128 + 6)];
            for (int i = env_offsets[e]; i < env_offsets[e + 1]; ++i) {
                double p[3], q[4], v[3], w[3], n[4];
                for (int c = 0; c < 3; ++c) {
                    p[c] = s->p[c * N + i];
                    v[c] = s->v[c * N + i];
                    w[c] = s->w[c * N + i];
                }
                for (int c = 0; c < 4; ++c) q[c] = s->q[c * N + i];
                if (act_type == ORC_ACT_RPM) {
                    for (int c = 0; c < 4; ++c) n[c] = clampd(act[c * N + i], 0.0, D.max_rpm);
                } else if (do_pid) {
                    double cmd[7];
                    for (int c = 0; c < rows; ++c) cmd[c] = act[c * N + i];
                    controller(P, &D, act_type, dt * ctrl_decim, N, i, cmd, p, q, v, w, s, n);
                } else {
                    for (int c = 0; c < 4; ++c) n[c] = s->rpm[c * N + i];
                }
                for (int c = 0; c < 4; ++c) s->rpm[c * N + i] = n[c];

                double F[4], T, tau[3], R[9];
                orc_motor(P, n, F, &T, tau);
                orc_quat_to_rot(q, R);
                double Fw[3] = {R[2] * T, R[5] * T, R[8] * T - P->m * P->g};

                const int32_t *nb = nbr + (size_t)i * K;
                int ood = 0;
                const float vrel = (float)net->ood_rel_speed;
                const int near_on = net->near_dz > 0.0 && net->near_r > 0.0;
                const float near_r2 = (float)(net->near_r * net->near_r);
                for (int t = 0; t < K; ++t) {
                    if (nb[t] < 0) continue;
                    const float dz = (float)p_pre[2 * N + nb[t]] - (float)p_pre[2 * N + i];
                    if (dz > 0.0f && dz < (float)net->dz_ood) ood = 1;
                    /* the horizontal distance squared as the neighbour ranking forms it */
                    volatile float dx = (float)p_pre[0 * N + nb[t]] - (float)p_pre[0 * N + i];
                    volatile float dy = (float)p_pre[1 * N + nb[t]] - (float)p_pre[1 * N + i];
                    volatile float ax = dx * dx, ay = dy * dy;
                    volatile float d2 = ax + ay;
                    if (near_on && fabsf(dz) < (float)net->near_dz && d2 < near_r2) ood = 1;
                    if (net->far_dz > 0.0 && fabsf(dz) > (float)net->far_dz) ood = 1;
                    for (int c = 0; c < 3 && vrel > 0.0f; ++c) {
                        const float dv = (float)v_pre[c * N + nb[t]] - (float)v_pre[c * N + i];
                        if (fabsf(dv) > vrel) ood = 1;
                    }
                }
                if (net->ood_speed > 0.0)
                    for (int c = 0; c < 3; ++c)
                        if (fabsf((float)v[c]) > (float)net->ood_speed) ood = 1;
                if (net->ood_tilt > 0.0) {
                    const double sh = sin(0.5 * net->ood_tilt);
                    volatile float a = (float)q[1] * (float)q[1];
                    volatile float b = (float)q[2] * (float)q[2];
                    volatile float t2 = a + b;
                    if (t2 > (float)(sh * sh)) ood = 1;
                }
                double yb[6];
                if (ood) {
                    double Fa[3] = {0.0, 0.0, 0.0}, Fd[3];
                    Fa[2] += orc_ground_effect(P, &D, n, p[2], q);
                    orc_drag(P, n, q, v, Fd);
                    for (int c = 0; c < 3; ++c) Fa[c] += Fd[c];
                    const double pi_[3] = {p_pre[0 * N + i], p_pre[1 * N + i], p_pre[2 * N + i]};
                    for (int j = env_offsets[e]; j < env_offsets[e + 1]; ++j) {
                        if (j == i) continue;
                        const double pj[3] = {p_pre[0 * N + j], p_pre[1 * N + j], p_pre[2 * N + j]};
                        Fa[2] += orc_downwash_pair(P, pi_, pj);
                    }
                    for (int c = 0; c < 3; ++c) Fw[c] += Fa[c];
                    for (int a = 0; a < 3; ++a)
                        yb[a] = R[0 * 3 + a] * Fa[0] + R[1 * 3 + a] * Fa[1] + R[2 * 3 + a] * Fa[2];
                    yb[3] = yb[4] = yb[5] = 0.0;
                } else {
                    double x[64], y[6];
                    features_one(&D, N, i, p_pre, v_pre, q, n, nb, K, x);
                    for (int f = 0; f < 64; ++f) x[f] = (x[f] - net->norm[f]) * net->norm[64 + f];
                    orc_mlp_forward(4, dims, net->W, net->b, 1, x, y, acts, 1);
                    for (int o = 0; o < 6; ++o) yb[o] = y[o] * net->norm[134 + o] + net->norm[128 + o];
                    for (int a = 0; a < 3; ++a)
                        Fw[a] += R[a * 3 + 0] * yb[0] + R[a * 3 + 1] * yb[1] + R[a * 3 + 2] * yb[2];
                    for (int c = 0; c < 3; ++c) tau[c] += yb[3 + c];
                }
                if (aero_out)
                    for (int o = 0; o < 6; ++o) aero_out[(size_t)i * 6 + o] = yb[o];
                if (fallback_out) fallback_out[i] = ood;

                orc_integrate(P, dt, Fw, tau, p, q, v, w);
                for (int c = 0; c < 3; ++c) {
                    s->p[c * N + i] = p[c];
                    s->v[c * N + i] = v[c];
                    s->w[c * N + i] = w[c];
                }
                for (int c = 0; c < 4; ++c) s->q[c * N + i] = q[c];
                if (obs && n_obs_slots > 0) {
                    double *o = obs + (size_t)(k % n_obs_slots) * 20 * N;
                    double rpy[3];
                    orc_euler_zyx(q, rpy);
                    const double row[20] = {p[0], p[1], p[2], q[0], q[1], q[2], q[3],
                                            rpy[0], rpy[1], rpy[2], v[0], v[1], v[2],
                                            w[0], w[1], w[2], n[0], n[1], n[2], n[3]};
                    for (int c = 0; c < 20; ++c) o[(size_t)c * N + i] = row[c];
                }
            }
        }
    }
    free(p_pre);
    free(v_pre);
    free(nbr);
    return rc;
}
