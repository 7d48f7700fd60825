"""Pins of the oracle's VEL, ATTITUDE and DSL-style PID controllers (Table
"Action types", Sec. "Control"): hover fixed points, exact steady states of
the closed loop, heading-frame velocity, and the closed-form motion of the
rate-limited DSL setpoint."""
import numpy as np
import pytest

import oracle as orc

DT = 1.0 / 240.0
DT_C = 5 * DT


def _yawq(psi):
    return np.array([np.cos(psi / 2), 0, 0, np.sin(psi / 2)])


def test_vel_and_attitude_hover_fixed_points():
    P = orc.cf2x()
    D = orc.derive(P)
    for psi in (0.0, 1.2):
        n, I = orc.vel_ctrl(P, DT_C, _yawq(psi), [0, 0, 0], [0, 0, 0], [0, 0, 0, 0], np.zeros(6))
        np.testing.assert_allclose(n, D.hover_rpm, rtol=1e-13)
        assert np.all(I == 0)
        n, I = orc.att_ctrl(P, DT_C, _yawq(psi), [0, 0, 0], [P.m * P.g, 0, 0, 0], np.zeros(6))
        np.testing.assert_allclose(n, D.hover_rpm, rtol=1e-13)


def _run(P, act_type, cmd, q0=(1, 0, 0, 0), steps=240 * 20, mask=0, ctl=None):
    s = orc.new_state(1)
    s["p"][:, 0] = [0, 0, 1]
    s["q"][:, 0] = q0
    if ctl is not None:
        s["ctl"][:, 0] = ctl
    act = np.asarray(cmd, dtype=np.float64).reshape(1, -1, 1)
    orc.step(P, DT, mask, act_type, 5, [0, 1], s, act, False, steps)
    return s


def test_vel_tracks_heading_frame_velocity_and_yaw_rate():
    P = orc.cf2x()
    # heading along +y: a forward command flies along world +y
    s = _run(P, orc.ACT_VEL, [0.5, 0.0, 0.2, 0.0], q0=_yawq(np.pi / 2))
    np.testing.assert_allclose(s["v"][:, 0], [0.0, 0.5, 0.2], atol=1e-4)
    s = _run(P, orc.ACT_VEL, [0.0, 0.0, 0.0, 0.7])
    assert s["w"][2, 0] == pytest.approx(0.7, abs=1e-6)
    np.testing.assert_allclose(s["v"][:, 0], 0.0, atol=1e-6)


def test_attitude_command_reaches_its_angles_and_rate():
    P = orc.cf2x()
    # roll and pitch are PD loops (zero Ki in Table "Default PIDControl gains"),
    # so constant targets are reached exactly
    s = _run(P, orc.ACT_ATTITUDE, [P.m * P.g, 0.1, -0.05, 0.0], steps=240 * 5)
    rpy = orc.euler_zyx(s["q"][:, 0])
    np.testing.assert_allclose(rpy[:2], [0.1, -0.05], atol=2e-4)
    s = _run(P, orc.ACT_ATTITUDE, [P.m * P.g, 0.0, 0.0, -0.4], steps=240 * 5)
    assert s["w"][2, 0] == pytest.approx(-0.4, abs=1e-6)


def test_dsl_setpoint_moves_at_the_rate_limits():
    P = orc.cf2x()
    p0 = np.array([0.0, 0.0, 1.0])
    sp = np.array([0.0, 0.0, 1.0, 0.0])
    I = np.zeros(6)
    wp = np.array([30.0, 40.0, 1.0, 2.5, 0, 0, 0])  # 50 m away, yaw 2.5 rad
    for k in range(1, 11):
        n, I, sp = orc.dsl_pid(P, DT_C, p0, [1, 0, 0, 0], [0, 0, 0], [0, 0, 0], wp, I, sp)
        dist = np.linalg.norm(sp[:3] - p0)
        assert dist == pytest.approx(k * P.dsl_max_speed * DT_C, rel=1e-12)
        np.testing.assert_allclose((sp[:3] - p0) / dist, [0.6, 0.8, 0.0], atol=1e-12)
        assert sp[3] == pytest.approx(k * P.dsl_max_yaw_rate * DT_C, rel=1e-12)
        assert np.all(np.abs(I[:3]) <= P.dsl_pos_i_clamp)
    # a waypoint inside one step is reached exactly
    sp2 = np.array([0.0, 0.0, 1.0, 0.0])
    _, _, sp2 = orc.dsl_pid(P, DT_C, p0, [1, 0, 0, 0], [0, 0, 0], [0, 0, 0],
                            [0.01, 0.0, 1.0, 0.05, 0, 0, 0], np.zeros(6), sp2)
    np.testing.assert_allclose(sp2, [0.01, 0.0, 1.0, 0.05], atol=1e-15)


def test_dsl_fixed_point_feed_forward_and_halved_clamps():
    P = orc.cf2x()
    D = orc.derive(P)
    p = [0.2, -0.3, 1.1]
    sp = np.array(p + [0.4])
    n, I, sp2 = orc.dsl_pid(P, DT_C, p, _yawq(0.4), [0, 0, 0], [0, 0, 0], p + [0.4, 0, 0, 0],
                            np.zeros(6), sp)
    np.testing.assert_allclose(n, D.hover_rpm, rtol=1e-13)
    # feed-forward vertical acceleration adds m * a_ff to the thrust
    n, _, _ = orc.dsl_pid(P, DT_C, p, _yawq(0.4), [0, 0, 0], [0, 0, 0], p + [0.4, 0, 0, 1.5],
                          np.zeros(6), sp.copy())
    _, T, tau = orc.motor(P, n)
    assert T == pytest.approx(P.m * (P.g + 1.5), rel=1e-12)
    np.testing.assert_allclose(tau, 0, atol=1e-15)
    assert P.dsl_pos_i_clamp == P.pos_i_clamp / 2 and P.dsl_att_i_clamp == P.att_i_clamp / 2
    I = np.zeros(6)
    sp = np.array([0.0, 0.0, 1.0, 0.0])
    for _ in range(400):
        _, I, sp = orc.dsl_pid(P, DT_C, [0, 0, 1], [1, 0, 0, 0], [0, 0, 0], [0, 0, 0],
                               [100, 0, 1, 3.0, 0, 0, 0], I, sp)
    assert np.abs(I[:3]).max() == P.dsl_pos_i_clamp


def test_dsl_closed_loop_reaches_waypoint():
    P = orc.cf2x()
    s = _run(P, orc.ACT_DSL, [1.5, -1.0, 1.4, 0.6, 0, 0, 0], mask=3, ctl=[0, 0, 1, 0],
             steps=240 * 20)
    np.testing.assert_allclose(s["p"][:, 0], [1.5, -1.0, 1.4], atol=0.02)
    np.testing.assert_allclose(s["ctl"][:, 0], [1.5, -1.0, 1.4, 0.6], atol=1e-12)
    assert orc.euler_zyx(s["q"][:, 0])[2] == pytest.approx(0.6, abs=0.01)
