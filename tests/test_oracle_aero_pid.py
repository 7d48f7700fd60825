"""Pins of the oracle's aerodynamic terms (Eq. (4)-(6)) and cascaded PID:
equilibria, special cases, symmetry/invariance properties and brute force."""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle as orc

DT = 1.0 / 240.0


def _quat_from_rot(r):
    x, y, z, w = r.as_quat()
    return np.array([w, x, y, z])


# ---------------------------------------------------------------- ground effect

def test_hover_in_ground_effect_is_an_equilibrium():
    P = orc.cf2x()
    for h in (0.06, 0.1, 0.3):
        # the rotor speed at which thrust plus the Eq. (4) lift equals weight
        n = np.sqrt(P.m * P.g / (4 * P.kf * (1 + P.C_gnd * (P.r_p / (4 * h)) ** 2)))
        s = orc.new_state(1)
        s["p"][2, 0] = h
        act = np.full((1, 4, 1), n)
        orc.step(P, DT, orc.AERO_GND, orc.ACT_RPM, 1, [0, 1], s, act, False, 1)
        assert abs(s["v"][2, 0]) < 1e-14
        # and without the effect the same speed sinks
        s2 = orc.new_state(1)
        s2["p"][2, 0] = h
        orc.step(P, DT, 0, orc.ACT_RPM, 1, [0, 1], s2, act, False, 1)
        assert s2["v"][2, 0] < -1e-4


def test_ground_effect_clip_inverse_square_and_gate():
    P = orc.cf2x()
    D = orc.derive(P)
    n = [15000, 14000, 16000, 15500]
    f = lambda h, q=(1, 0, 0, 0): orc.ground_effect(P, n, h, q)
    assert f(0.2) / f(0.4) == pytest.approx(4.0, rel=1e-14)
    assert f(0.01) == f(D.h_clip) == f(-1.0) > 0
    # h_clip: one rotor at MAX_RPM gains MAX_THRUST/15 there (the reading)
    one = orc.ground_effect(P, [D.max_rpm, 0, 0, 0], D.h_clip, (1, 0, 0, 0))
    assert one == pytest.approx(D.max_thrust / 15, rel=1e-13)
    # gate: on while |roll|,|pitch| < pi/2; equivalently the body z axis points up
    rng = np.random.default_rng(20)
    for _ in range(200):
        r = Rotation.random(random_state=rng)
        q = _quat_from_rot(r)
        up = r.as_matrix()[2, 2]
        if abs(up) < 1e-6:
            continue
        assert (f(0.3, q) > 0) == (up > 0)
    assert f(0.3, _quat_from_rot(Rotation.from_euler("x", 179, degrees=True))) == 0.0
    assert f(0.3, _quat_from_rot(Rotation.from_euler("y", 91, degrees=True))) == 0.0
    assert f(0.3, _quat_from_rot(Rotation.from_euler("y", 89, degrees=True))) > 0.0


# ---------------------------------------------------------------- drag

def test_drag_acts_along_body_axes_with_its_coefficients():
    P = orc.cf2x()
    rng = np.random.default_rng(21)
    n = np.array([14000.0, 15000.0, 13000.0, 16000.0])
    S = np.sum(2 * np.pi * n / 60)
    for _ in range(20):
        r = Rotation.random(random_state=rng)
        q = _quat_from_rot(r)
        Rm = r.as_matrix()
        for axis, c in ((0, P.c_xy), (1, P.c_xy), (2, P.c_z)):
            vw = 0.7 * Rm[:, axis]  # velocity along a body axis, world frame
            np.testing.assert_allclose(orc.drag(P, n, q, vw), -c * S * vw, rtol=1e-12, atol=1e-20)


def test_drag_linear_in_velocity_and_rotor_speed_and_zero_when_stopped():
    P = orc.cf2x()
    q = _quat_from_rot(Rotation.from_euler("xyz", [0.3, -0.2, 1.0]))
    n = np.array([14000.0, 15000.0, 13000.0, 16000.0])
    v = np.array([0.4, -1.1, 0.3])
    F = orc.drag(P, n, q, v)
    np.testing.assert_allclose(orc.drag(P, n, q, 2.5 * v), 2.5 * F, rtol=1e-13)
    np.testing.assert_allclose(orc.drag(P, 2 * n, q, v), 2 * F, rtol=1e-13)
    assert np.all(orc.drag(P, [0, 0, 0, 0], q, v) == 0)


# ---------------------------------------------------------------- downwash

def test_downwash_pair_special_values():
    P = orc.cf2x()
    low = np.array([0.1, -0.2, 1.0])
    for dz in (0.8, 1.0, 1.7):
        up = low + [0, 0, dz]
        f0 = orc.downwash_pair(P, low, up)
        assert f0 < 0
        # the upper drone feels nothing from the lower one
        assert orc.downwash_pair(P, up, low) == 0.0
        beta = abs(P.C2 * dz + P.C3)
        side = up + [beta * np.cos(0.3), beta * np.sin(0.3), 0]
        # Gaussian profile in the lateral offset with width |beta|
        assert orc.downwash_pair(P, low, side) / f0 == pytest.approx(np.exp(-0.5), rel=1e-13)
        side2 = up + [2 * beta, 0, 0]
        assert orc.downwash_pair(P, low, side2) / f0 == pytest.approx(np.exp(-2.0), rel=1e-12)
    # inverse square in the vertical gap on the axis, scale C1 (r_p/4)^2
    a1 = orc.downwash_pair(P, low, low + [0, 0, 0.9])
    a2 = orc.downwash_pair(P, low, low + [0, 0, 1.8])
    assert a1 / a2 == pytest.approx(4.0, rel=1e-13)
    assert -a1 * 0.9 ** 2 == pytest.approx(P.C1 * (P.r_p / 4) ** 2, rel=1e-13)
    # cut-offs: same height, below, and lateral distance >= 10 m
    assert orc.downwash_pair(P, low, low + [0.05, 0, 0]) == 0.0
    assert orc.downwash_pair(P, low, low + [0, 0, -0.5]) == 0.0
    far = low + [0, 0, 100.0]
    assert orc.downwash_pair(P, low, far + [10.0, 0, 0]) == 0.0
    assert orc.downwash_pair(P, low, far + [9.99, 0, 0]) < 0.0


def _dw_forces(P, pos):
    """Per-drone downwash force of a single env through the batched oracle."""
    n = pos.shape[1]
    s = orc.new_state(n)
    s["p"][:] = pos
    Y = orc.aero_residual(P, orc.AERO_DW, [0, n], s, rpm=np.zeros((4, n)))
    return Y[:, 2]  # level drones: body z = world z


def test_downwash_env_sweep_equals_brute_force_sum():
    P = orc.cf2x()
    rng = np.random.default_rng(22)
    for m in (1, 2, 3, 4):
        pos = rng.uniform([-0.3, -0.3, 0.5], [0.3, 0.3, 2.0], size=(m, 3)).T.copy()
        got = _dw_forces(P, pos)
        for i in range(m):
            ref = 0.0
            for j in range(m):
                if j == i or not pos[2, j] > pos[2, i]:
                    continue
                dz = pos[2, j] - pos[2, i]
                dxy = np.hypot(pos[0, j] - pos[0, i], pos[1, j] - pos[1, i])
                beta = P.C2 * dz + P.C3
                ref -= P.C1 * (P.r_p / (4 * dz)) ** 2 * np.exp(-0.5 * (dxy / beta) ** 2)
            assert got[i] == pytest.approx(ref, rel=1e-12, abs=1e-300)


def test_downwash_invariances():
    P = orc.cf2x()
    rng = np.random.default_rng(23)
    pos = rng.uniform([-0.3, -0.3, 0.5], [0.3, 0.3, 2.0], size=(6, 3)).T.copy()
    f = _dw_forces(P, pos)
    assert np.count_nonzero(f) >= 3
    perm = rng.permutation(6)
    np.testing.assert_allclose(_dw_forces(P, pos[:, perm].copy()), f[perm], rtol=1e-12)
    shift = pos + np.array([[3.0], [-7.0], [0.25]])
    np.testing.assert_allclose(_dw_forces(P, shift), f, rtol=1e-9)
    th = 1.1
    Rz = np.array([[np.cos(th), -np.sin(th), 0], [np.sin(th), np.cos(th), 0], [0, 0, 1]])
    np.testing.assert_allclose(_dw_forces(P, Rz @ pos), f, rtol=1e-9)


def test_stacked_pair_lower_drone_thrust_balances_wake():
    # Fig. "downwash": under PID and the full aero mode the lower of two
    # stacked drones settles at a thrust equal to its weight plus the wake.
    P = orc.cf2x()
    D = orc.derive(P)
    s = orc.new_state(2)
    s["p"][:, 0] = [0.0, 0.0, 1.0]
    s["p"][:, 1] = [0.0, 0.0, 2.2]
    tgt = np.array([[0.0, 0.0], [0.0, 0.0], [1.0, 2.2], [0.0, 0.0]])[None]
    orc.step(P, DT, orc.AERO_GND | orc.AERO_DRAG | orc.AERO_DW, orc.ACT_PID, 5, [0, 2], s,
             tgt, False, 240 * 40)
    assert np.max(np.abs(s["v"])) < 2e-3
    T = P.kf * np.sum(s["rpm"] ** 2, axis=0)
    f_dw = -orc.downwash_pair(P, s["p"][:, 0], s["p"][:, 1])
    g_lo = orc.ground_effect(P, s["rpm"][:, 0], s["p"][2, 0], s["q"][:, 0])
    assert T[1] == pytest.approx(P.m * P.g, rel=2e-3)
    assert T[0] + g_lo == pytest.approx(P.m * P.g + f_dw, rel=2e-3)
    assert f_dw > 0.05 * P.m * P.g
    assert T[0] > 1.03 * T[1]
    assert D.hover_rpm < s["rpm"][0, 0] < D.max_rpm


# ---------------------------------------------------------------- PID

def test_pid_hover_fixed_point():
    P = orc.cf2x()
    D = orc.derive(P)
    for yaw in (0.0, 0.9):
        q = [np.cos(yaw / 2), 0, 0, np.sin(yaw / 2)]
        n, I = orc.pid(P, 5 * DT, [0.3, -0.2, 1.1], q, [0, 0, 0], [0, 0, 0],
                       [0.3, -0.2, 1.1, yaw], np.zeros(6))
        np.testing.assert_allclose(n, D.hover_rpm, rtol=1e-13)
        assert np.all(I == 0)


def test_pid_allocation_reproduces_its_demands():
    # Level, at rest, integrals zero: the demanded thrust is m (Kp e_z + Ki e_z dt_c + g)
    # and the yaw torque Kp e_psi + Ki e_psi dt_c; the rotor speeds must
    # realise exactly those through the motor model (allocation inverse).
    P = orc.cf2x()
    dt_c = 5 * DT
    ez, epsi = 0.3, 0.2
    n, I = orc.pid(P, dt_c, [0, 0, 1], [1, 0, 0, 0], [0, 0, 0], [0, 0, 0],
                   [0, 0, 1 + ez, epsi], np.zeros(6))
    _, T, tau = orc.motor(P, n)
    Iz = ez * dt_c
    assert T == pytest.approx(P.m * (P.pos_kp[2] * ez + P.pos_ki[2] * Iz + P.g), rel=1e-12)
    assert tau[2] == pytest.approx(P.att_kp[2] * epsi + P.att_ki[2] * epsi * dt_c, rel=1e-12)
    np.testing.assert_allclose(tau[:2], 0, atol=1e-18)
    np.testing.assert_allclose(I, [0, 0, Iz, 0, 0, epsi * dt_c], atol=1e-15)


def test_pid_saturates_and_clamps_integrals():
    P = orc.cf2x()
    D = orc.derive(P)
    I = np.zeros(6)
    for _ in range(500):
        n, I = orc.pid(P, 5 * DT, [0, 0, 0], [1, 0, 0, 0], [0, 0, 0], [0, 0, 0],
                       [50, -50, 60, 3.0], I)
        assert np.all(n >= 0) and np.all(n <= D.max_rpm * (1 + 1e-15))
    assert np.all(np.abs(I[:3]) <= P.pos_i_clamp) and np.all(np.abs(I[3:]) <= P.att_i_clamp)
    assert np.abs(I[:3]).max() == P.pos_i_clamp


def test_pid_reaches_waypoint():
    P = orc.cf2x()
    s = orc.new_state(1)
    s["p"][:, 0] = [0.5, -0.5, 0.5]
    s["q"][:, 0] = [np.cos(0.4), 0, 0, np.sin(0.4)]
    tgt = np.array([0.0, 0.0, 1.0, 0.0]).reshape(1, 4, 1)
    orc.step(P, DT, orc.AERO_GND | orc.AERO_DRAG, orc.ACT_PID, 5, [0, 1], s, tgt, False, 240 * 15)
    np.testing.assert_allclose(s["p"][:, 0], [0, 0, 1], atol=0.03)
    assert abs(orc.euler_zyx(s["q"][:, 0])[2]) < 0.02
