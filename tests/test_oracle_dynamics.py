"""Pins of the FP64 oracle's rigid-body dynamics against things other than
itself: printed constants, closed forms of the discrete map, library
rotation routines, conservation laws and equilibria."""
import json
import os

import numpy as np
import pytest
from scipy.linalg import expm
from scipy.spatial.transform import Rotation

import oracle as orc

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")
DT = 1.0 / 240.0


def _rand_quats(rng, n):
    q = rng.normal(size=(n, 4))
    return q / np.linalg.norm(q, axis=1, keepdims=True)


def _one_drone_state(p=(0, 0, 1), q=(1, 0, 0, 0), v=(0, 0, 0), w=(0, 0, 0)):
    s = orc.new_state(1)
    s["p"][:, 0], s["q"][:, 0], s["v"][:, 0], s["w"][:, 0] = p, q, v, w
    return s


def _run_rpm(P, s, n_rpm, steps, mask=0, dt=DT):
    act = np.tile(np.asarray(n_rpm, dtype=np.float64).reshape(1, 4, 1), (1, 1, 1))
    return orc.step(P, dt, mask, orc.ACT_RPM, 1, [0, 1], s, act, False, steps)


def test_constants_match_printed_tables():
    g = json.load(open(GOLDEN))
    P = orc.cf2x()
    for k, v in g["drone_cf2x"].items():
        if not k.startswith("_"):
            assert getattr(P, k) == v, k
    for k in ("C1", "C2", "C3"):
        assert getattr(P, k) == g["downwash"][k]
    for k, v in g["pid_gains"].items():
        if k.startswith("_"):
            continue
        got = getattr(P, k)
        got = list(got) if not isinstance(got, float) else got
        assert got == v, k


def test_rotation_matrix_matches_scipy():
    rng = np.random.default_rng(10)
    for q in _rand_quats(rng, 50):
        R = orc.quat_to_rot(q)
        Rs = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
        np.testing.assert_allclose(R, Rs, atol=1e-14)


def test_euler_zyx_matches_scipy():
    rng = np.random.default_rng(11)
    for q in _rand_quats(rng, 50):
        ypr = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_euler("ZYX")
        np.testing.assert_allclose(orc.euler_zyx(q), ypr[::-1], atol=1e-12)


def test_hover_rpm_gives_zero_acceleration():
    P = orc.cf2x()
    D = orc.derive(P)
    for yaw in (0.0, 0.7, -2.5):
        s = _one_drone_state(q=(np.cos(yaw / 2), 0, 0, np.sin(yaw / 2)))
        _run_rpm(P, s, [D.hover_rpm] * 4, 1000)
        assert np.max(np.abs(s["v"])) < 1e-12
        assert np.max(np.abs(s["w"])) == 0.0
        np.testing.assert_allclose(s["p"][:, 0], [0, 0, 1], atol=1e-10)


def test_max_rpm_gives_thrust_to_weight():
    P = orc.cf2x()
    D = orc.derive(P)
    _, T, _ = orc.motor(P, [D.max_rpm] * 4)
    assert T == pytest.approx(P.thrust2weight * P.m * P.g, rel=1e-14)
    # an RPM action above MAX_RPM is clipped to it
    s1, s2 = _one_drone_state(), _one_drone_state()
    _run_rpm(P, s1, [D.max_rpm] * 4, 3)
    _run_rpm(P, s2, [3 * D.max_rpm] * 4, 3)
    np.testing.assert_array_equal(s1["v"], s2["v"])


@pytest.mark.parametrize("mask", [0, orc.AERO_GND | orc.AERO_DRAG])
def test_free_fall_discrete_closed_form(mask):
    # n = 0: every aerodynamic term is proportional to n or n^2 and vanishes.
    P = orc.cf2x()
    rng = np.random.default_rng(12)
    p0, v0 = np.array([0.2, -0.1, 1.5]), np.array([0.3, -0.2, 0.5])
    q0 = _rand_quats(rng, 1)[0]
    s = _one_drone_state(p=p0, q=q0, v=v0)
    K = 240
    _run_rpm(P, s, [0, 0, 0, 0], K, mask=mask)
    g = np.array([0, 0, P.g])
    np.testing.assert_allclose(s["v"][:, 0], v0 - K * DT * g, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(s["p"][:, 0], p0 + K * DT * v0 - g * DT * DT * K * (K + 1) / 2,
                               rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(s["q"][:, 0], q0, atol=1e-15)


def test_pure_spin_closed_form():
    P = orc.cf2x()  # Ixx == Iyy
    w0 = 7.3
    q0 = np.array([np.cos(0.2), np.sin(0.2) * 0.6, 0.0, np.sin(0.2) * 0.8])
    s = _one_drone_state(q=q0, w=(0, 0, w0))
    for k in (1, 17, 240):
        s2 = {kk: vv.copy() for kk, vv in s.items()}
        _run_rpm(P, s2, [0, 0, 0, 0], k)
        assert s2["w"][2, 0] == w0 and s2["w"][0, 0] == 0.0 and s2["w"][1, 0] == 0.0
        a = 0.5 * k * w0 * DT
        expect = orc.quat_mul(q0, [np.cos(a), 0, 0, np.sin(a)])
        # compare as rotations (q and -q are the same attitude)
        r1 = Rotation.from_quat(np.r_[s2["q"][1:, 0], s2["q"][0, 0]])
        r2 = Rotation.from_quat(np.r_[expect[1:], expect[0]])
        assert (r1.inv() * r2).magnitude() < 1e-12


def test_exp_map_matches_matrix_exponential():
    # Isotropic inertia and no rotors: omega is constant over the step and
    # the attitude must advance by R <- R expm(dt [omega]x) (body-frame rate).
    P = orc.cf2x()
    P.Iyy = P.Ixx
    P.Izz = P.Ixx
    rng = np.random.default_rng(13)
    for q0 in _rand_quats(rng, 10):
        w = rng.normal(size=3) * 20
        _, q1, _, w1 = orc.integrate(P, DT, [0, 0, 0], [0, 0, 0], [0, 0, 0], q0, [0, 0, 0], w)
        np.testing.assert_allclose(w1, w, rtol=1e-15)
        W = np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])
        R_expect = orc.quat_to_rot(q0) @ expm(DT * W)
        np.testing.assert_allclose(orc.quat_to_rot(q1), R_expect, atol=1e-13)


def test_axisymmetric_torque_free_discrete_closed_form():
    # Ixx = Iyy = I: omega_z is constant; explicit Euler maps (wx, wy) by a
    # rotation of atan(kappa dt) scaled by sqrt(1 + (kappa dt)^2),
    # kappa = (Izz - I) wz / I.
    P = orc.cf2x()
    wz, wx0, wy0 = 10.0, 0.3, -0.2
    s = _one_drone_state(w=(wx0, wy0, wz))
    K = 240
    _run_rpm(P, s, [0, 0, 0, 0], K)
    kap = (P.Izz - P.Ixx) * wz / P.Ixx
    ang, sc = K * np.arctan(kap * DT), np.sqrt(1 + (kap * DT) ** 2) ** K
    ex = sc * (np.cos(ang) * wx0 - np.sin(ang) * wy0)
    ey = sc * (np.sin(ang) * wx0 + np.cos(ang) * wy0)
    np.testing.assert_allclose(s["w"][:, 0], [ex, ey, wz], rtol=1e-11)
    assert np.hypot(ex, ey) / np.hypot(wx0, wy0) == pytest.approx(1.065, abs=2e-3)


def _invariants(P, s):
    q, w = s["q"][:, 0], s["w"][:, 0]
    J = np.array([P.Ixx, P.Iyy, P.Izz])
    L = orc.quat_to_rot(q) @ (J * w)
    E = 0.5 * np.sum(J * w * w)
    return L, E


def test_torque_free_invariants_converge_first_order():
    # World angular momentum and kinetic energy are conserved by the exact
    # flow; the explicit scheme's drift over a fixed time must shrink ~dt.
    P = orc.cf2x()
    P.Iyy = 1.8e-5  # a generic (triaxial) body
    drifts = []
    for dt in (1 / 240, 1 / 480, 1 / 960):
        s = _one_drone_state(w=(3.0, -4.0, 5.0))
        L0, E0 = _invariants(P, s)
        _run_rpm(P, s, [0, 0, 0, 0], int(round(0.5 / dt)), dt=dt)
        L1, E1 = _invariants(P, s)
        drifts.append((np.linalg.norm(L1 - L0) / np.linalg.norm(L0), abs(E1 - E0) / E0))
    drifts = np.array(drifts)
    for c in range(2):
        r1, r2 = drifts[0, c] / drifts[1, c], drifts[1, c] / drifts[2, c]
        assert 1.6 < r1 < 2.4 and 1.6 < r2 < 2.4, drifts
    assert drifts[2, 0] < 0.05 and drifts[2, 1] < 0.05


def test_quaternion_stays_unit():
    P = orc.cf2x()
    D = orc.derive(P)
    rng = np.random.default_rng(14)
    n = 8
    s = orc.new_state(n)
    s["q"][:] = _rand_quats(rng, n).T
    s["w"][:] = rng.normal(size=(3, n)) * 5
    act = (D.hover_rpm * (1 + rng.uniform(-0.3, 0.3, size=(300, 4, n))))
    for k in range(300):
        orc.step(P, DT, 0, orc.ACT_RPM, 1, np.arange(n + 1), s, act[k:k + 1], False, 1)
        assert np.max(np.abs(np.linalg.norm(s["q"], axis=0) - 1)) < 1e-14


def test_motor_torques_from_lever_arms():
    # X configuration: rotors on the diagonals at distance L; the roll/pitch
    # torque is sum r_i x (0,0,F_i).  Motor positions implied by the printed
    # mixer: 0 (+,+), 1 (-,+), 2 (-,-), 3 (+,-) in units of L/sqrt(2).
    P = orc.cf2x()
    a = P.L / np.sqrt(2)
    r = a * np.array([[1, 1, 0], [-1, 1, 0], [-1, -1, 0], [1, -1, 0]], dtype=float)
    rng = np.random.default_rng(15)
    for _ in range(20):
        n = rng.uniform(0, 20000, 4)
        F, T, tau = orc.motor(P, n)
        np.testing.assert_allclose(F, P.kf * n * n, rtol=1e-15)
        lever = sum(np.cross(r[i], [0, 0, F[i]]) for i in range(4))
        np.testing.assert_allclose(tau[:2], lever[:2], rtol=1e-13, atol=1e-20)
        # reaction torques: equal speeds cancel, diagonal pairs co-rotate
        assert T == pytest.approx(F.sum(), rel=1e-15)
    _, _, tau = orc.motor(P, [12000] * 4)
    assert tau[2] == 0.0
    _, _, t0 = orc.motor(P, [12000, 0, 0, 0])
    _, _, t2 = orc.motor(P, [0, 0, 12000, 0])
    _, _, t1 = orc.motor(P, [0, 12000, 0, 0])
    assert t0[2] == t2[2] < 0 < t1[2] and abs(t0[2]) == pytest.approx(P.km * 12000 ** 2)
