"""Pins of the oracle's classic Runge-Kutta step (the integrator of the MuJoCo
physics modes, Table "Physics modes").

* Linear dynamics: with fixed attitude and rotor speeds the translational
  motion under blade drag (Eq. 5) is the affine ODE p' = v, v' = A v + b, for
  which one RK4 step is exactly the degree-4 Taylor polynomial of exp(h M)
  applied to the augmented state; K steps are its K-th power.
* Free fall is reproduced exactly (RK4 integrates cubics exactly), and a
  constant body rate about an axis where w x J w = 0 rotates the quaternion
  by the same degree-4 polynomial of the rate matrix, renormalised.
* With every aerodynamic term on (ground effect, drag, downwash between two
  drones) and torques that tumble the body, halving the step divides the
  error by about 16 (the semi-implicit Euler step: by about 2).
"""
import numpy as np
import pytest

import oracle as orc

H = 1.0 / 240.0


def _taylor4(M):
    I = np.eye(M.shape[0])
    out, term = I.copy(), I.copy()
    for k in range(1, 5):
        term = term @ M / k
        out = out + term
    return out


def _one(P, n_rot, p, v, q=(1, 0, 0, 0), w=(0, 0, 0)):
    s = orc.new_state(1)
    s["p"][:, 0], s["v"][:, 0], s["q"][:, 0], s["w"][:, 0] = p, v, q, w
    act = np.asarray(n_rot, dtype=np.float64).reshape(1, 4, 1)
    return s, act


def test_drag_motion_is_the_truncated_exponential():
    P = orc.cf2x()
    D = orc.derive(P)
    n = np.full(4, 0.93 * D.hover_rpm)
    K = 240
    s, act = _one(P, n, [0.1, 0.2, 1.5], [1.0, -0.5, 0.3])
    s_eu = {k: v.copy() for k, v in s.items()}
    orc.step(P, H, orc.AERO_DRAG, orc.ACT_RPM, 1, [0, 1], s, act, False, K, integrator="rk4")
    orc.step(P, H, orc.AERO_DRAG, orc.ACT_RPM, 1, [0, 1], s_eu, act, False, K)
    S = 4 * 2 * np.pi * n[0] / 60.0
    _, T, tau = orc.motor(P, n)
    np.testing.assert_allclose(tau, 0, atol=1e-18)
    M = np.zeros((7, 7))
    M[0:3, 3:6] = np.eye(3)
    M[3:6, 3:6] = -np.diag([P.c_xy, P.c_xy, P.c_z]) * S / P.m
    M[5, 6] = T / P.m - P.g
    y = np.linalg.matrix_power(_taylor4(H * M), K) @ np.array([0.1, 0.2, 1.5, 1.0, -0.5, 0.3, 1.0])
    np.testing.assert_allclose(s["p"][:, 0], y[0:3], rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(s["v"][:, 0], y[3:6], rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(s["q"][:, 0], [1, 0, 0, 0], atol=1e-15)
    np.testing.assert_allclose(s["w"][:, 0], 0, atol=1e-15)
    # the Euler step of the same problem is measurably different
    assert np.abs(s_eu["p"][:, 0] - y[0:3]).max() > 1e-5


@pytest.mark.parametrize("w", [(0.0, 0.0, 2.3), (0.9, -1.2, 0.0)])
def test_free_fall_and_constant_rate_rotation(w):
    P = orc.cf2x()
    q0 = np.array([0.8, 0.1, -0.3, 0.5])
    q0 /= np.linalg.norm(q0)
    p0, v0 = np.array([0.0, 0.5, 3.0]), np.array([0.4, -0.2, 1.0])
    K = 180
    s, act = _one(P, np.zeros(4), p0, v0, q0, w)
    orc.step(P, H, 7, orc.ACT_RPM, 1, [0, 1], s, act, False, K, integrator="rk4")
    t = K * H
    np.testing.assert_allclose(s["p"][:, 0], p0 + v0 * t - 0.5 * P.g * t * t * np.array([0, 0, 1]),
                               rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(s["w"][:, 0], w, atol=1e-15)
    # q' = q (x) [0, w] / 2 = Omega q with Omega the right-multiplication matrix
    a, b, c = np.asarray(w) / 2
    Om = np.array([[0, -a, -b, -c], [a, 0, c, -b], [b, -c, 0, a], [c, b, -a, 0]])
    step = _taylor4(H * Om)
    q = q0.copy()
    for _ in range(K):
        q = step @ q
        q /= np.linalg.norm(q)
    np.testing.assert_allclose(s["q"][:, 0], q, atol=1e-14)
    # and the polynomial is within its truncation error of the exact rotation
    th = np.linalg.norm(w) * t
    ax = np.asarray(w) / np.linalg.norm(w)
    exact = orc.quat_mul(q0, np.r_[np.cos(th / 2), np.sin(th / 2) * ax])
    np.testing.assert_allclose(q, exact, atol=1e-11)


def _pair_run(dt, steps, integrator):
    P = orc.cf2x()
    D = orc.derive(P)
    s = orc.new_state(2)
    s["p"][:, 0], s["p"][:, 1] = [0.0, 0.0, 0.5], [0.04, -0.03, 0.85]
    s["v"][:, 0], s["v"][:, 1] = [0.3, -0.2, 0.1], [-0.1, 0.2, 0.0]
    s["w"][:, 0], s["w"][:, 1] = [1.5, -2.0, 0.7], [-0.4, 0.9, -1.1]
    h = D.hover_rpm
    act = np.array([[h * 1.03, h * 1.01], [h * 0.97, h * 1.02],
                    [h * 1.01, h * 0.98], [h * 0.99, h * 0.99]]).reshape(1, 4, 2)
    orc.step(P, dt, 7, orc.ACT_RPM, 1, [0, 2], s, act, False, steps, integrator=integrator)
    return np.concatenate([s[k].ravel() for k in ("p", "q", "v", "w")])


def test_fourth_order_convergence_with_all_aero_terms():
    t_end = 0.25
    ref = _pair_run(t_end / 3840, 3840, "rk4")
    e = [np.abs(_pair_run(t_end / k, k, "rk4") - ref).max() for k in (60, 120, 240)]
    r = [e[0] / e[1], e[1] / e[2]]
    assert all(12.0 < x < 20.0 for x in r), (e, r)
    e_eu = [np.abs(_pair_run(t_end / k, k, "euler") - ref).max() for k in (60, 120)]
    assert 1.6 < e_eu[0] / e_eu[1] < 2.5, e_eu


def test_pid_hover_is_a_fixed_point_and_rk4_rejects_the_surrogate():
    P = orc.cf2x()
    s = orc.new_state(1)
    s["p"][:, 0] = [0.3, -0.2, 1.0]
    act = np.array([0.3, -0.2, 1.0, 0.0]).reshape(1, 4, 1)
    orc.step(P, H, orc.AERO_DRAG, orc.ACT_PID, 5, [0, 1], s, act, False, 480, integrator="rk4")
    np.testing.assert_allclose(s["p"][:, 0], [0.3, -0.2, 1.0], atol=1e-9)
    np.testing.assert_allclose(s["v"][:, 0], 0, atol=1e-9)
    with pytest.raises(ValueError):
        orc.step(P, H, orc.AERO_SURROGATE, orc.ACT_PID, 5, [0, 1], s, act, False, 1,
                 integrator="rk4")
