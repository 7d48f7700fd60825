"""Pins of the oracle's wind models (Sec. "Wind and turbulence"): the
counter-based generator against its published known-answer vectors; the
Box-Muller normals against the normal law; the Dryden recursion's variance
growth sigma^2 (1 - alpha^{2k}) and lag covariance alpha^m, and the isotropy
of the MIL-F-8785C scales at 1000 ft; the gust envelope and the renewal
fraction of gusty steps; the sinusoid and the constant-wind drag in closed
form (terminal velocity = mean wind); COMBINED = sum of the models."""
import json
import math
import os

import numpy as np
import pytest
from scipy import stats

import oracle as orc

H = 1.0 / 240.0
HERE = os.path.dirname(os.path.abspath(__file__))


def test_philox_known_answers():
    kat = json.load(open(os.path.join(HERE, "golden", "philox4x32_10_kat.json")))
    for v in kat["vectors"]:
        got = orc.philox4x32([int(x, 16) for x in v["counter"]], [int(x, 16) for x in v["key"]])
        assert got == [int(x, 16) for x in v["output"]]


def _hover_run(n, wind, steps, z=1.0, step0=0):
    """n drones at hover speed, no aero: the only unbalanced force is the wind."""
    P = orc.cf2x()
    s = orc.wind_state(orc.new_state(n))
    s["p"][2] = z
    h = orc.derive(P).hover_rpm
    vs = []
    for k in range(steps):
        orc.step(P, H, 0, orc.ACT_RPM, 1, np.arange(n + 1), s, np.full((1, 4, n), h), False, 1,
                 step0=step0 + k, wind=wind)
        vs.append((s["v"].copy(), s["wind"].copy()))
    return P, s, vs


def test_dryden_normals_variance_growth_and_covariance():
    sigma, V = 0.7, 5.0
    W = orc.make_wind(orc.WIND_DRYDEN, cd_area=1e-9, dryden_sigma=sigma, dryden_airspeed=V, seed=11)
    n, K, m = 20000, 300, 100
    _, _, vs = _hover_run(n, W, K + m)
    h_ft = 10.0  # z = 1 m is below the 10 ft floor
    Lu = h_ft / (0.177 + 8.23e-4 * h_ft) ** 1.2 * 0.3048
    Lw = h_ft * 0.3048
    for c, L in ((0, Lu), (1, Lu), (2, Lw)):
        a = math.exp(-H * V / L)
        x1 = vs[0][1][c]
        xi = x1 / (sigma * math.sqrt(1 - a * a))
        assert abs(xi.mean()) < 0.03 and abs(xi.var() - 1) < 0.04
        assert stats.kstest(xi, "norm").pvalue > 1e-3
        xk, xkm = vs[K - 1][1][c], vs[K + m - 1][1][c]
        var = sigma ** 2 * (1 - a ** (2 * K))
        assert xk.var() == pytest.approx(var, rel=0.05)
        assert np.mean(xk * xkm) == pytest.approx(a ** m * var, rel=0.08)


def test_dryden_scales_are_isotropic_at_1000_ft():
    W = orc.make_wind(orc.WIND_DRYDEN, cd_area=1e-9, dryden_sigma=1.0, dryden_airspeed=30.0, seed=12)
    _, _, vs = _hover_run(4000, W, 200, z=1000 * 0.3048)
    x = vs[-1][1][:3]
    # L_u = L_w = 1000 ft there, so all three axes have one variance
    v = x.var(axis=1)
    assert v[0] == pytest.approx(v[2], rel=0.08) and v[1] == pytest.approx(v[2], rel=0.08)


def test_gust_envelope_and_renewal_fraction():
    P = orc.cf2x()
    amp, T = 0.02, 0.25  # 60 steps
    W = orc.make_wind(orc.WIND_GUST, gust_prob=1.0, gust_duration=T, gust_amp=amp, seed=13)
    _, s, vs = _hover_run(3, W, 130)
    ng = 60
    for i in range(3):
        v = np.zeros(3)
        for k in range(130):
            kk = k % ng
            start = k - kk
            hd = 2 * math.pi * (orc.philox4x32([i, start, 0, 1], [13, 0])[1] >> 8) / 2 ** 24
            F = amp * math.sin(math.pi * kk / ng) * np.array([math.cos(hd), math.sin(hd), 0.0])
            v = v + H * F / P.m
            np.testing.assert_allclose(vs[k][0][:, i], v, atol=1e-12)
    # trigger probability p: the gusty fraction of a renewal process
    p = 0.02
    W = orc.make_wind(orc.WIND_GUST, gust_prob=p, gust_duration=T, gust_amp=amp, seed=14)
    _, _, vs = _hover_run(2000, W, 600)
    active = np.mean([np.mean(x[1][3] >= 0) for x in vs[300:]])
    assert active == pytest.approx(ng / (ng + (1 - p) / p), abs=0.02)
    W = orc.make_wind(orc.WIND_GUST, gust_prob=0.0, gust_duration=T, gust_amp=amp, seed=14)
    _, s, _ = _hover_run(50, W, 100)
    assert np.all(s["wind"][3] == -1) and np.all(np.abs(s["v"]) < 1e-12)


def test_sinusoid_and_constant_wind_closed_forms():
    A, w = 0.01, 3.0
    W = orc.make_wind(orc.WIND_SINUSOIDAL, sin_amp=A, sin_omega=w)
    P, s, _ = _hover_run(1, W, 50, step0=1000)
    t = (1000 + np.arange(50)) * H
    F = A * np.stack([np.sin(w * t), np.cos(w * t), 0.3 * np.sin(2 * w * t)])
    np.testing.assert_allclose(s["v"][:, 0], H * F.sum(axis=1) / P.m, rtol=1e-10, atol=1e-14)
    # constant wind: first-step quadratic drag, then the drone drifts up to the wind speed
    vw = np.array([2.0, -1.0, 0.0])
    W = orc.make_wind(orc.WIND_CONSTANT, v_mean=tuple(vw), rho=1.2, cd_area=0.02)
    P, s, vs = _hover_run(1, W, 1)
    np.testing.assert_allclose(vs[0][0][:, 0], H * 0.5 * 1.2 * 0.02 * np.linalg.norm(vw) * vw / P.m, rtol=1e-12)
    # the relative air speed decays as u0 / (1 + k |u0| t), k = rho CdA / (2 m), along the wind
    P, s, vs = _hover_run(1, W, 240 * 60)
    u = vw - s["v"][:, 0]
    k = 0.5 * 1.2 * 0.02 / P.m
    u0 = np.linalg.norm(vw)
    assert np.linalg.norm(u) == pytest.approx(u0 / (1 + k * u0 * 60.0), rel=2e-3)
    np.testing.assert_allclose(u / np.linalg.norm(u), vw / u0, atol=1e-9)


def test_combined_is_the_sum_of_the_models():
    kw = dict(v_mean=(1.0, 0.5, 0.0), rho=1.2, cd_area=0.01, gust_prob=1.0, gust_duration=0.2, gust_amp=0.01,
              dryden_sigma=0.5, dryden_airspeed=3.0, sin_amp=0.005, sin_omega=2.0, seed=21)
    dv = {}
    for m in (1, 2, 4, 8, 15):
        P, s, _ = _hover_run(5, orc.make_wind(m, **kw), 1, step0=77)
        dv[m] = s["v"].copy()
    np.testing.assert_allclose(dv[15], dv[1] + dv[2] + dv[4] + dv[8], rtol=1e-12, atol=1e-18)
    for m in (1, 4, 8):
        assert np.all(np.linalg.norm(dv[m], axis=0) > 1e-9), m


def test_per_drone_mean_wind_equals_separate_runs():
    """Per-drone mean winds (the table's per-episode wind magnitude) give
    each drone exactly the trajectory of a run with that drone's mean wind
    for everyone; the quadratic drag still drives each one to its own
    terminal velocity, the local mean wind."""
    rng = np.random.default_rng(9)
    n = 5
    vm = rng.uniform(-1.0, 1.0, (3, n))
    vm[2] *= 0.2
    kw = dict(models=orc.WIND_CONSTANT | orc.WIND_DRYDEN, dryden_sigma=0.3, dryden_airspeed=1.0, seed=4)
    _, s_all, _ = _hover_run(n, orc.make_wind(**kw, v_mean_drone=vm), 30)
    for i in range(n):
        # drone i alone keeps its own counter word through drone_id
        _, s_i, _ = _hover_run(1, orc.make_wind(**kw, v_mean=tuple(vm[:, i]), drone_id=np.array([i])), 30)
        for k in ("p", "v", "q", "w", "wind"):
            np.testing.assert_array_equal(s_i[k][..., 0], s_all[k][..., i], err_msg=k)
    # from rest the air speed u = v_mean - v keeps its direction and decays as
    # u0 / (1 + k |u0| t / m), k = rho CdA / 2 (the ODE's solution; the
    # semi-implicit steps follow it to O(dt))
    P, s_long, _ = _hover_run(n, orc.make_wind(orc.WIND_CONSTANT, v_mean_drone=vm, cd_area=0.05), 2400)
    u = vm - s_long["v"]
    sp = np.linalg.norm(vm, axis=0)
    k = 0.5 * 1.225 * 0.05
    want = sp / (1 + k * sp * 2400 * H / P.m)
    np.testing.assert_allclose(np.linalg.norm(u, axis=0), want, rtol=5e-3)
    np.testing.assert_allclose(np.sum(u * vm, axis=0) / (np.linalg.norm(u, axis=0) * sp), 1.0, atol=1e-9)
