"""Pins of the oracle's domain-randomised step (Table "Recommended
domain-randomization ranges"): unit factors reproduce the plain step; the
randomised mass, kf and g move the hover speed to its closed form; inertia,
arm length and km scale the first-step body rates as Eq. 2-3 say; each
aerodynamic factor scales its term's velocity increment; the motor lag
follows the exponential step response; bias and MAX_RPM clip; action latency
delays the applied action by the drone's delay, across launches."""
import numpy as np
import pytest

import oracle as orc

H = 1.0 / 240.0
NS = len(orc.DR_ROWS)
ROW = {k: i for i, k in enumerate(orc.DR_ROWS)}


def _ones(n):
    return {"scale": np.ones((NS, n)), "tau_mot": np.zeros(n), "delay": np.zeros(n, dtype=np.int32)}


def _state(n, z=1.0):
    s = orc.new_state(n)
    s["p"][2] = z
    return s


def test_unit_factors_reproduce_the_plain_step():
    rng = np.random.default_rng(40)
    P = orc.cf2x()
    D = orc.derive(P)
    m = np.array([1, 3, 8, 2])
    off = np.concatenate([[0], np.cumsum(m)])
    n = off[-1]
    base = _state(n)
    base["p"][:] = rng.uniform(-0.3, 0.3, (3, n)) + np.array([[0], [0], [1.0]])
    base["v"][:] = rng.normal(0, 0.3, (3, n))
    base["w"][:] = rng.normal(0, 0.5, (3, n))
    for act_type, act in ((orc.ACT_RPM, D.hover_rpm * rng.uniform(0.9, 1.1, (10, 4, n))),
                          (orc.ACT_PID, np.broadcast_to(np.r_[0.1, 0.2, 1.2, 0.3][None, :, None], (10, 4, n)).copy())):
        a = {k: v.copy() for k, v in base.items()}
        b = orc.dr_state({k: v.copy() for k, v in base.items()}, act_type)
        oa = orc.step(P, H, 7, act_type, 5, off, a, act, True, 10, n_obs_slots=10)
        ob = orc.step(P, H, 7, act_type, 5, off, b, act, True, 10, n_obs_slots=10, dr=_ones(n))
        np.testing.assert_allclose(ob, oa, rtol=1e-14, atol=1e-14)
        for k in ("p", "q", "v", "w", "rpm", "pid_int"):
            np.testing.assert_allclose(b[k], a[k], rtol=1e-14, atol=1e-14)


def test_randomised_hover_speed_is_a_fixed_point():
    P = orc.cf2x()
    dr = _ones(3)
    dr["scale"][ROW["m"]] = [1.15, 0.85, 1.0]
    dr["scale"][ROW["kf"]] = [0.9, 1.1, 1.0]
    dr["scale"][ROW["g"]] = [1.01, 0.99, 1.02]
    m, kf, g = P.m * dr["scale"][ROW["m"]], P.kf * dr["scale"][ROW["kf"]], P.g * dr["scale"][ROW["g"]]
    n_h = np.sqrt(m * g / (4 * kf))
    s = orc.dr_state(_state(3), orc.ACT_RPM)
    act = np.tile(n_h, (4, 1))[None]
    orc.step(P, H, 0, orc.ACT_RPM, 1, [0, 1, 2, 3], s, act, False, 240, dr=dr)
    np.testing.assert_allclose(s["p"][2], 1.0, atol=1e-10)
    np.testing.assert_allclose(s["v"], 0, atol=1e-10)
    # the nominal hover speed leaves the closed-form semi-implicit drift
    s = orc.dr_state(_state(3), orc.ACT_RPM)
    h = orc.derive(P).hover_rpm
    K = 24
    orc.step(P, H, 0, orc.ACT_RPM, 1, [0, 1, 2, 3], s, np.full((1, 4, 3), h), False, K, dr=dr)
    a_z = (4 * kf * h * h - m * g) / m
    np.testing.assert_allclose(s["v"][2], K * H * a_z, rtol=1e-10)
    np.testing.assert_allclose(s["p"][2] - 1.0, H * H * a_z * K * (K + 1) / 2, rtol=1e-9)


def test_inertia_arm_length_and_km_factors_scale_first_step_rates():
    P = orc.cf2x()
    h = orc.derive(P).hover_rpm
    n = np.array([1.04, 1.01, 0.97, 0.99]) * h
    dr = _ones(2)
    dr["scale"][ROW["J"]] = [1.2, 0.8]
    dr["scale"][ROW["L"]] = [1.02, 0.98]
    dr["scale"][ROW["km"]] = [0.85, 1.15]
    dr["scale"][ROW["kf"]] = [1.1, 0.9]
    s = orc.dr_state(_state(2), orc.ACT_RPM)
    orc.step(P, H, 0, orc.ACT_RPM, 1, [0, 1, 2], s, np.tile(n[:, None], (1, 2))[None], False, 1, dr=dr)
    for i in range(2):
        kf = P.kf * dr["scale"][ROW["kf"], i]
        km = P.km * dr["scale"][ROW["km"], i]
        l = P.L * dr["scale"][ROW["L"], i] / np.sqrt(2)
        J = np.array([P.Ixx, P.Iyy, P.Izz]) * dr["scale"][ROW["J"], i]
        F = kf * n * n
        tau = np.array([l * (F[0] + F[1] - F[2] - F[3]), l * (-F[0] + F[1] + F[2] - F[3]),
                        km * (-n[0] ** 2 + n[1] ** 2 - n[2] ** 2 + n[3] ** 2)])
        np.testing.assert_allclose(s["w"][:, i], H * tau / J, rtol=1e-12)


@pytest.mark.parametrize("term,mask,row", [("drag", orc.AERO_DRAG, "drag"),
                                           ("ground", orc.AERO_GND, "C_gnd"),
                                           ("downwash", orc.AERO_DW, "C1")])
def test_aero_factors_scale_their_terms(term, mask, row):
    P = orc.cf2x()
    h = orc.derive(P).hover_rpm
    s0 = _state(2, z=0.0)
    s0["p"][:, 0] = [0.0, 0.0, 0.2]
    s0["p"][:, 1] = [0.01, -0.005, 1.2]
    s0["v"][:, 0] = [0.8, -0.5, 0.3]
    s0["v"][:, 1] = [-0.4, 0.2, 0.1]
    act = np.full((1, 4, 2), 1.05 * h)
    dv = {}
    for f, msk in (("none", 0), (1.0, mask), (1.27, mask)):
        dr = _ones(2)
        dr["scale"][ROW[row]] = 1.0 if f == "none" else f
        s = orc.dr_state({k: v.copy() for k, v in s0.items()}, orc.ACT_RPM)
        orc.step(P, H, msk, orc.ACT_RPM, 1, [0, 2], s, act, False, 1, dr=dr)
        dv[f] = s["v"] - s0["v"]
    base = dv[1.0] - dv["none"]
    assert np.abs(base).max() > 1e-6
    np.testing.assert_allclose(dv[1.27] - dv["none"], 1.27 * base, rtol=1e-9, atol=1e-15)


def test_motor_lag_step_response_and_bias_clip():
    P = orc.cf2x()
    D = orc.derive(P)
    dr = _ones(2)
    dr["tau_mot"][:] = [0.02, 0.045]
    s = orc.dr_state(_state(2), orc.ACT_RPM)
    s["rpm"][:] = 9000.0
    c = 15000.0
    obs = orc.step(P, H, 0, orc.ACT_RPM, 1, [0, 1, 2], s, np.full((1, 4, 2), c), False, 30,
                   n_obs_slots=30, dr=dr)
    k = np.arange(1, 31)[:, None]
    expect = c + (9000.0 - c) * np.exp(-k * H / dr["tau_mot"][None, :])
    np.testing.assert_allclose(obs[:, 16, :], expect, rtol=1e-12)
    # bias then clip to the drone's MAX_RPM
    dr = _ones(1)
    dr["scale"][ROW["bias0"]:ROW["bias3"] + 1, 0] = [1.02, 0.97, 1.0, 1.05]
    dr["scale"][ROW["max_rpm"], 0] = 0.96
    for a, expect in ((30000.0, np.full(4, 0.96 * D.max_rpm)),
                      (10000.0, 10000.0 * np.array([1.02, 0.97, 1.0, 1.05]))):
        s = orc.dr_state(_state(1), orc.ACT_RPM)
        orc.step(P, H, 0, orc.ACT_RPM, 1, [0, 1], s, np.full((1, 4, 1), a), False, 1, dr=dr)
        np.testing.assert_allclose(s["rpm"][:, 0], expect, rtol=1e-15)


def test_action_latency_delays_actions_across_launches():
    P = orc.cf2x()
    n = 3
    dr = _ones(n)
    dr["delay"][:] = [0, 3, 7]
    K = 16
    act = (10000.0 + 100.0 * np.arange(K))[:, None, None] * np.ones((K, 4, n))
    s = orc.dr_state(_state(n), orc.ACT_RPM)
    obs = orc.step(P, H, 0, orc.ACT_RPM, 1, [0, 1, 2, 3], s, act, True, K, n_obs_slots=K, dr=dr)
    for i, d in enumerate(dr["delay"]):
        expect = act[np.maximum(np.arange(K) - d, 0), 0, i]
        np.testing.assert_array_equal(obs[:, 16, i], expect)
    # the same rollout in two launches of 5 and 11 steps
    s2 = orc.dr_state(_state(n), orc.ACT_RPM)
    o1 = orc.step(P, H, 0, orc.ACT_RPM, 1, [0, 1, 2, 3], s2, act[:5], True, 5, n_obs_slots=5, dr=dr)
    o2 = orc.step(P, H, 0, orc.ACT_RPM, 1, [0, 1, 2, 3], s2, act[5:], True, 11, step0=5, n_obs_slots=11, dr=dr)
    np.testing.assert_array_equal(np.concatenate([o1, o2]), obs)
    for k in ("p", "v", "rpm"):
        np.testing.assert_array_equal(s2[k], s[k])


def test_controllers_keep_nominal_constants():
    """The nominal PID with a saturated integral leaves the closed-form height
    offset of a drone whose mass is off by a factor s: the vertical loop
    balances m s g = m (Kp e + Ki I_max sgn(e) + g)."""
    P = orc.cf2x()
    for ms in (1.2, 0.8):
        dr = _ones(1)
        dr["scale"][ROW["m"]] = ms
        dr["delay"][:] = 6
        dr["tau_mot"][:] = 0.03
        s = orc.dr_state(_state(1), orc.ACT_PID)
        wp = np.array([0.0, 0.0, 1.4, 0.0]).reshape(1, 4, 1)
        orc.step(P, H, 0, orc.ACT_PID, 5, [0, 1], s, wp, False, 240 * 60, dr=dr)
        sg = np.sign(ms - 1)
        e = ((ms - 1) * P.g - P.pos_ki[2] * P.pos_i_clamp * sg) / P.pos_kp[2]
        assert s["p"][2, 0] == pytest.approx(1.4 - e, abs=1e-6)
        assert s["pid_int"][2, 0] == P.pos_i_clamp * sg
        assert s["act_count"][0] == orc.DR_HIST
    # one controller update sees neither the factors nor the lag
    rng = np.random.default_rng(41)
    s0 = _state(2)
    s0["v"][:] = rng.normal(0, 0.2, (3, 2))
    s0["w"][:] = rng.normal(0, 0.2, (3, 2))
    wp = np.array([[0.3, 0.1], [0.2, -0.4], [1.1, 0.8], [0.1, -0.2]])[None]
    outs = []
    for f in (1.0, 1.17):
        dr = _ones(2)
        dr["scale"][:ROW["g"] + 1] = f
        dr["tau_mot"][:] = 0.02 if f != 1.0 else 0.0
        s = orc.dr_state({k: v.copy() for k, v in s0.items()}, orc.ACT_PID)
        orc.step(P, H, 7, orc.ACT_PID, 5, [0, 2], s, wp, False, 1, dr=dr)
        outs.append((s["rpm_cmd"].copy(), s["pid_int"].copy()))
    np.testing.assert_array_equal(outs[0][0], outs[1][0])
    np.testing.assert_array_equal(outs[0][1], outs[1][1])


def test_sensor_noise_statistics_and_exact_rows():
    """Per-step Gaussian sensor noise with the table's standard deviations on
    position, velocity, roll/pitch/yaw and body rates; quaternion and rotor
    speed rows untouched; same seed, same draws."""
    from scipy import stats
    P = orc.cf2x()
    h = orc.derive(P).hover_rpm
    n = 20000
    sig = (0.01, 0.05, np.radians(1.0), 0.05)
    act = np.full((1, 4, n), h)
    clean_s = orc.dr_state(_state(n), orc.ACT_RPM)
    clean = orc.step(P, H, 0, orc.ACT_RPM, 1, np.arange(n + 1), clean_s, act, False, 1, n_obs_slots=1,
                     dr=_ones(n))[0]
    outs = []
    for seed in (5, 5, 6):
        dr = dict(_ones(n), noise=sig, seed=seed)
        s = orc.dr_state(_state(n), orc.ACT_RPM)
        outs.append(orc.step(P, H, 0, orc.ACT_RPM, 1, np.arange(n + 1), s, act, False, 1, n_obs_slots=1,
                             dr=dr)[0])
        for k in ("p", "v", "q", "w"):
            np.testing.assert_array_equal(s[k], clean_s[k])  # the state is not disturbed
    np.testing.assert_array_equal(outs[0], outs[1])
    assert np.abs(outs[0] - outs[2]).max() > 0
    d = outs[0] - clean
    np.testing.assert_array_equal(d[3:7], 0)
    np.testing.assert_array_equal(d[16:20], 0)
    for rows, sd in ((range(0, 3), sig[0]), (range(10, 13), sig[1]), (range(7, 10), sig[2]), (range(13, 16), sig[3])):
        for r in rows:
            z = d[r] / sd
            assert abs(z.mean()) < 0.03 and abs(z.std() - 1) < 0.03, r
            assert stats.kstest(z, "norm").pvalue > 1e-3
    assert abs(np.corrcoef(d[0], d[10])[0, 1]) < 0.03


def test_sensor_latency_delays_the_rows_across_launches():
    P = orc.cf2x()
    h = orc.derive(P).hover_rpm
    n, K = 3, 14
    rng = np.random.default_rng(44)
    act = h * (1 + rng.uniform(-0.05, 0.05, size=(K, 4, n)))
    ref_s = orc.dr_state(_state(n), orc.ACT_RPM)
    ref = orc.step(P, H, 0, orc.ACT_RPM, 1, [0, 1, 2, 3], ref_s, act, True, K, n_obs_slots=K, dr=_ones(n))
    dr = dict(_ones(n), obs_delay=np.array([0, 2, 5], dtype=np.int32))
    s = orc.dr_state(_state(n), orc.ACT_RPM)
    o1 = orc.step(P, H, 0, orc.ACT_RPM, 1, [0, 1, 2, 3], s, act[:4], True, 4, n_obs_slots=4, dr=dr)
    o2 = orc.step(P, H, 0, orc.ACT_RPM, 1, [0, 1, 2, 3], s, act[4:], True, K - 4, step0=4,
                  n_obs_slots=K - 4, dr=dr)
    got = np.concatenate([o1, o2])
    for i, dly in enumerate((0, 2, 5)):
        src = np.maximum(np.arange(K) - dly, 0)
        np.testing.assert_array_equal(got[:, :, i], ref[src][:, :, i])
    for k in ("p", "v", "q", "w", "rpm"):
        np.testing.assert_array_equal(s[k], ref_s[k])


def test_sensor_ring_advances_on_steps_without_observations():
    """The sensor latency ring is written on every step, whether or not the
    launch returns observations, so the row returned after K steps does not
    depend on which earlier steps were observed."""
    P = orc.cf2x()
    h = orc.derive(P).hover_rpm
    n, K = 3, 11
    rng = np.random.default_rng(45)
    act = h * (1 + rng.uniform(-0.05, 0.05, size=(K, 4, n)))
    dr = dict(_ones(n), obs_delay=np.array([1, 3, 7], dtype=np.int32), noise=(0.01, 0.05, 0.02, 0.05), seed=9)
    a = orc.dr_state(_state(n), orc.ACT_RPM)
    every = orc.step(P, H, 0, orc.ACT_RPM, 1, [0, 1, 2, 3], a, act, True, K, n_obs_slots=K, dr=dr)
    b = orc.dr_state(_state(n), orc.ACT_RPM)
    orc.step(P, H, 0, orc.ACT_RPM, 1, [0, 1, 2, 3], b, act[:6], True, 6, dr=dr)
    last = orc.step(P, H, 0, orc.ACT_RPM, 1, [0, 1, 2, 3], b, act[6:], True, K - 6, step0=6, n_obs_slots=1, dr=dr)
    np.testing.assert_array_equal(last[-1], every[-1])


def test_drone_id_keeps_the_draws_of_a_sub_batch():
    """A sub-batch run with each drone's Philox counter word set to its index
    in the whole batch reproduces that batch's rows exactly (sensor noise and
    wind draws are keyed by the counter word, environments are independent)."""
    P = orc.cf2x()
    h = orc.derive(P).hover_rpm
    off = np.array([0, 2, 5, 6], dtype=np.int32)
    n, K = 6, 9
    rng = np.random.default_rng(46)
    base = _state(n)
    base["p"][:2] += rng.uniform(-0.2, 0.2, (2, n))
    base["p"][2] += np.array([0.0, 0.1, 0.0, 0.25, 0.5, 0.0])
    act = h * (1 + rng.uniform(-0.05, 0.05, size=(K, 4, n)))
    wkw = dict(models=orc.WIND_DRYDEN | orc.WIND_GUST, dryden_sigma=0.5, dryden_airspeed=2.0,
               gust_prob=0.3, gust_amp=0.02, seed=12)

    def run(idx, o):
        dr = dict(_ones(n), noise=(0.01, 0.05, 0.02, 0.05), seed=3,
                  obs_delay=np.array([0, 1, 2, 3, 4, 5], dtype=np.int32))
        dr = {k: (v[..., idx] if isinstance(v, np.ndarray) else v) for k, v in dr.items()}
        dr["drone_id"] = idx
        s = orc.wind_state(orc.dr_state({k: v[..., idx].copy() for k, v in base.items()}, orc.ACT_RPM))
        obs = orc.step(P, H, 7, orc.ACT_RPM, 1, o, s, act[:, :, idx], True, K, n_obs_slots=K, dr=dr,
                       wind=orc.make_wind(**wkw, drone_id=idx))
        return s, obs

    full_s, full_o = run(np.arange(n, dtype=np.int32), off)
    idx = np.arange(2, 5, dtype=np.int32)
    sub_s, sub_o = run(idx, np.array([0, 3], dtype=np.int32))
    np.testing.assert_array_equal(sub_o, full_o[:, :, idx])
    for k in ("p", "v", "q", "w", "wind"):
        np.testing.assert_array_equal(sub_s[k], full_s[k][..., idx])
    assert np.abs(full_s["wind"][0]).max() > 0


def test_sticky_observation_bias_is_added_to_the_delayed_rows():
    """A per-drone constant bias on the p, v, rpy, w rows (the sticky
    per-episode observation bias recommended with the table) shifts every
    returned row by exactly that bias, delayed or not, and leaves the state
    and the quaternion and rotor rows alone."""
    P = orc.cf2x()
    h = orc.derive(P).hover_rpm
    n, K = 4, 10
    rng = np.random.default_rng(47)
    act = h * (1 + rng.uniform(-0.05, 0.05, size=(K, 4, n)))
    bias = rng.normal(0, 0.05, (12, n))
    rows = [0, 1, 2, 10, 11, 12, 7, 8, 9, 13, 14, 15]
    for od in (None, np.array([0, 1, 3, 6], dtype=np.int32)):
        plain_s = orc.dr_state(_state(n), orc.ACT_RPM)
        plain = orc.step(P, H, 0, orc.ACT_RPM, 1, np.arange(n + 1), plain_s, act, True, K, n_obs_slots=K,
                         dr=dict(_ones(n), obs_delay=od))
        s = orc.dr_state(_state(n), orc.ACT_RPM)
        got = orc.step(P, H, 0, orc.ACT_RPM, 1, np.arange(n + 1), s, act, True, K, n_obs_slots=K,
                       dr=dict(_ones(n), obs_delay=od, obs_bias=bias))
        want = plain.copy()
        for b, r in enumerate(rows):
            want[:, r] += bias[b]
        np.testing.assert_array_equal(got, want)
        for k in ("p", "v", "q", "w", "rpm"):
            np.testing.assert_array_equal(s[k], plain_s[k])


def test_oracle_structs_match_their_c_layout(tmp_path):
    """The ctypes mirrors of the oracle's structs have the C header's sizes
    and field offsets, so that every field (counts, rings, counter words,
    bias) reaches the C code where it is meant to."""
    import ctypes
    import os
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no gcc")
    here = os.path.dirname(os.path.abspath(orc.__file__))
    pairs = (("orc_params", orc.Params), ("orc_derived", orc.Derived), ("orc_net", orc.Net),
             ("orc_state", orc._CState), ("orc_wind", orc._CWind), ("orc_dr", orc._CDr))
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "md_oracle.h"', "int main(void) {"]
    for cname, cls in pairs:
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for f, _ in cls._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, f, cname, f))
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.check_call([gcc, "-std=c11", "-I", here, str(src), "-o", str(exe)])
    got = {}
    for line in subprocess.check_output([str(exe)]).decode().splitlines():
        a, b, c = line.split()
        got[(a, b)] = int(c)
    for cname, cls in pairs:
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert got[(cname, f)] == getattr(cls, f).offset, (cname, f)
