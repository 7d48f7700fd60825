"""GPU parity of the plain step (libmd HIP kernels) against the FP64 oracle,
called through the C ABI on the seeded workloads, plus layout, chunking and
error-path behaviour."""
import numpy as np
import pytest

import parity_util as pu
from paper_2606_08039_amd import md, workloads as wl

pytestmark = pytest.mark.gpu


def _per_step_from_obs(w, obs, s0, steps):
    """RPM workloads: the KIN rows hold the full state; step the oracle once
    from each GPU state and compare with the next GPU state."""
    worst = {k: 0.0 for k in pu.BLOCKS}
    prev = s0
    for k in steps:
        if k > 0:
            prev = pu.obs_to_state(obs[k - 1], prev)
        ref, robs, _ = pu.oracle_one_step(w, prev, k, obs_slots=1)
        got = pu.obs_to_state(obs[k])
        e = pu.assert_blocks(got, ref, what="step %d" % k)
        # observation extras: roll/pitch/yaw
        a, b = obs[k][7:10].astype(np.float64), robs[0][7:10]
        assert np.max(np.abs(a - b)) <= pu.TOL * max(1.0, np.max(np.abs(b))), k
        worst = {kk: max(worst[kk], e[kk]) for kk in worst}
    return worst


def test_single_drone_rpm_per_step():
    w = wl.single(pu.hover_rpm(), n_steps=240, seed=0)
    g = pu.DeviceRun(w)
    obs = g.run(240, obs_slots=240)
    g.close()
    worst = _per_step_from_obs(w, obs, w["state"], range(240))
    print("single drone, 240 steps, worst scaled error per block:", worst)


def test_fast_spin_takes_the_exact_sine_and_cosine():
    """Body rates of 150-260 rad/s put th = |w| dt / 2 above 1/4, where the
    exponential map leaves its Taylor series for sine and cosine; per-step
    parity with the oracle over 40 steps (ground effect and drag on)."""
    w = wl.single(pu.hover_rpm(), n_steps=40, seed=5)
    w = dict(w, aero_mask=3)
    w["state"]["w"][:, 0] = (150.0, -80.0, 200.0)
    assert np.linalg.norm(w["state"]["w"][:, 0]) * wl.DT / 2 > 0.25
    g = pu.DeviceRun(w)
    obs = g.run(40, obs_slots=40)
    g.close()
    worst = _per_step_from_obs(w, obs, w["state"], range(40))
    print("fast spin, 40 steps, worst scaled error per block:", worst)


def test_single_drone_hover_1000_steps_trajectory():
    w = wl.single(pu.hover_rpm(), n_steps=1000, jitter=0.0, seed=0)
    g = pu.DeviceRun(w)
    g.run(1000)
    got = g.snapshot()
    g.close()
    ref, _, _ = pu.oracle_one_step(w, w["state"], 0, n_steps=1000)
    dp = np.max(np.abs(got["p"].astype(np.float64) - ref["p"]))
    print("hover 1000 steps: |dp| =", dp)
    assert dp <= 1e-3
    # float32 rounding of HOVER_RPM alone leaves |a| < 1e-6 m/s^2: < 1e-5 m over 4.2 s
    assert np.max(np.abs(ref["p"][:, 0] - [0, 0, 1])) < 1e-5


def test_single_drone_rpm_trajectory_240_steps():
    w = wl.single(pu.hover_rpm(), n_steps=240, seed=0)
    g = pu.DeviceRun(w)
    g.run(240)
    got = g.snapshot()
    g.close()
    ref, _, _ = pu.oracle_one_step(w, w["state"], 0, n_steps=240)
    assert np.max(np.abs(got["p"] - ref["p"])) <= 1e-3


def _snapshot_parity(w, ks, env_subset=None, mask=None, obs=False, cfg=None):
    """Launch [0, k) then one more step; compare that step with the oracle
    stepped from the GPU snapshot (optionally on a subset of environments)."""
    worst = {kk: 0.0 for kk in pu.BLOCKS}
    g = pu.DeviceRun(w, mask=mask, cfg=cfg)
    try:
        for k in ks:
            if k > g.step_index:
                g.run(k - g.step_index)
            s0 = g.snapshot()
            gobs = g.run(1, obs_slots=1 if obs else 0)
            s1 = g.snapshot()
            ref, robs, idx = pu.oracle_one_step(w, s0, k, env_subset=env_subset, mask=mask,
                                                obs_slots=1 if obs else 0)
            e = pu.assert_blocks(s1, ref, idx, what="step %d" % k)
            if w["act_type"] == "pid":
                e2 = pu.block_errors(s1, ref, idx, blocks=("pid_int",))
                assert e2["pid_int"] <= pu.TOL, (k, e2)
            if obs:
                a = gobs[0] if idx is None else gobs[0][:, idx]
                sc = np.maximum(np.max(np.abs(robs[0]), axis=0), 1.0)
                assert np.max(np.max(np.abs(a - robs[0]), axis=0) / sc) <= pu.TOL, k
            worst = {kk: max(worst[kk], e[kk]) for kk in worst}
    finally:
        g.close()
    return worst


def test_pid_field_per_step_small():
    w = wl.subset_envs(wl.pid_field(n_envs=4096, n_steps=2400, seed=1), 512)
    worst = _snapshot_parity(w, list(range(0, 12)) + [37, 240, 241, 600])
    print("pid field (512 envs), worst:", worst)


def test_pid_field_full_size_sampled():
    w = wl.pid_field(n_envs=4096, n_steps=2400, seed=1)
    worst = _snapshot_parity(w, [0, 4, 5, 1203, 2399], obs=True)
    print("pid field 4096 envs, worst:", worst)


@pytest.mark.parametrize("cfg", ["default", "autotuned"])
def test_ragged_downwash_full_size_per_step(cfg):
    """The ragged 1024-environment layout, every drone at every one of its
    100 steps, in the default configuration and in the one the autotuner
    picks for it (the benchmark's: several lanes per drone, their partial
    sums combined across lanes)."""
    w = wl.ragged_grid(pu.hover_rpm(), n_envs=1024, n_steps=100, seed=2)
    g = pu.DeviceRun(w)
    c = None
    if cfg == "autotuned":
        md.md_autotune(g.ctx, g.state, g.action_slice(0, 10), w["action_per_step"], n_steps=10, cache_path="")
        c = md.md_get_launch_config(g.ctx)
    obs = g.run(100, obs_slots=100)
    g.close()
    worst = _per_step_from_obs(w, obs, w["state"], range(100))
    print("ragged grid 1024 envs, %s %s, worst:" % (cfg, c), worst)


@pytest.mark.parametrize("cfg", ["default", "autotuned", "rotation"])
def test_formation_full_size_sampled(cfg):
    """The benchmark workload at full size: the default configuration, the
    one the autotuner picks (the benchmark's), and the rotation sweep."""
    w = wl.formation(n_envs=8192, n_steps=1000, seed=4)
    if cfg == "default":
        c = None
    elif cfg == "rotation":
        c = dict(lanes_per_drone=1, unroll=1, waves_per_group=8, pair_symmetric=3)
    else:
        g = pu.DeviceRun(w)
        md.md_autotune(g.ctx, g.state, g.action_slice(0, 50), w["action_per_step"], n_steps=50, cache_path="")
        c = md.md_get_launch_config(g.ctx)
        g.close()
    rng = np.random.default_rng(0)
    envs = np.sort(rng.choice(8192, 48, replace=False))
    worst = _snapshot_parity(w, [0, 1, 5, 333, 999], env_subset=envs, obs=True, cfg=c)
    print("formation 8192x32 (48 sampled envs), %s %s, worst:" % (cfg, c), worst)


def test_lattice8_sampled():
    w = wl.lattice(n_envs=16384, shape=(2, 2, 2), n_steps=1000, seed=3)
    rng = np.random.default_rng(1)
    envs = np.sort(rng.choice(16384, 64, replace=False))
    worst = _snapshot_parity(w, [0, 3, 10, 500], env_subset=envs)
    print("lattice 16384x8 (64 sampled envs), worst:", worst)


@pytest.mark.parametrize("mask", [0, 1, 2, 4, 7])
def test_each_aero_term_on_ragged_layout(mask):
    w = wl.ragged_grid(pu.hover_rpm(), n_envs=64, n_steps=20, seed=5)
    g = pu.DeviceRun(w, mask=mask)
    obs = g.run(20, obs_slots=20)
    g.close()
    w = dict(w, aero_mask=mask)
    _per_step_from_obs(w, obs, w["state"], range(20))


def test_packing_is_bitwise_invariant_to_environment_order():
    w = wl.ragged_grid(pu.hover_rpm(), n_envs=300, n_steps=30, seed=6)
    perm = np.random.default_rng(7).permutation(300)
    wp = wl.permute_envs(w, perm)
    g1, g2 = pu.DeviceRun(w), pu.DeviceRun(wp)
    g1.run(30)
    g2.run(30)
    a, b = g1.snapshot(), g2.snapshot()
    g1.close()
    g2.close()
    for k in ("p", "q", "v", "w", "rpm"):
        np.testing.assert_array_equal(a[k][:, wp["drone_index"]], b[k])


def test_chunked_launches_equal_one_launch():
    # PID phase carried by step0; held actions; bitwise equal
    w = wl.lattice(n_envs=256, shape=(2, 2, 2), n_steps=60, seed=8)
    g1, g2 = pu.DeviceRun(w), pu.DeviceRun(w)
    g1.run(60)
    for k in (7, 13, 1, 39):
        g2.run(k)
    a, b = g1.snapshot(), g2.snapshot()
    g1.close()
    g2.close()
    for k in a:
        np.testing.assert_array_equal(a[k], b[k])


def test_observation_ring_keeps_last_steps():
    w = wl.ragged_grid(pu.hover_rpm(), n_envs=16, n_steps=10, seed=9)
    g1, g2 = pu.DeviceRun(w), pu.DeviceRun(w)
    full = g1.run(10, obs_slots=10)
    ring = g2.run(10, obs_slots=4)
    g1.close()
    g2.close()
    for k in range(6, 10):
        np.testing.assert_array_equal(ring[k % 4], full[k])


def test_held_action_equals_repeated_per_step_action():
    w = wl.ragged_grid(pu.hover_rpm(), n_envs=32, n_steps=1, seed=10)
    w_rep = dict(w, action=np.repeat(w["action"], 12, axis=0), action_per_step=True)
    w_hold = dict(w, action=w["action"], action_per_step=False)
    g1, g2 = pu.DeviceRun(w_rep), pu.DeviceRun(w_hold)
    g1.run(12)
    g2.run(12)
    a, b = g1.snapshot(), g2.snapshot()
    g1.close()
    g2.close()
    for k in ("p", "q", "v", "w", "rpm"):
        np.testing.assert_array_equal(a[k], b[k])


@pytest.mark.parametrize("sizes", [[0, 3, 0, 1, 0], [64, 65, 1, 2], [200, 7], [1024, 5, 0]])
def test_edge_layouts(sizes):
    rng = np.random.default_rng(11)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
    n = int(off[-1])
    s = wl.empty_state(n)
    s["p"][:] = rng.uniform([-1, -1, 0.2], [1, 1, 2.5], size=(n, 3)).T
    act = (pu.hover_rpm() * (1 + rng.uniform(-0.1, 0.1, size=(5, 4, n)))).astype(np.float32)
    w = dict(name="edge", env_offsets=off, state=s, action=act, action_per_step=True,
             aero_mask=7, act_type="rpm", ctrl_decim=1, n_steps=5, dt=wl.DT)
    g = pu.DeviceRun(w)
    obs = g.run(5, obs_slots=5)
    g.close()
    _per_step_from_obs(w, obs, s, range(5))


def test_zero_steps_and_zero_drones_are_no_ops():
    w = wl.ragged_grid(pu.hover_rpm(), n_envs=8, n_steps=1, seed=12)
    g = pu.DeviceRun(w)
    before = g.snapshot()
    g.run(0)
    after = g.snapshot()
    g.close()
    for k in before:
        np.testing.assert_array_equal(before[k], after[k])
    p = pu.params()
    ctx = md.md_create(p, wl.DT, 7, md.MD_ACT_RPM, 1)
    md.md_bind_layout(ctx, [0, 0, 0])
    import torch
    st = md.DeviceState(0)
    md.md_step(ctx, st, torch.zeros(4, device="cuda"), False, None, 0, 3, 0)
    md.md_destroy(ctx)


def test_error_paths():
    import ctypes
    import torch
    p = pu.params()
    ctx = md.md_create(p, wl.DT, 7, md.MD_ACT_RPM, 1)
    st = md.DeviceState(4)
    act = torch.zeros((1, 4, 4), device="cuda")
    with pytest.raises(md.MdError) as ei:
        md.md_step(ctx, st, act, False, None, 0, 1, 0)
    assert ei.value.status == md.MD_E_LAYOUT
    with pytest.raises(md.MdError) as ei:
        md.md_bind_layout(ctx, [0, 1025])
    assert ei.value.status == md.MD_E_UNSUPPORTED
    with pytest.raises(md.MdError) as ei:
        md.md_bind_layout(ctx, [0, 3, 2, 4])
    assert ei.value.status == md.MD_E_LAYOUT
    md.md_bind_layout(ctx, [0, 4])
    L = md.lib()
    bad = md.md_state(st.t["p"].data_ptr(), None, None, None, None, None)
    assert L.md_step(ctx, ctypes.byref(bad), ctypes.c_void_p(act.data_ptr()), 0, None, 0, 1, 0,
                     None) == md.MD_E_INVALID_ARG
    assert "null" in md.md_last_error(ctx)
    md.md_step(ctx, st, act, False, None, 0, 1, 0)
    torch.cuda.synchronize()
    md.md_destroy(ctx)
