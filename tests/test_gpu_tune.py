"""GPU checks of the launch configurations, the autotuner and captured
rollouts: every configuration computes the same physics (bitwise for the
one-lane sweeps and the pair-symmetric sweep), the tuner leaves the caller's
state untouched and caches its choice, graph replays equal eager launches."""
import json
import os

import numpy as np
import pytest

import parity_util as pu
from paper_2606_08039_amd import md, workloads as wl

pytestmark = pytest.mark.gpu


def _run_cfg(w, cfg, steps):
    g = pu.DeviceRun(w)
    if cfg is not None:
        md.md_set_launch_config(g.ctx, **cfg)
    g.run(steps)
    s = g.snapshot()
    g.close()
    return s


WORKLOADS = {
    "formation": lambda: wl.subset_envs(wl.formation(n_envs=8192, seed=4), 512),
    "ragged": lambda: wl.ragged_grid(pu.hover_rpm(), n_envs=300, n_steps=20, seed=6),
}


@pytest.mark.parametrize("name", list(WORKLOADS))
def test_one_lane_configs_are_bitwise_identical(name):
    w = WORKLOADS[name]()
    steps = 20
    ref = _run_cfg(w, dict(lanes_per_drone=1, unroll=1, waves_per_group=1, pair_symmetric=0), steps)
    for cfg in (dict(lanes_per_drone=1, unroll=4, waves_per_group=1, pair_symmetric=1),
                dict(lanes_per_drone=1, unroll=2, waves_per_group=4, pair_symmetric=1),
                dict(lanes_per_drone=1, unroll=4, waves_per_group=2, pair_symmetric=0)):
        got = _run_cfg(w, cfg, steps)
        for k in ("p", "q", "v", "w", "rpm", "pid_int"):
            np.testing.assert_array_equal(got[k], ref[k], err_msg="%s %s" % (cfg, k))


def test_multi_lane_sweeps_match_the_oracle_per_step():
    w = wl.ragged_grid(pu.hover_rpm(), n_envs=200, n_steps=10, seed=7)
    for lpd in (2, 4):
        g = pu.DeviceRun(w)
        md.md_set_launch_config(g.ctx, lanes_per_drone=lpd, unroll=2, waves_per_group=2)
        obs = g.run(10, obs_slots=10)
        g.close()
        prev = w["state"]
        for k in range(10):
            if k > 0:
                prev = pu.obs_to_state(obs[k - 1], prev)
            ref, _, _ = pu.oracle_one_step(w, prev, k)
            pu.assert_blocks(pu.obs_to_state(obs[k]), ref, what="lpd %d step %d" % (lpd, k))


def test_invalid_configs_are_rejected():
    w = wl.ragged_grid(pu.hover_rpm(), n_envs=8, n_steps=1, seed=8)
    g = pu.DeviceRun(w)
    with pytest.raises(md.MdError):
        md.md_set_launch_config(g.ctx, lanes_per_drone=4, waves_per_group=1)  # 16 slots < 32 drones
    with pytest.raises(md.MdError):
        md.md_set_launch_config(g.ctx, lanes_per_drone=2, pair_symmetric=1, waves_per_group=2)
    with pytest.raises(md.MdError):
        md.md_set_launch_config(g.ctx, lanes_per_drone=3)
    with pytest.raises(md.MdError):  # the permute sweep exists with unroll 1 only
        md.md_set_launch_config(g.ctx, lanes_per_drone=1, unroll=2, pair_symmetric=2)
    md.md_set_launch_config(g.ctx, lanes_per_drone=1, unroll=1, pair_symmetric=2)
    g.close()


def test_autotune_keeps_state_and_caches_choice(tmp_path):
    w = wl.subset_envs(wl.formation(n_envs=8192, seed=4), 256)
    g = pu.DeviceRun(w)
    before = g.snapshot()
    cache = str(tmp_path / "tune.json")
    cfg = md.md_autotune(g.ctx, g.state, g.action, False, n_steps=10, cache_path=cache)
    after = g.snapshot()
    for k in before:
        np.testing.assert_array_equal(before[k], after[k])
    rec = json.load(open(cache))
    assert len(rec) == 1 and rec[0]["lpd"] == cfg["lanes_per_drone"] and rec[0]["sym"] == cfg["pair_symmetric"]
    # a second context with the same layout takes the cached choice
    g2 = pu.DeviceRun(w)
    md.md_set_launch_config(g2.ctx, lanes_per_drone=1, unroll=1, waves_per_group=1)
    cfg2 = md.md_autotune(g2.ctx, g2.state, g2.action, False, n_steps=10, cache_path=cache)
    assert cfg2 == cfg
    g.run(5)
    g2.run(5)
    a, b = g.snapshot(), g2.snapshot()
    g.close()
    g2.close()
    if cfg["lanes_per_drone"] == 1:
        for k in a:
            np.testing.assert_array_equal(a[k], b[k])


def test_autotune_with_observations_keeps_state_and_caches_apart(tmp_path):
    import torch
    w = wl.subset_envs(wl.formation(n_envs=8192, seed=4), 256)
    g = pu.DeviceRun(w)
    before = g.snapshot()
    cache = str(tmp_path / "tune.json")
    obs = torch.empty((10, 20, g.n), dtype=torch.float32, device="cuda")
    cfg = md.md_autotune_obs(g.ctx, g.state, g.action, False, obs, 10, n_steps=10, cache_path=cache)
    after = g.snapshot()
    for k in before:
        np.testing.assert_array_equal(before[k], after[k])
    assert md.md_get_launch_config(g.ctx) == cfg
    # the choice timed with observations is cached apart from the one without
    md.md_autotune(g.ctx, g.state, g.action, False, n_steps=10, cache_path=cache)
    rec = json.load(open(cache))
    assert len(rec) == 2 and sum(r["sig"].endswith("_obs") for r in rec) == 1
    for bad in ((None, 10), (obs, 0)):
        with pytest.raises(md.MdError):
            md.md_autotune_obs(g.ctx, g.state, g.action, False, bad[0], bad[1], n_steps=10, cache_path="")
    g.close()


def test_graph_replays_equal_eager_launches():
    import torch
    w = wl.subset_envs(wl.formation(n_envs=8192, seed=4), 128)
    ge, gg = pu.DeviceRun(w), pu.DeviceRun(w)
    graph = md.md_rollout_graph_create(gg.ctx, gg.state, gg.action, False, None, 0,
                                       steps_per_launch=10, n_launches=3, step0=0)
    for rep in range(3):
        md.md_graph_launch(graph)
        torch.cuda.synchronize()
        # eager reference: the same 30 steps with the same step indices (the
        # graph replays step0 = 0..29 each time)
        for l in range(3):
            md.md_step(ge.ctx, ge.state, ge.action, False, None, 0, 10, 10 * l)
        torch.cuda.synchronize()
        _ = torch.ones(1000, device="cuda").sum().item()  # eager work between replays
        a, b = ge.snapshot(), gg.snapshot()
        for k in a:
            np.testing.assert_array_equal(a[k], b[k], err_msg="replay %d %s" % (rep, k))
    md.md_graph_destroy(graph)
    ge.close()
    gg.close()


def test_stale_graph_is_refused_on_the_host():
    """A captured rollout holds the context's lane tables and settings as they
    were at capture: after re-binding (which frees those tables), a new launch
    configuration, a settings change or md_destroy, md_graph_launch returns
    MD_E_LAYOUT without launching anything.  Every check is host-side."""
    import torch
    w = wl.subset_envs(wl.formation(n_envs=8192, seed=4), 64)

    def capture(g):
        return md.md_rollout_graph_create(g.ctx, g.state, g.action, False, None, 0,
                                          steps_per_launch=5, n_launches=2, step0=0)

    def expect_stale(graph):
        before = g.snapshot()
        with pytest.raises(md.MdError) as ei:
            md.md_graph_launch(graph)
        assert ei.value.status == md.MD_E_LAYOUT
        torch.cuda.synchronize()
        after = g.snapshot()
        for k in before:
            np.testing.assert_array_equal(before[k], after[k], err_msg="a stale graph advanced %s" % k)

    g = pu.DeviceRun(w)
    graph = capture(g)
    md.md_graph_launch(graph)  # fresh: runs
    torch.cuda.synchronize()
    md.md_bind_layout(g.ctx, w["env_offsets"])  # same offsets, new tables
    expect_stale(graph)
    md.md_graph_destroy(graph)

    graph = capture(g)
    cfg = md.md_get_launch_config(g.ctx)
    other = dict(lanes_per_drone=1, unroll=1, waves_per_group=2, pair_symmetric=0)
    assert other != cfg
    md.md_set_launch_config(g.ctx, **other)
    expect_stale(graph)
    md.md_graph_destroy(graph)

    # setting the same configuration again keeps a graph valid
    graph = capture(g)
    md.md_set_launch_config(g.ctx, **other)
    md.md_graph_launch(graph)
    torch.cuda.synchronize()
    md.md_set_wind(g.ctx, models=md.MD_WIND_CONSTANT, v_mean=(0.1, 0.0, 0.0))
    expect_stale(graph)
    md.md_graph_destroy(graph)

    graph = capture(g)
    md.md_destroy(g.ctx)
    g.ctx = None
    with pytest.raises(md.MdError) as ei:
        md.md_graph_launch(graph)
    assert ei.value.status == md.MD_E_LAYOUT
    md.md_graph_destroy(graph)  # valid after the context is gone
