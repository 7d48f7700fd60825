"""GPU parity of the classic Runge-Kutta step (md_set_integrator MD_INTEG_RK4)
against the oracle's RK4 step: per-step criterion from GPU snapshots on a
ragged (thinned) lattice, the 8192 x 32 formation (sampled environments,
both neighbour sweeps), each aerodynamic term, every action type; bitwise
agreement of the all-pairs and pair-symmetric sweeps; error paths.

The downwash cases use layered workloads.  On layouts with coplanar drones
(the 0.15 m grid) the Runge-Kutta stages move coplanar drones apart by
rounding-sized amounts, so the strict dz > 0 gate and the 1/dz^2 factor of
Eq. 6 turn rounding differences between float32 and the FP64 oracle into
arbitrarily large force differences: per-step parity is not defined there
(the semi-implicit Euler step evaluates Eq. 6 at stored positions only,
which both sides share exactly)."""
import numpy as np
import pytest

import parity_util as pu
from paper_2606_08039_amd import md, workloads as wl

pytestmark = pytest.mark.gpu

SYM = dict(lanes_per_drone=1, unroll=4, waves_per_group=1, pair_symmetric=1)
ALL = dict(lanes_per_drone=1, unroll=2, waves_per_group=1, pair_symmetric=0)


def _rk(w):
    return dict(w, integrator="rk4")


def _parity(w, ks, env_subset=None, mask=None, cfg=None, extra=()):
    worst = {}
    g = pu.DeviceRun(w, mask=mask, cfg=cfg)
    try:
        for k in ks:
            if k > g.step_index:
                g.run(k - g.step_index)
            s0 = g.snapshot()
            gobs = g.run(1, obs_slots=1)
            s1 = g.snapshot()
            ref, robs, idx = pu.oracle_one_step(w, s0, k, env_subset=env_subset, mask=mask, obs_slots=1)
            e = pu.assert_blocks(s1, ref, idx, blocks=pu.BLOCKS + tuple(extra), what="rk4 step %d" % k)
            a = gobs[0] if idx is None else gobs[0][:, idx]
            sc = np.maximum(np.max(np.abs(robs[0]), axis=0), 1.0)
            assert np.max(np.max(np.abs(a - robs[0]), axis=0) / sc) <= pu.TOL, k
            worst = {kk: max(worst.get(kk, 0.0), v) for kk, v in e.items()}
    finally:
        g.close()
    return worst


def _ragged_lattice(n_envs, seed):
    return wl.thin_envs(wl.subset_envs(wl.formation(n_envs=8192, n_steps=100, seed=4), n_envs), seed)


def test_ragged_lattice_per_step():
    w = _rk(_ragged_lattice(1024, 8))
    print("rk4 ragged lattice 1024 envs, worst:", _parity(w, [0, 1, 2, 5, 50, 99], extra=("pid_int",)))


def test_ragged_grid_without_downwash_per_step():
    w = _rk(wl.ragged_grid(pu.hover_rpm(), n_envs=1024, n_steps=100, seed=2))
    print("rk4 ragged grid (GND|DRAG), worst:", _parity(w, [0, 1, 2, 50, 99], mask=3))


@pytest.mark.parametrize("cfg", [SYM, ALL], ids=["sym", "allpairs"])
def test_formation_full_size_sampled(cfg):
    w = _rk(wl.formation(n_envs=8192, n_steps=1000, seed=4))
    rng = np.random.default_rng(0)
    envs = np.sort(rng.choice(8192, 32, replace=False))
    worst = _parity(w, [0, 1, 5, 333], env_subset=envs, cfg=cfg, extra=("pid_int",))
    print("rk4 formation 8192x32 (32 sampled envs)", cfg, "worst:", worst)


@pytest.mark.parametrize("mask", [0, 1, 2, 4, 7])
def test_each_aero_term_on_ragged_layout(mask):
    w = _rk(_ragged_lattice(64, 9))
    _parity(w, [0, 3, 19], mask=mask)


@pytest.mark.parametrize("kind", ["vel", "attitude", "dsl"])
def test_controllers_per_step(kind):
    p = md.md_default_params_cf2x()
    w = _rk(wl.commanded(kind, p.m * p.g, n_envs=256, n_steps=240, seed=5))
    extra = ("pid_int",) + (("ctl",) if kind == "dsl" else ())
    _parity(w, [0, 1, 5, 6, 239], extra=extra)


def test_symmetric_and_all_pairs_sweeps_are_bitwise_equal():
    w = _rk(_ragged_lattice(300, 10))
    out = []
    for cfg in (ALL, SYM, dict(ALL, waves_per_group=2, unroll=1)):
        g = pu.DeviceRun(w, cfg=cfg)
        g.run(30)  # the held PID waypoints serve every step
        out.append(g.snapshot())
        g.close()
    for o in out[1:]:
        for k in pu.BLOCKS:
            np.testing.assert_array_equal(o[k], out[0][k], err_msg=k)


def test_single_drone_trajectory_and_difference_from_euler():
    w = _rk(wl.single(pu.hover_rpm(), n_steps=240, seed=0))
    g = pu.DeviceRun(w)
    g.run(240)
    got = g.snapshot()
    g.close()
    ref, _, _ = pu.oracle_one_step(w, w["state"], 0, n_steps=240)
    dp = np.max(np.abs(got["p"].astype(np.float64) - ref["p"]))
    eu, _, _ = pu.oracle_one_step(dict(w, integrator="euler"), w["state"], 0, n_steps=240)
    d_eu = np.max(np.abs(eu["p"] - ref["p"]))
    print("rk4 single drone 240 steps: |dp| gpu-oracle %.3g, rk4-euler %.3g" % (dp, d_eu))
    assert dp <= 1e-4 and d_eu > 10 * dp


def test_error_paths():
    p = md.md_default_params_cf2x()
    ctx = md.md_create(p, wl.DT, md.MD_AERO_SURROGATE, md.MD_ACT_PID, 5)
    with pytest.raises(md.MdError):
        md.md_set_integrator(ctx, md.MD_INTEG_RK4)
    md.md_destroy(ctx)
    ctx = md.md_create(p, wl.DT, 7, md.MD_ACT_RPM, 1)
    with pytest.raises(md.MdError):
        md.md_set_integrator(ctx, 7)
    md.md_bind_layout(ctx, np.array([0, 5, 9], dtype=np.int32))
    md.md_set_launch_config(ctx, lanes_per_drone=2, unroll=1, waves_per_group=1, pair_symmetric=0)
    md.md_set_integrator(ctx, md.MD_INTEG_RK4)
    assert md.md_get_integrator(ctx) == md.MD_INTEG_RK4
    assert md.md_get_launch_config(ctx)["lanes_per_drone"] == 1
    with pytest.raises(md.MdError):
        md.md_set_launch_config(ctx, lanes_per_drone=4, unroll=1, waves_per_group=1, pair_symmetric=0)
    md.md_destroy(ctx)
