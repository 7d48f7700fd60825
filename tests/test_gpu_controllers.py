"""GPU parity of the VEL, ATTITUDE and DSL-style PID action types against the
FP64 oracle (per-step criterion from GPU snapshots, including the controller
integrals and the DSL setpoint), and their closed-loop behaviour on the GPU."""
import numpy as np
import pytest

import parity_util as pu
from paper_2606_08039_amd import md, workloads as wl

pytestmark = pytest.mark.gpu


def _hover_thrust():
    p = md.md_default_params_cf2x()
    return p.m * p.g


@pytest.mark.parametrize("kind", ["vel", "attitude", "dsl"])
def test_controller_per_step_parity(kind):
    w = wl.commanded(kind, _hover_thrust(), n_envs=1024, n_steps=480, seed=5)
    g = pu.DeviceRun(w)
    worst = {}
    try:
        for k in (0, 1, 4, 5, 6, 10, 97, 240, 479):
            if k > g.step_index:
                g.run(k - g.step_index)
            s0 = g.snapshot()
            g.run(1)
            s1 = g.snapshot()
            ref, _, _ = pu.oracle_one_step(w, s0, k)
            e = pu.assert_blocks(s1, ref, blocks=pu.BLOCKS + ("pid_int",) + (("ctl",) if kind == "dsl" else ()),
                                 what="%s step %d" % (kind, k))
            worst = {kk: max(worst.get(kk, 0.0), v) for kk, v in e.items()}
    finally:
        g.close()
    print(kind, "worst:", worst)


def test_vel_command_is_tracked_on_gpu():
    w = wl.commanded("vel", _hover_thrust(), n_envs=256, n_steps=2400, seed=6)
    w = dict(w, aero_mask=0)
    g = pu.DeviceRun(w)
    g.run(2400)
    s = g.snapshot()
    g.close()
    cmd = w["action"][0]
    # final yaw rate equals the command (rate loop, torque-free yaw)
    np.testing.assert_allclose(s["w"][2], cmd[3], atol=1e-3)
    assert np.all(np.isfinite(s["p"]))


def test_dsl_setpoint_block_reaches_waypoints():
    w = wl.commanded("dsl", _hover_thrust(), n_envs=256, n_steps=2400, seed=7)
    g = pu.DeviceRun(w)
    g.run(2400)
    s = g.snapshot()
    g.close()
    cmd = w["action"][0]
    np.testing.assert_allclose(s["ctl"][0:3], cmd[0:3], atol=1e-5)
