"""GPU checks of the wave-shuffle pair-symmetric sweep (pair_symmetric 2):
per-step parity with the oracle on ragged layered lattices (odd and even
environment sizes up to 64, idle lanes, 1-4 waves per workgroup), the
coplanar grid, RK4 and domain randomisation; bitwise invariance to the
environment order and to chunking; rejection of environments above 64."""
import numpy as np
import pytest

import parity_util as pu
from paper_2606_08039_amd import md, workloads as wl

pytestmark = pytest.mark.gpu


def shfl(waves=1, unroll=1):
    return dict(lanes_per_drone=1, unroll=unroll, waves_per_group=waves, pair_symmetric=2)


def _snap_parity(w, ks, cfg, blocks=pu.BLOCKS, env_subset=None):
    g = pu.DeviceRun(w, cfg=cfg)
    worst = {}
    try:
        for k in ks:
            if k > g.step_index:
                g.run(k - g.step_index)
            s0 = g.snapshot()
            g.run(1)
            s1 = g.snapshot()
            ref, _, idx = pu.oracle_one_step(w, s0, k, env_subset=env_subset)
            e = pu.assert_blocks(s1, ref, idx, blocks=blocks, what="shuffle sweep step %d" % k)
            worst = {kk: max(worst.get(kk, 0.0), v) for kk, v in e.items()}
    finally:
        g.close()
    return worst


def _ragged(n_envs, seed, shape=(4, 4, 2), m_lo=2):
    return wl.thin_envs(wl.lattice(n_envs=n_envs, shape=shape, n_steps=100, seed=seed), seed + 100, m_lo=m_lo)


@pytest.mark.parametrize("waves", [1, 2, 4])
def test_ragged_lattice_per_step(waves):
    w = _ragged(600, 3)
    worst = _snap_parity(w, [0, 1, 7, 60], shfl(waves), blocks=pu.BLOCKS + ("pid_int",))
    print("shuffle sweep, ragged lattice, %d waves: %s" % (waves, worst))


def test_environments_up_to_64_drones():
    w = _ragged(200, 5, shape=(4, 4, 4), m_lo=33)  # 33..64 drones, one environment per wave
    _snap_parity(w, [0, 1, 30], shfl(2), blocks=pu.BLOCKS + ("pid_int",))


def test_coplanar_grid_per_step():
    w = wl.ragged_grid(pu.hover_rpm(), n_envs=300, n_steps=10, seed=7)
    g = pu.DeviceRun(w, cfg=shfl(1))
    obs = g.run(10, obs_slots=10)
    g.close()
    prev = w["state"]
    for k in range(10):
        if k > 0:
            prev = pu.obs_to_state(obs[k - 1], prev)
        ref, _, _ = pu.oracle_one_step(w, prev, k)
        pu.assert_blocks(pu.obs_to_state(obs[k]), ref, what="coplanar step %d" % k)


def test_rk4_and_domain_randomization():
    w = dict(wl.subset_envs(wl.formation(n_envs=8192, n_steps=1000, seed=4), 128), integrator="rk4")
    _snap_parity(w, [0, 1, 5], shfl(8), blocks=pu.BLOCKS + ("pid_int",))
    base = wl.subset_envs(wl.formation(n_envs=8192, n_steps=1000, seed=4), 128)
    w = dict(base, dr=wl.domain_randomization(base, 61))
    _snap_parity(w, [0, 1, 13], shfl(8), blocks=pu.BLOCKS + ("pid_int", "rpm_cmd"))


def test_bitwise_invariance_to_order_and_chunking():
    w = _ragged(300, 9)
    rng = np.random.default_rng(3)
    perm = rng.permutation(len(w["env_offsets"]) - 1)
    wp = wl.permute_envs(w, perm)
    a = pu.DeviceRun(w, cfg=shfl(2))
    a.run(25)
    sa = a.snapshot()
    a.close()
    b = pu.DeviceRun(wp, cfg=shfl(4))
    for k in (5, 20):
        b.run(k)
    sb = b.snapshot()
    b.close()
    idx = wp["drone_index"]
    for k in ("p", "q", "v", "w", "rpm", "pid_int"):
        np.testing.assert_array_equal(sb[k], sa[k][:, idx], err_msg=k)


def test_environments_above_64_are_rejected():
    w = _ragged(4, 11, shape=(5, 5, 3), m_lo=70)
    g = pu.DeviceRun(w)
    with pytest.raises(md.MdError):
        md.md_set_launch_config(g.ctx, **shfl(2))
    g.close()
