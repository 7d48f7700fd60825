"""GPU checks of the rotation sweep (pair_symmetric 3): on layouts whose
environments all have one power-of-two size, interleaved in their wave, it
gives bitwise the rows and state of the wave-permute sweep (pair_symmetric
2) for every size 2..64, partially filled waves, empty environments, several
waves per workgroup, domain randomisation and wind, and in the RK4 kernel;
per-step parity with the oracle; the configuration is refused where it does
not apply."""
import numpy as np
import pytest

import parity_util as pu
from paper_2606_08039_amd import md, workloads as wl

pytestmark = pytest.mark.gpu

SHAPES = {2: (2, 1, 1), 4: (2, 2, 1), 8: (2, 2, 2), 16: (4, 2, 2), 32: (4, 4, 2), 64: (4, 4, 4)}


def cfg(sym, waves=1):
    return dict(lanes_per_drone=1, unroll=1, waves_per_group=waves, pair_symmetric=sym)


def _uniform(m, n_envs, seed, n_steps=40):
    return wl.lattice(n_envs=n_envs, shape=SHAPES[m], n_steps=n_steps, seed=seed)


def _same(w, waves, steps=(7, 13, 20)):
    """Bitwise equality of rows and state between pair_symmetric 2 and 3."""
    a = pu.DeviceRun(w, cfg=cfg(2, waves))
    b = pu.DeviceRun(w, cfg=cfg(3, waves))
    try:
        for k in steps:
            oa = a.run(k, obs_slots=k)
            ob = b.run(k, obs_slots=k)
            np.testing.assert_array_equal(ob, oa)
        sa, sb = a.snapshot(), b.snapshot()
        for key in sa:
            np.testing.assert_array_equal(sb[key], sa[key], err_msg=key)
    finally:
        a.close()
        b.close()


@pytest.mark.parametrize("m", [2, 4, 8, 16, 32, 64])
@pytest.mark.parametrize("waves", [1, 4])
def test_bitwise_equal_to_wave_permute_sweep(m, waves):
    # 37 environments: the last wave is partially filled for every m < 64
    _same(_uniform(m, 37, 20 + m), waves)


def test_empty_environments_and_trailing_groups():
    w = _uniform(32, 45, 71)
    sizes = np.diff(w["env_offsets"])
    keep = np.ones(len(sizes), dtype=bool)
    keep[[0, 3, 44]] = False
    # drop three environments but keep their (now empty) entries in the layout
    off = np.concatenate([[0], np.cumsum(np.where(keep, sizes, 0))]).astype(np.int32)
    idx = np.concatenate([np.arange(w["env_offsets"][e], w["env_offsets"][e + 1]) for e in range(len(sizes)) if keep[e]])
    state = {k: np.ascontiguousarray(v[:, idx]) for k, v in w["state"].items()}
    act = np.ascontiguousarray(w["action"][:, :, idx])
    w2 = dict(w, env_offsets=off, state=state, action=act)
    _same(w2, 2)


def test_domain_randomization_and_wind():
    base = _uniform(32, 64, 72)
    w = wl.randomized(base, 73)
    _same(w, 2)


def test_per_step_parity_with_the_oracle():
    w = _uniform(16, 300, 74, n_steps=100)
    g = pu.DeviceRun(w, cfg=cfg(3, 2))
    try:
        for k in (0, 1, 9, 60):
            if k > g.step_index:
                g.run(k - g.step_index)
            s0 = g.snapshot()
            g.run(1)
            s1 = g.snapshot()
            ref, _, _ = pu.oracle_one_step(w, s0, k)
            pu.assert_blocks(s1, ref, blocks=pu.BLOCKS + ("pid_int",), what="rotation sweep step %d" % k)
    finally:
        g.close()


def test_refused_where_it_does_not_apply():
    ragged = wl.thin_envs(wl.lattice(n_envs=64, shape=(4, 4, 2), n_steps=10, seed=5), 6)
    odd = wl.lattice(n_envs=64, shape=(3, 2, 2), n_steps=10, seed=5)  # 12 drones: not a power of two
    for w in (ragged, odd):
        g = pu.DeviceRun(w)
        with pytest.raises(md.MdError):
            md.md_set_launch_config(g.ctx, **cfg(3))
        g.close()
    g = pu.DeviceRun(_uniform(32, 8, 5))
    with pytest.raises(md.MdError):
        md.md_set_launch_config(g.ctx, lanes_per_drone=1, unroll=2, waves_per_group=1, pair_symmetric=3)
    md.md_set_launch_config(g.ctx, **cfg(3))
    g.close()


def test_rk4_bitwise_equal_to_wave_permute_sweep():
    _same(dict(_uniform(32, 37, 75), integrator="rk4"), 2)
    _same(dict(_uniform(8, 37, 76), integrator="rk4"), 1)
