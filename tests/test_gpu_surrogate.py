"""GPU parity of the surrogate path: training-sample generation (neighbours,
features, plain residual) and the step with the in-step BF16 MFMA network,
its fallback and its judge, against the FP64 oracle."""
import numpy as np
import pytest

import oracle as orc
import parity_util as pu
from paper_2606_08039_amd import md, workloads as wl

pytestmark = pytest.mark.gpu


def _datagen(w, steps_before=0):
    import torch
    g = pu.DeviceRun(w)
    if steps_before:
        g.run(steps_before)
    s = g.snapshot()
    n = g.n
    X = torch.zeros((n, 64), device="cuda")
    Y = torch.zeros((n, 6), device="cuda")
    nbr = torch.zeros((n, 8), dtype=torch.int32, device="cuda")
    md.md_datagen(g.ctx, g.state, 7, X, Y, nbr)
    torch.cuda.synchronize()
    out = (s, X.cpu().numpy(), Y.cpu().numpy(), nbr.cpu().numpy())
    g.close()
    return out


@pytest.mark.parametrize("kind", ["lattice8", "formation", "ragged"])
def test_datagen_matches_oracle(kind):
    if kind == "lattice8":
        w = wl.subset_envs(wl.lattice(n_envs=16384, shape=(2, 2, 2), seed=3), 512)
    elif kind == "formation":
        w = wl.subset_envs(wl.formation(n_envs=8192, seed=4), 128)
    else:
        w = wl.ragged_grid(pu.hover_rpm(), n_envs=128, n_steps=3, seed=2)
    s32, X, Y, nbr = _datagen(w, steps_before=3)
    s = pu.to_oracle_state(s32)
    P = pu.oracle_params()
    ref_nbr = orc.knn(w["env_offsets"], s["p"], 8)
    np.testing.assert_array_equal(nbr, ref_nbr)
    Xr = orc.features(P, w["env_offsets"], s, ref_nbr)
    err = np.abs(X - Xr)
    assert np.max(err / np.maximum(np.abs(Xr), 1.0)) < 1e-6, np.max(err)
    Yr = orc.aero_residual(P, 7, w["env_offsets"], s)
    sc = np.maximum(np.max(np.abs(Yr[:, :3]), axis=1), 1e-3)
    e = np.max(np.abs(Y[:, :3] - Yr[:, :3]), axis=1) / sc
    # All downwash terms share one sign, so the sum's relative error is bounded
    # by the worst term's: float32 exp(-u) with u = dxy^2 / (2 beta^2) carries
    # about u times the relative error of u (a few ulp), plus a few ulp.
    tol = (6.0 + 4.0 * _max_exponent(P, w["env_offsets"], s)) * 2.0 ** -23
    print("%s: worst residual error (scaled) %.2e (bound %.2e), max |F| %.3g"
          % (kind, e.max(), tol.max(), np.abs(Yr).max()))
    assert np.all(e <= np.maximum(tol, 1e-5))
    assert np.all(Y[:, 3:] == 0)


def _max_exponent(P, off, s):
    """Per drone, the largest downwash exponent dxy^2 / (2 beta^2) among the
    pairs that act on it (0 if none)."""
    out = np.zeros(int(off[-1]))
    p = s["p"]
    for e in range(len(off) - 1):
        i0, i1 = int(off[e]), int(off[e + 1])
        dz = p[2, i0:i1][None, :] - p[2, i0:i1][:, None]
        dx = p[0, i0:i1][None, :] - p[0, i0:i1][:, None]
        dy = p[1, i0:i1][None, :] - p[1, i0:i1][:, None]
        d2 = dx * dx + dy * dy
        beta = P.C2 * dz + P.C3
        u = np.where((dz > 0) & (d2 < 100), d2 / (2 * beta * beta + 1e-300), 0.0)
        out[i0:i1] = u.max(axis=1)
    return out


def _random_net(rng, scale=0.5):
    parts = []
    for sh in md.MLP_SHAPES:
        if len(sh) == 2:
            parts.append(rng.normal(size=sh) * np.sqrt(2.0 / sh[1]) * scale)
        else:
            parts.append(rng.normal(size=sh) * 0.05)
    flat = md.mlp_flatten(parts)
    xm = np.zeros(64)
    xs = np.ones(64)
    xs[10:58] = 2.0  # relative positions / velocities
    ym = np.array([0.0, 0.0, -0.01, 0.0, 0.0, 0.0])
    ys = np.array([0.005, 0.005, 0.01, 1e-7, 1e-7, 1e-7])
    return flat, np.concatenate([xm, xs, ym, ys]).astype(np.float32)


class SurRun(pu.DeviceRun):
    def __init__(self, w, flat, norm, dz_ood=1e-3, judge_stride=0):
        import torch
        self.w = w
        self.p = pu.params()
        self.mask = md.MD_AERO_SURROGATE
        self.ctx = md.md_create(self.p, w["dt"], self.mask, pu.ACT[w["act_type"]], w["ctrl_decim"])
        md.md_bind_layout(self.ctx, w["env_offsets"])
        md.md_load_surrogate(self.ctx, flat, norm, dz_ood, judge_stride)
        self.n = int(w["env_offsets"][-1])
        self.state = md.DeviceState.from_numpy(w["state"])
        self.action = torch.from_numpy(np.ascontiguousarray(w["action"], dtype=np.float32)).cuda()
        self.step_index = 0


def _oracle_sur_step(w, s32, k, flat, norm, dz_ood=1e-3, env_subset=None, ood=None):
    P = pu.oracle_params()
    net, keep = orc.make_net(flat, norm, dz_ood, **(ood or {}))
    off = np.asarray(w["env_offsets"], dtype=np.int64)
    s = pu.to_oracle_state(s32)
    act = w["action"]
    idx = None
    sub_off = np.asarray(off, dtype=np.int32)
    if env_subset is not None:
        idx = np.concatenate([np.arange(off[e], off[e + 1]) for e in env_subset])
        m = np.array([off[e + 1] - off[e] for e in env_subset])
        sub_off = np.concatenate([[0], np.cumsum(m)]).astype(np.int32)
        s = {kk: np.ascontiguousarray(v[:, idx]) for kk, v in s.items()}
        act = act[:, :, idx]
    a = act[k:k + 1] if w["action_per_step"] else act[0:1]
    _, aero, fb = orc.step_surrogate(P, w["dt"], pu.ORC_ACT[w["act_type"]],
                                     w["ctrl_decim"], sub_off, s, np.ascontiguousarray(a, dtype=np.float64),
                                     w["action_per_step"], 1, net, step0=k)
    return s, aero, fb, idx


@pytest.mark.parametrize("kind", ["lattice8", "formation"])
def test_surrogate_step_matches_oracle(kind):
    rng = np.random.default_rng(50)
    flat, norm = _random_net(rng)
    if kind == "lattice8":
        w = wl.subset_envs(wl.lattice(n_envs=16384, shape=(2, 2, 2), seed=3), 256)
        envs = None
    else:
        w = wl.formation(n_envs=8192, seed=4)
        envs = np.sort(rng.choice(8192, 32, replace=False))
    g = SurRun(w, flat, norm)
    worst = {k: 0.0 for k in pu.BLOCKS}
    try:
        for k in (0, 1, 4, 5, 40):
            if k > g.step_index:
                g.run(k - g.step_index)
            s0 = g.snapshot()
            g.run(1)
            s1 = g.snapshot()
            ref, aero, fb, idx = _oracle_sur_step(w, s0, k, flat, norm, env_subset=envs)
            e = pu.assert_blocks(s1, ref, idx, what="surrogate step %d" % k)
            worst = {kk: max(worst[kk], e[kk]) for kk in worst}
            assert np.abs(aero[:, :3]).max() > 1e-3  # the network does act
    finally:
        g.close()
    print("%s surrogate step, worst:" % kind, worst)


def test_surrogate_fallback_near_the_downwash_singularity():
    rng = np.random.default_rng(51)
    flat, norm = _random_net(rng)
    s = wl.empty_state(4)
    s["p"][:, 0] = [0.0, 0.0, 1.0]
    s["p"][:, 1] = [0.05, 0.0, 1.0004]   # 0.4 mm above drone 0: singular downwash
    s["p"][:, 2] = [0.0, 0.0, 0.5]
    s["p"][:, 3] = [2.0, 0.0, 0.6]
    hover = pu.hover_rpm()
    act = np.full((1, 4, 4), hover, dtype=np.float32)
    w = dict(name="pair", env_offsets=np.array([0, 2, 4], dtype=np.int32), state=s, action=act,
             action_per_step=False, aero_mask=md.MD_AERO_SURROGATE, act_type="rpm", ctrl_decim=1,
             n_steps=1, dt=wl.DT)
    g = SurRun(w, flat, norm, dz_ood=1e-3, judge_stride=1)
    s0 = g.snapshot()
    g.run(1)
    s1 = g.snapshot()
    j = md.md_judge_stats(g.ctx)
    g.close()
    ref, aero, fb, _ = _oracle_sur_step(w, s0, 0, flat, norm)
    assert list(fb) == [1, 0, 0, 0]
    assert aero[0, 2] < -1.0
    pu.assert_blocks(s1, ref)
    assert j["n_fallback"] == 1 and j["n_judged"] == 3 and j["n_drone_steps"] == 4


def test_judge_matches_oracle_force_error():
    rng = np.random.default_rng(52)
    flat, norm = _random_net(rng)
    w = wl.subset_envs(wl.lattice(n_envs=16384, shape=(2, 2, 2), seed=3), 128)
    g = SurRun(w, flat, norm, judge_stride=1)
    s0 = g.snapshot()
    md.md_judge_reset(g.ctx)
    g.run(1)
    j = md.md_judge_stats(g.ctx)
    g.close()
    ref, aero, fb, _ = _oracle_sur_step(w, s0, 0, flat, norm)
    # plain residual at the pre-step state with this step's rotor speeds
    P = pu.oracle_params()
    s = pu.to_oracle_state(s0)
    Yp = orc.aero_residual(P, 7, w["env_offsets"], s, rpm=ref["rpm"])
    ok = fb == 0
    err2 = np.sum((aero[ok, :3] - Yp[ok, :3]) ** 2)
    ref2 = np.sum(Yp[ok, :3] ** 2)
    assert j["n_judged"] == ok.sum()
    assert j["force_rel_err"] == pytest.approx(np.sqrt(err2 / ref2), rel=1e-3)


def test_out_of_distribution_fallback_matches_oracle():
    """Fast, relatively fast and tilted drones take the plain terms on both
    sides (decisions in binary32), and the step matches the oracle."""
    rng = np.random.default_rng(53)
    flat, norm = _random_net(rng)
    w = wl.subset_envs(wl.lattice(n_envs=16384, shape=(2, 2, 2), seed=3), 128)
    n = int(w["env_offsets"][-1])
    st = {k: v.copy() for k, v in w["state"].items()}
    pick = rng.choice(n, 60, replace=False)
    st["v"][:, pick[:20]] += rng.uniform(-3, 3, size=(3, 20))            # fast
    th = rng.uniform(0.01, 0.2, size=20)                                 # tilted up to 11 degrees
    st["q"][:, pick[20:40]] = np.stack([np.cos(th / 2), np.sin(th / 2), np.zeros(20), np.zeros(20)])
    st["v"][2, pick[40:]] += rng.uniform(-2.5, 2.5, size=20)            # vertical speed only
    w = dict(w, state=st)
    ood = dict(ood_speed=1.5, ood_rel_speed=2.0, ood_tilt=np.radians(2.0))
    g = SurRun(w, flat, norm, judge_stride=1)
    md.md_set_surrogate_ood(g.ctx, 1.5, 2.0, np.radians(2.0))
    s0 = g.snapshot()
    md.md_judge_reset(g.ctx)
    g.run(1)
    s1 = g.snapshot()
    j = md.md_judge_stats(g.ctx)
    g.close()
    ref, aero, fb, _ = _oracle_sur_step(w, s0, 0, flat, norm, ood=ood)
    assert fb.sum() > 40
    assert j["n_fallback"] == fb.sum()
    pu.assert_blocks(s1, ref, what="ood step")
