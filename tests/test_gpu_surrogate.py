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
    tol = _residual_bound(P, w["env_offsets"], s)
    err = np.max(np.abs(Y[:, :3] - Yr[:, :3]), axis=1)
    sc = np.maximum(np.max(np.abs(Yr[:, :3]), axis=1), 1e-3)
    print("%s: residual error / bound worst %.3f; bound relative to max(|F|, 1e-3 N): median %.2e, max %.2e"
          % (kind, np.max(err / tol), np.median(tol / sc), np.max(tol / sc)))
    assert np.all(np.isfinite(tol))
    assert np.all(err <= tol), np.argmax(err / tol)
    assert np.all(Y[:, 3:] == 0)


def _residual_bound(P, off, s):
    """Per drone, a bound on the float32 error of the body-frame residual force
    (absolute, N), each term weighted by its own magnitude (units of
    u = 2^-23, the float32 unit roundoff times 2):
      downwash pair j (Eq. 6), t_j = K1/dz^2 exp(-x_j), x_j = dxy^2/(2 beta^2):
        |t_j| (6 + (4 + 2 kappa_j) x_j) -- the factor 1/dz^2 and the product
        (a few roundings, the reciprocal), and the exponential, whose relative
        error is x_j times that of its argument (dxy^2 and 1/beta^2: a few
        roundings, and kappa_j = (|C2 dz| + |C3|) / |beta| for the
        cancellation in beta = C2 dz + C3 with rounded constants);
      the summation of the M - 1 terms in float32: (M / 2) sum |t_j|;
      ground effect, drag, the world force's components and the rotation into
        the body frame: 8 (|F_gnd| + |F_drag|_1 + sum |t_j|).
    Stored positions are the same float32 values on both sides, so dz, dxy
    and the gates are exact."""
    p = s["p"]
    n = int(off[-1])
    r_p = P.r_p
    K1 = P.C1 * r_p * r_p / 16.0
    wsum = np.zeros(n)   # sum |t_j| (6 + (4 + 2 kappa) x)
    tsum = np.zeros(n)   # sum |t_j|
    msz = np.zeros(n)
    for e in range(len(off) - 1):
        i0, i1 = int(off[e]), int(off[e + 1])
        if i1 - i0 < 2:
            continue
        dz = p[2, i0:i1][None, :] - p[2, i0:i1][:, None]
        dx = p[0, i0:i1][None, :] - p[0, i0:i1][:, None]
        dy = p[1, i0:i1][None, :] - p[1, i0:i1][:, None]
        d2 = dx * dx + dy * dy
        on = (dz > 0) & (d2 < 100)
        beta = P.C2 * dz + P.C3
        b2 = beta * beta
        with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
            x = np.where(on & (b2 > 0), d2 / (2 * b2), np.where(d2 > 0, np.inf, 0.0))
            t = np.where(on, K1 / np.where(on, dz * dz, 1.0) * np.exp(-x), 0.0)
            kappa = np.where(b2 > 0, (np.abs(P.C2 * dz) + abs(P.C3)) / np.sqrt(b2), 0.0)
            w_ = np.where(t > 0, t * (6.0 + (4.0 + 2.0 * kappa) * x), 0.0)
        wsum[i0:i1] = w_.sum(axis=1)
        tsum[i0:i1] = t.sum(axis=1)
        msz[i0:i1] = i1 - i0
    g = np.linalg.norm(orc.aero_residual(P, 1, off, s)[:, :3], axis=1)
    dr = np.sum(np.abs(orc.aero_residual(P, 2, off, s)[:, :3]), axis=1) * np.sqrt(3.0)
    u = 2.0 ** -23
    return u * (wsum + 0.5 * msz * tsum + 8.0 * (g + dr + tsum)) + 1e-30


@pytest.mark.parametrize("kind", ["lattice8", "formation", "ragged"])
def test_knn_lists_valid_against_exact_distances(kind):
    """The GPU's neighbour lists judged by exact FP64 horizontal distances,
    not by the binary32 recipe both sides share: per drone, min(8, M - 1)
    distinct same-environment neighbours other than itself, in ascending
    exact distance, every chosen one no farther than the exact 8th-nearest
    distance and every one left out no nearer, each up to float32 rounding of
    the squared distance (relative 2^-20, several times the few roundings of
    dx*dx + dy*dy)."""
    if kind == "lattice8":
        w = wl.subset_envs(wl.lattice(n_envs=16384, shape=(2, 2, 2), seed=3), 512)
    elif kind == "formation":
        w = wl.subset_envs(wl.formation(n_envs=8192, seed=4), 128)
    else:
        w = wl.ragged_grid(pu.hover_rpm(), n_envs=128, n_steps=3, seed=2)
    s32, _, _, nbr = _datagen(w, steps_before=3)
    p = s32["p"].astype(np.float64)
    off = w["env_offsets"]
    eps = 2.0 ** -20
    for e in range(len(off) - 1):
        i0, i1 = int(off[e]), int(off[e + 1])
        m = i1 - i0
        for i in range(i0, i1):
            d2 = (p[0, i0:i1] - p[0, i]) ** 2 + (p[1, i0:i1] - p[1, i]) ** 2
            d2[i - i0] = np.inf
            lst = nbr[i]
            k = min(8, m - 1)
            assert np.all(lst[k:] == -1), (i, lst)
            ch = lst[:k]
            assert len(set(ch.tolist())) == k and np.all((ch >= i0) & (ch < i1)) and i not in ch, (i, lst)
            dc = d2[ch - i0]
            assert np.all(dc[1:] >= dc[:-1] * (1 - eps)), (i, dc)
            if k == 0 or k == m - 1:
                continue
            d8 = np.sort(d2)[k - 1]
            assert np.all(dc <= d8 * (1 + eps)), (i, dc, d8)
            rest = np.setdiff1d(np.arange(i0, i1), np.append(ch, i)) - i0
            assert np.all(d2[rest] >= d8 * (1 - eps)), (i, d8)


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


def test_region_fallback_matches_oracle():
    """Drones with a neighbour inside the cylinder (|dz| < 0.6 m, lateral
    distance < 0.85 m) or more than 3 m away vertically take the plain terms
    on both sides (binary32 decisions on the stored positions), and the step
    matches the oracle."""
    rng = np.random.default_rng(54)
    flat, norm = _random_net(rng)
    w = wl.subset_envs(wl.lattice(n_envs=16384, shape=(2, 2, 2), seed=3), 128)
    st = {k: v.copy() for k, v in w["state"].items()}
    off = w["env_offsets"]
    for e in range(0, 128, 4):
        i0 = off[e]
        k = (e // 4) % 4
        st["p"][:, i0 + 1] = st["p"][:, i0] + np.array([[0.5, 0.2, 0.0], [0.1, 0.1, 0.4], [0.0, 0.3, -0.55],
                                                         [0.1, 0.0, -3.5]][k])
    w = dict(w, state=st)
    region = dict(near_dz=0.6, near_r=0.85, far_dz=3.0)
    g = SurRun(w, flat, norm, dz_ood=0.0, judge_stride=1)
    md.md_set_surrogate_region(g.ctx, **region)
    s0 = g.snapshot()
    md.md_judge_reset(g.ctx)
    g.run(1)
    s1 = g.snapshot()
    j = md.md_judge_stats(g.ctx)
    g.close()
    ref, aero, fb, _ = _oracle_sur_step(w, s0, 0, flat, norm, dz_ood=0.0, ood=region)
    assert fb.sum() >= 64
    assert j["n_fallback"] == fb.sum()
    pu.assert_blocks(s1, ref, what="region fallback step")


def _moving_formation(n_envs, shift, shape=None):
    """Formation environments (or lattices of `shape`) whose waypoints lie
    `shift` metres off in x and y, so that every drone flies off and the bins'
    candidate lists must be rebuilt along the way."""
    if shape is None:
        w = wl.subset_envs(wl.formation(n_envs=8192, seed=4), n_envs)
    else:
        w = wl.lattice(n_envs=n_envs, shape=shape, seed=5)
    w = dict(w)
    act = np.array(w["action"], copy=True)
    act[:, 0] += shift
    act[:, 1] -= 0.5 * shift
    w["action"] = act
    return w


@pytest.mark.parametrize("shift,shape", [(0.0, None), (1.5, None), (1.5, (16, 8, 2)), (1.5, (16, 16, 2))])
def test_knn_candidate_lists_equal_full_ranking_bitwise(shift, shape):
    """The surrogate step with candidate lists against the same step ranking
    every same-environment drone every step: bitwise equal state after 300
    steps; with the waypoints moved the lists are rebuilt on the way.  The
    formation has one-wave bins; 256- and 512-drone environments fill four-
    and eight-wave bins (more than 64 KB of LDS)."""
    rng = np.random.default_rng(53)
    flat, norm = _random_net(rng)
    w = _moving_formation(96 if shape is None else 4, shift, shape)
    out = {}
    for reuse in (True, False):
        g = SurRun(w, flat, norm, judge_stride=64)
        md.md_set_surrogate_knn_reuse(g.ctx, reuse)
        md.md_judge_reset(g.ctx)
        obs = g.run(300, obs_slots=300)
        out[reuse] = (g.snapshot(), obs, md.md_judge_stats(g.ctx))
        g.close()
    (a, oa, ja), (b, ob, jb) = out[True], out[False]
    for k in ("p", "q", "v", "w", "rpm", "pid_int"):
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)
    np.testing.assert_array_equal(oa, ob)
    n = int(w["env_offsets"][-1])
    assert jb["n_knn_full"] == n * 300
    moved = float(np.max(np.hypot(a["p"][0] - w["state"]["p"][0], a["p"][1] - w["state"]["p"][1])))
    print("shift %.1f: full rankings %d of %d drone-steps with lists (max lateral travel %.2f m)"
          % (shift, ja["n_knn_full"], n * 300, moved))
    assert ja["n_knn_full"] >= n  # the first step of the launch
    if shift > 0:
        assert ja["n_knn_full"] > n and ja["n_knn_full"] < n * 300 / 2
    else:
        assert ja["n_knn_full"] < n * 300 / 10
