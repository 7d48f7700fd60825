"""Pins of the oracle's surrogate support: neighbour search against a brute
force sort, features against library rotations, the MLP forward/backward
against PyTorch float64 autograd and central finite differences, Adam against
torch.optim.Adam, bfloat16 rounding against PyTorch's conversion."""
import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation

import oracle as orc


def _env_positions(rng, sizes):
    off = np.zeros(len(sizes) + 1, dtype=np.int32)
    off[1:] = np.cumsum(sizes)
    p = rng.uniform(-1, 1, size=(3, off[-1])).astype(np.float32).astype(np.float64)
    return off, p


def test_knn_matches_brute_force_sort():
    rng = np.random.default_rng(30)
    off, p = _env_positions(rng, [1, 2, 5, 9, 12, 33])
    # plant exact ties: two drones at the same offset from a third
    p[:, 10] = p[:, 9] + [0.25, 0, 0]
    p[:, 11] = p[:, 9] + [-0.25, 0, 0]
    # a drone straight above another is its nearest neighbour whatever the height
    p[:, 20] = p[:, 19] + [1e-3, 0, 0.9]
    nbr = orc.knn(off, p, 8)
    pf = p.astype(np.float32)
    for e in range(len(off) - 1):
        for i in range(off[e], off[e + 1]):
            js = np.array([j for j in range(off[e], off[e + 1]) if j != i], dtype=np.int64)
            d = pf[:, js] - pf[:, [i]]
            d2 = d[0] * d[0] + d[1] * d[1]  # horizontal, float32
            assert d2.dtype == np.float32
            order = js[np.lexsort((js, d2))][:8]
            expect = np.full(8, -1)
            expect[: len(order)] = order
            np.testing.assert_array_equal(nbr[i], expect)
    assert nbr[9][0] == 10 and nbr[9][1] == 11  # tie broken to the lower index
    assert nbr[19][0] == 20 and nbr[20][0] == 19


def test_features_match_library_rotations():
    rng = np.random.default_rng(31)
    P = orc.cf2x()
    D = orc.derive(P)
    off, p = _env_positions(rng, [3, 10])
    n = off[-1]
    s = orc.new_state(n)
    s["p"][:] = p
    rots = Rotation.random(n, random_state=rng)
    xyzw = rots.as_quat()
    s["q"][:] = np.stack([xyzw[:, 3], xyzw[:, 0], xyzw[:, 1], xyzw[:, 2]])
    s["v"][:] = rng.normal(size=(3, n))
    s["rpm"][:] = rng.uniform(10000, 20000, size=(4, n))
    nbr = orc.knn(off, p, 8)
    X = orc.features(P, off, s, nbr)
    assert X.shape == (n, 64)
    np.testing.assert_allclose(X[:, 0:3], rots.inv().apply(s["v"].T), atol=1e-12)
    np.testing.assert_allclose(X[:, 3:6], rots.inv().apply([0, 0, 1]), atol=1e-12)
    np.testing.assert_allclose(X[:, 6:10], s["rpm"].T / D.hover_rpm, rtol=1e-15)
    for i in range(n):
        for t in range(8):
            j = nbr[i, t]
            blk = X[i, 10 + 6 * t: 16 + 6 * t]
            if j < 0:
                assert np.all(blk == 0)
            else:
                np.testing.assert_allclose(blk[:3], p[:, j] - p[:, i], rtol=1e-15)
                np.testing.assert_allclose(blk[3:], s["v"][:, j] - s["v"][:, i], rtol=1e-15)
    np.testing.assert_array_equal(X[:, 58], p[2])
    # ground proximity: 1 at or below the clip height, (h_clip / z)^2 above
    np.testing.assert_allclose(X[:, 59], np.minimum(1.0, (D.h_clip / p[2]) ** 2) * (p[2] > 0)
                               + (p[2] <= 0), rtol=1e-15)
    assert np.all(X[:, 60:] == 0)


def test_aero_residual_is_body_frame_sum_of_terms():
    rng = np.random.default_rng(32)
    P = orc.cf2x()
    off, p = _env_positions(rng, [4])
    p[2] += 1.5
    s = orc.new_state(4)
    s["p"][:] = p
    rots = Rotation.random(4, random_state=rng)
    xyzw = rots.as_quat()
    s["q"][:] = np.stack([xyzw[:, 3], xyzw[:, 0], xyzw[:, 1], xyzw[:, 2]])
    s["v"][:] = rng.normal(size=(3, 4))
    rpm = rng.uniform(10000, 20000, size=(4, 4))
    mask = orc.AERO_GND | orc.AERO_DRAG | orc.AERO_DW
    Y = orc.aero_residual(P, mask, off, s, rpm)
    for i in range(4):
        Fw = orc.drag(P, rpm[:, i], s["q"][:, i], s["v"][:, i])
        Fw[2] += orc.ground_effect(P, rpm[:, i], p[2, i], s["q"][:, i])
        for j in range(4):
            if j != i:
                Fw[2] += orc.downwash_pair(P, p[:, i], p[:, j])
        np.testing.assert_allclose(Y[i, :3], rots[i].inv().apply(Fw), rtol=1e-10, atol=1e-18)
        assert np.all(Y[i, 3:] == 0)


def _net(rng, dims):
    Ws = [rng.normal(size=(dims[l + 1], dims[l])) / np.sqrt(dims[l]) for l in range(len(dims) - 1)]
    bs = [rng.normal(size=dims[l + 1]) * 0.1 for l in range(len(dims) - 1)]
    return Ws, bs


def _torch_net(Ws, bs):
    layers = []
    for l, (W, b) in enumerate(zip(Ws, bs)):
        lin = torch.nn.Linear(W.shape[1], W.shape[0]).double()
        with torch.no_grad():
            lin.weight.copy_(torch.from_numpy(W))
            lin.bias.copy_(torch.from_numpy(b))
        layers.append(lin)
        if l < len(Ws) - 1:
            layers.append(torch.nn.SiLU())
    return torch.nn.Sequential(*layers)


def test_mlp_forward_backward_match_torch_float64():
    rng = np.random.default_rng(33)
    dims = [64, 128, 128, 128, 6]
    Ws, bs = _net(rng, dims)
    X = rng.normal(size=(37, 64))
    dY = rng.normal(size=(37, 6))
    Y, acts = orc.mlp_forward(Ws, bs, X)
    net = _torch_net(Ws, bs)
    xt = torch.from_numpy(X).requires_grad_(True)
    yt = net(xt)
    np.testing.assert_allclose(Y, yt.detach().numpy(), rtol=1e-12, atol=1e-13)
    yt.backward(torch.from_numpy(dY))
    dWs, dbs, dX = orc.mlp_backward(Ws, bs, X, acts, dY, want_dx=True)
    lins = [m for m in net if isinstance(m, torch.nn.Linear)]
    for l, lin in enumerate(lins):
        np.testing.assert_allclose(dWs[l], lin.weight.grad.numpy(), rtol=1e-10, atol=1e-12)
        np.testing.assert_allclose(dbs[l], lin.bias.grad.numpy(), rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(dX, xt.grad.numpy(), rtol=1e-10, atol=1e-12)


def test_mlp_backward_matches_central_differences():
    rng = np.random.default_rng(34)
    dims = [7, 9, 8, 3]
    Ws, bs = _net(rng, dims)
    X = rng.normal(size=(5, 7))
    dY = rng.normal(size=(5, 3))
    loss = lambda Ws_, bs_: float(np.sum(orc.mlp_forward(Ws_, bs_, X)[0] * dY))
    _, acts = orc.mlp_forward(Ws, bs, X)
    dWs, dbs, _ = orc.mlp_backward(Ws, bs, X, acts, dY)
    h = 1e-6
    for l in range(len(Ws)):
        for (o, c) in [(0, 0), (1, 2), (dims[l + 1] - 1, dims[l] - 1)]:
            Wp = [W.copy() for W in Ws]
            Wm = [W.copy() for W in Ws]
            Wp[l][o, c] += h
            Wm[l][o, c] -= h
            fd = (loss(Wp, bs) - loss(Wm, bs)) / (2 * h)
            assert dWs[l][o, c] == pytest.approx(fd, rel=1e-6, abs=1e-9)
        bp = [b.copy() for b in bs]
        bm = [b.copy() for b in bs]
        bp[l][1] += h
        bm[l][1] -= h
        fd = (loss(Ws, bp) - loss(Ws, bm)) / (2 * h)
        assert dbs[l][1] == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_adam_matches_torch():
    rng = np.random.default_rng(35)
    w0 = rng.normal(size=50)
    grads = [rng.normal(size=50) for _ in range(4)]
    wt = torch.nn.Parameter(torch.from_numpy(w0.copy()))
    opt = torch.optim.Adam([wt], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    w, m1, m2 = w0.copy(), np.zeros(50), np.zeros(50)
    for t, g in enumerate(grads, start=1):
        wt.grad = torch.from_numpy(g.copy())
        opt.step()
        orc.adam(w, g.copy(), m1, m2, 1e-2, 0.9, 0.999, 1e-8, t)
    np.testing.assert_allclose(w, wt.detach().numpy(), rtol=1e-13, atol=1e-15)


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(36)
    x = rng.normal(size=2000).astype(np.float32) * np.exp(rng.uniform(-20, 20, 2000)).astype(np.float32)
    # exact ties between two bfloat16 values
    ties = np.array([1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -3.0 - 2 ** -7], dtype=np.float32)
    x = np.concatenate([x, ties])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(orc.bf16_round(x.astype(np.float64)), ref)


def test_bf16_forward_rounds_input_and_hidden_only():
    rng = np.random.default_rng(37)
    Ws, bs = _net(rng, [5, 6, 2])
    X = rng.normal(size=(3, 5))
    Y, acts = orc.mlp_forward(Ws, bs, X, bf16_acts=True)
    Xr = orc.bf16_round(X)
    z1 = Xr @ Ws[0].T + bs[0]
    h1 = orc.bf16_round(z1 / (1 + np.exp(-z1)))
    np.testing.assert_allclose(Y, h1 @ Ws[1].T + bs[1], rtol=1e-13)


def _lattice_pair_state(dz_low):
    """Two envs: a stacked pair (lower drone dz_low below the upper one) and a
    lone drone; level, at rest."""
    s = orc.new_state(3)
    s["p"][:, 0] = [0.0, 0.0, 1.0]
    s["p"][:, 1] = [0.05, 0.0, 1.0 + dz_low]
    s["p"][:, 2] = [3.0, 1.0, 0.7]
    s["v"][:, 0] = [0.1, -0.2, 0.05]
    return s, np.array([0, 2, 3], dtype=np.int32)


def _flat_zero():
    return np.zeros(42118, dtype=np.float32)


def _norm_identity():
    return np.concatenate([np.zeros(64), np.ones(64), np.zeros(6), np.ones(6)]).astype(np.float32)


def test_surrogate_step_with_zero_network_is_the_aero_free_step():
    P = orc.cf2x()
    D = orc.derive(P)
    rng = np.random.default_rng(38)
    s1, off = _lattice_pair_state(0.9)
    s2 = {k: v.copy() for k, v in s1.items()}
    act = (D.hover_rpm * (1 + rng.uniform(-0.05, 0.05, size=(5, 4, 3))))
    net, keep = orc.make_net(_flat_zero(), _norm_identity(), 1e-3)
    orc.step_surrogate(P, 1 / 240, orc.ACT_RPM, 1, off, s1, act, True, 5, net)
    orc.step(P, 1 / 240, 0, orc.ACT_RPM, 1, off, s2, act, True, 5)
    for k in s1:
        np.testing.assert_array_equal(s1[k], s2[k])


def test_surrogate_step_constant_body_force_closed_form():
    # W = 0, output bias b4 -> constant standardised output; body force
    # y = b4 * y_std + y_mean on a level hovering drone changes v by dt F / m.
    P = orc.cf2x()
    D = orc.derive(P)
    flat = _flat_zero()
    flat[42112:42118] = [0.5, -1.0, 2.0, 0.0, 0.0, 0.0]
    norm = _norm_identity()
    norm[134:140] = [0.01, 0.01, 0.01, 1.0, 1.0, 1.0]
    norm[128:131] = [0.001, 0.0, -0.002]
    s = orc.new_state(1)
    s["p"][:, 0] = [0, 0, 1]
    net, keep = orc.make_net(flat, norm, 1e-3)
    act = np.full((1, 4, 1), D.hover_rpm)
    _, aero, fb = orc.step_surrogate(P, 1 / 240, orc.ACT_RPM, 1, [0, 1], s, act, False, 1, net)
    f32 = lambda x: float(np.float32(x))
    F = np.array([0.5 * f32(0.01) + f32(0.001), -1.0 * f32(0.01), 2.0 * f32(0.01) + f32(-0.002)])
    np.testing.assert_allclose(aero[0, :3], F, rtol=1e-12)
    np.testing.assert_allclose(s["v"][:, 0], F / P.m / 240, rtol=1e-9, atol=1e-15)
    assert fb[0] == 0


def test_surrogate_fallback_takes_the_plain_terms():
    P = orc.cf2x()
    D = orc.derive(P)
    s, off = _lattice_pair_state(4e-4)  # drone 1 sits 0.4 mm above drone 0
    s_ref = {k: v.copy() for k, v in s.items()}
    net, keep = orc.make_net(_flat_zero(), _norm_identity(), 1e-3)
    act = np.full((1, 4, 3), D.hover_rpm)
    _, aero, fb = orc.step_surrogate(P, 1 / 240, orc.ACT_RPM, 1, off, s, act, False, 1, net)
    assert list(fb) == [1, 0, 0]
    Y = orc.aero_residual(P, 7, off, s_ref, rpm=np.full((4, 3), D.hover_rpm))
    np.testing.assert_allclose(aero[0], Y[0], rtol=1e-12)
    assert aero[0, 2] < -1.0  # the singular downwash is large here
    # the fallback drone's step equals the plain full-aero step
    orc.step(P, 1 / 240, 7, orc.ACT_RPM, 1, off, s_ref, act, False, 1)
    for k in ("p", "v", "w", "q"):
        np.testing.assert_allclose(s[k][:, 0], s_ref[k][:, 0], rtol=1e-12, atol=1e-15)


def test_out_of_distribution_fallback_checks():
    """Each optional check sends exactly the drones beyond its threshold to the
    plain terms: a fast drone (speed), a drone whose neighbour moves fast
    relative to it (relative speed, both members of the pair), a tilted drone
    (tilt), with the thresholds just above and below the values."""
    P = orc.cf2x()
    D = orc.derive(P)
    s0, off = _lattice_pair_state(0.9)
    s0["v"][:, 0] = [1.6, 0.0, 0.0]         # drone 0: 1.6 m/s, 1.6 m/s relative to drone 1
    th = np.radians(3.0)                    # drone 2: tilted 3 degrees about x
    s0["q"][:, 2] = [np.cos(th / 2), np.sin(th / 2), 0.0, 0.0]
    act = np.full((1, 4, 3), D.hover_rpm)
    cases = [(dict(ood_speed=1.5), [1, 0, 0]), (dict(ood_speed=1.7), [0, 0, 0]),
             (dict(ood_rel_speed=1.5), [1, 1, 0]), (dict(ood_rel_speed=1.7), [0, 0, 0]),
             (dict(ood_tilt=np.radians(2.9)), [0, 0, 1]), (dict(ood_tilt=np.radians(3.1)), [0, 0, 0])]
    for kw, expect in cases:
        s = {k: v.copy() for k, v in s0.items()}
        net, keep = orc.make_net(_flat_zero(), _norm_identity(), 1e-3, **kw)
        _, aero, fb = orc.step_surrogate(P, 1 / 240, orc.ACT_RPM, 1, off, s, act, False, 1, net)
        assert list(fb) == expect, (kw, list(fb))
        Y = orc.aero_residual(P, 7, off, s0, rpm=np.full((4, 3), D.hover_rpm))
        for i in range(3):
            if expect[i]:
                np.testing.assert_allclose(aero[i], Y[i], rtol=1e-12, atol=1e-18)
            else:
                np.testing.assert_array_equal(aero[i], 0.0)


def test_region_fallback_checks():
    """The region fallback sends exactly the drones with a neighbour (among
    their 8 nearest) inside the cylinder |dz| < near_dz, dxy < near_r, above
    or below, or beyond |dz| > far_dz, to the plain terms: checked against the
    rule evaluated directly on the neighbour lists, on random environments
    with pairs placed just inside and just outside each bound."""
    P = orc.cf2x()
    D = orc.derive(P)
    rng = np.random.default_rng(71)
    sizes = [6] * 40
    off, p = _env_positions(rng, sizes)
    p *= 2.0
    n = int(off[-1])
    near_dz, near_r, far_dz = 0.6, 0.85, 3.0
    # for each environment: drone 1 relative to drone 0 just inside / outside
    for e in range(40):
        i0 = off[e]
        kind = e % 5
        dx = {0: 0.80, 1: 0.90, 2: 0.30, 3: 0.30, 4: 0.20}[kind]
        dz = {0: 0.30, 1: 0.30, 2: 0.59, 3: -0.61, 4: -3.2}[kind]
        p[:, i0 + 1] = p[:, i0] + np.array([dx, 0.0, dz])
    p = p.astype(np.float32).astype(np.float64)
    s = {"p": p, "q": np.tile([[1.0], [0.0], [0.0], [0.0]], (1, n)), "v": np.zeros((3, n)),
         "w": np.zeros((3, n)), "rpm": np.full((4, n), D.hover_rpm), "pid_int": np.zeros((6, n))}
    nbr = orc.knn(off, p, 8)
    p32 = p.astype(np.float32)
    expect = np.zeros(n, dtype=bool)
    for i in range(n):
        for j in nbr[i]:
            if j < 0:
                continue
            dz = np.float32(p32[2, j] - p32[2, i])
            ddx, ddy = np.float32(p32[0, j] - p32[0, i]), np.float32(p32[1, j] - p32[1, i])
            d2 = np.float32(np.float32(ddx * ddx) + np.float32(ddy * ddy))
            if (abs(dz) < np.float32(near_dz) and d2 < np.float32(near_r * near_r)) or abs(dz) > np.float32(far_dz):
                expect[i] = True
    assert 10 < expect.sum() < n - 10
    act = np.full((1, 4, n), D.hover_rpm)
    net, keep = orc.make_net(_flat_zero(), _norm_identity(), 0.0, near_dz=near_dz, near_r=near_r, far_dz=far_dz)
    _, aero, fb = orc.step_surrogate(P, 1 / 240, orc.ACT_RPM, 1, off, {k: v.copy() for k, v in s.items()},
                                     act, False, 1, net)
    np.testing.assert_array_equal(fb.astype(bool), expect)
    # each bound off: no region fallback
    net0, keep0 = orc.make_net(_flat_zero(), _norm_identity(), 0.0)
    _, _, fb0 = orc.step_surrogate(P, 1 / 240, orc.ACT_RPM, 1, off, {k: v.copy() for k, v in s.items()},
                                   act, False, 1, net0)
    assert fb0.sum() == 0
