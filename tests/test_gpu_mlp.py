"""GPU parity of the surrogate network's training kernels (BF16 MFMA forward,
backward, Adam) against the FP64 oracle network evaluated on the same
bfloat16-rounded weights and inputs."""
import numpy as np
import pytest

import oracle as orc
from paper_2606_08039_amd import md

pytestmark = pytest.mark.gpu


def _init(rng):
    parts = []
    for sh in md.MLP_SHAPES:
        if len(sh) == 2:
            parts.append(rng.normal(size=sh) * np.sqrt(2.0 / sh[1]))
        else:
            parts.append(rng.normal(size=sh) * 0.1)
    return md.mlp_flatten(parts)


def _norm(rng):
    xm = rng.normal(size=64) * 0.3
    xs = rng.uniform(0.5, 3.0, size=64)
    ym = rng.normal(size=6) * 0.01
    ys = rng.uniform(0.01, 0.1, size=6)
    return np.concatenate([xm, xs, ym, ys]).astype(np.float32)


def _oracle_forward(flat, norm, X):
    parts = md.mlp_unflatten(flat.astype(np.float64))
    Ws = [orc.bf16_round(parts[2 * l]) for l in range(4)]
    bs = [parts[2 * l + 1] for l in range(4)]
    xs = (X.astype(np.float64) - norm[:64].astype(np.float64)) * norm[64:128].astype(np.float64)
    Ystd, acts = orc.mlp_forward(Ws, bs, xs, bf16_acts=True)
    Y = Ystd * norm[134:140].astype(np.float64) + norm[128:134].astype(np.float64)
    return Y, Ystd, acts, Ws, bs, orc.bf16_round(xs)


def _data(rng, B):
    X = rng.normal(size=(B, 64)).astype(np.float32)
    X[:, 59:] = 0.0
    T = (rng.normal(size=(B, 6)) * 0.05).astype(np.float32)
    return X, T


def _gpu(flat, norm, X, T=None, max_batch=None):
    import torch
    m = md.md_mlp_create(max_batch or X.shape[0])
    md.md_mlp_set_params(m, flat)
    md.md_mlp_set_norm(m, norm)
    Xd = torch.from_numpy(X).cuda()
    Yd = torch.zeros((X.shape[0], 6), device="cuda")
    md.md_mlp_forward(m, Xd, Y=Yd)
    out = {"Y": None, "grads": None, "loss": None, "m": m}
    if T is not None:
        Td = torch.from_numpy(T).cuda()
        md.md_mlp_backward(m, Td)
        out["grads"] = md.md_mlp_get_grads(m)
        out["loss"] = md.md_mlp_loss(m)
        out["Td"] = Td
    torch.cuda.synchronize()
    out["Y"] = Yd.cpu().numpy()
    out["Xd"] = Xd
    return out


def test_forward_matches_oracle():
    rng = np.random.default_rng(40)
    flat, norm = _init(rng), _norm(rng)
    X, _ = _data(rng, 1000)  # ragged: not a multiple of the 64-row tile
    g = _gpu(flat, norm, X)
    md.md_mlp_destroy(g["m"])
    Y, Ystd, _, _, _, _ = _oracle_forward(flat, norm, X)
    ys = norm[134:140]
    e = (g["Y"] - Y) / ys  # in standardised units
    rel = np.linalg.norm(e) / np.linalg.norm(Ystd)
    print("forward: relative error %.2e, max abs (std units) %.2e" % (rel, np.abs(e).max()))
    assert rel < 2e-3 and np.abs(e).max() < 2e-2


def test_backward_matches_oracle_per_layer():
    rng = np.random.default_rng(41)
    flat, norm = _init(rng), _norm(rng)
    X, T = _data(rng, 777)
    g = _gpu(flat, norm, X, T)
    md.md_mlp_destroy(g["m"])
    Y, Ystd, acts, Ws, bs, Xused = _oracle_forward(flat, norm, X)
    Tstd = (T.astype(np.float64) - norm[128:134]) / norm[134:140]
    B = X.shape[0]
    dY = 2.0 * (Ystd - Tstd) / (B * 6)
    dWs, dbs, _ = orc.mlp_backward(Ws, bs, Xused, acts, dY)
    ref = md.mlp_flatten([x for pair in zip(dWs, dbs) for x in pair]).astype(np.float64)
    got = md.mlp_unflatten(g["grads"].astype(np.float64))
    refp = md.mlp_unflatten(ref)
    for i, (a, b) in enumerate(zip(got, refp)):
        rel = np.linalg.norm(a - b) / np.linalg.norm(b)
        print("grad block %d: relative error %.2e" % (i, rel))
        assert rel <= 2e-2, i
    loss_ref = np.mean((Ystd - Tstd) ** 2)
    assert g["loss"] == pytest.approx(loss_ref, rel=1e-2)


def test_backward_is_deterministic():
    rng = np.random.default_rng(42)
    flat, norm = _init(rng), _norm(rng)
    X, T = _data(rng, 3000)
    g1 = _gpu(flat, norm, X, T)
    g2 = _gpu(flat, norm, X, T)
    md.md_mlp_destroy(g1["m"])
    md.md_mlp_destroy(g2["m"])
    np.testing.assert_array_equal(g1["grads"], g2["grads"])


def test_adam_step_matches_oracle():
    rng = np.random.default_rng(43)
    flat, norm = _init(rng), _norm(rng)
    X, T = _data(rng, 512)
    g = _gpu(flat, norm, X, T)
    m = g["m"]
    p = flat.astype(np.float64).copy()
    m1, m2 = np.zeros_like(p), np.zeros_like(p)
    for t in (1, 2, 3):
        grads = md.md_mlp_get_grads(m).astype(np.float64)
        md.md_mlp_adam(m, 1e-3, 0.9, 0.999, 1e-8)
        orc.adam(p, grads, m1, m2, 1e-3, 0.9, 0.999, 1e-8, t)
        got = md.md_mlp_get_params(m).astype(np.float64)
        np.testing.assert_allclose(got, p, rtol=1e-5, atol=1e-7)
        # next gradients from the updated weights
        md.md_mlp_forward(m, g["Xd"])
        md.md_mlp_backward(m, g["Td"])
    md.md_mlp_destroy(m)


def test_training_fits_a_smooth_target():
    import torch
    rng = np.random.default_rng(44)
    B, N = 1024, 16384
    X = rng.normal(size=(N, 64)).astype(np.float32)
    X[:, 59:] = 0
    Wt = rng.normal(size=(64, 6)) / 8
    T = np.tanh(X @ Wt).astype(np.float32) * 0.1
    norm = np.concatenate([np.zeros(64), np.ones(64), np.zeros(6),
                           np.full(6, 0.1)]).astype(np.float32)
    m = md.md_mlp_create(B)
    md.md_mlp_set_params(m, _init(rng) * 0.5)
    md.md_mlp_set_norm(m, norm)
    Xd, Td = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    losses = []
    for it in range(400):
        o = (it * B) % N
        md.md_mlp_forward(m, Xd[o:o + B])
        md.md_mlp_backward(m, Td[o:o + B])
        md.md_mlp_adam(m, 2e-3)
        if it % 50 == 0 or it == 399:
            losses.append(md.md_mlp_loss(m))
    md.md_mlp_destroy(m)
    print("training losses:", losses)
    assert losses[-1] < 0.1 * losses[0]


def test_forward_rejects_oversized_batch():
    import torch
    m = md.md_mlp_create(16)
    X = torch.zeros((32, 64), device="cuda")
    with pytest.raises(md.MdError):
        md.md_mlp_forward(m, X)
    with pytest.raises(md.MdError):
        md.md_mlp_backward(m, torch.zeros((16, 6), device="cuda"))
    md.md_mlp_destroy(m)
