"""Training-data generation, training and storage of the aerodynamic-residual
surrogate.  This module only sequences libmd calls (rollouts, sample
generation, forward/backward/Adam launches) and moves buffers; every
arithmetic step of the physics and of the network runs in libmd's kernels.

Data recipe (seeded): lattice workloads (2x2x2 and 4x4x2 lattices, lateral
pitch U[1.0,1.3] m, vertical pitch U[0.9,1.0] m, lower layer z ~ U[0.3,0.5],
PID waypoints = lattice point + U[-0.05,0.05]^3, start = waypoint +
U[-0.1,0.1]^3) are flown by the plain model (ground effect + drag +
downwash, PID every 5 steps); every `every` steps the waypoints are drawn
again and one sample per drone is taken: 60 features and the body-frame
residual of Eq. 4-6.

Weights file: a little-endian binary with magic b"MDSURR01", a uint32 JSON
header length, the JSON header (shape, training record), then float32
parameters [42118] and normalisation [140].
"""
import json
import math
import os
import struct
import time

import numpy as np

from . import md, workloads as wl

MAGIC = b"MDSURR01"
HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "weights", "surrogate_cf2x_v1.bin")


def generate(n_envs, shape, snapshots, every, seed, warmup_steps=60, device="cuda"):
    """Samples (X [S*N][64], Y [S*N][6]) as CUDA float32 tensors."""
    import torch
    w = wl.lattice(n_envs=n_envs, shape=shape, n_steps=every, seed=seed)
    rng = np.random.default_rng(seed + 1000)
    p = md.md_default_params_cf2x()
    ctx = md.md_create(p, w["dt"], 7, md.MD_ACT_PID, w["ctrl_decim"])
    try:
        md.md_bind_layout(ctx, w["env_offsets"])
        st = md.DeviceState.from_numpy(w["state"], device)
        n = st.n
        X = torch.empty((snapshots * n, 64), dtype=torch.float32, device=device)
        Y = torch.empty((snapshots * n, 6), dtype=torch.float32, device=device)
        tgt = torch.from_numpy(w["action"]).to(device)
        step = 0
        if warmup_steps:
            md.md_step(ctx, st, tgt, False, None, 0, warmup_steps, step)
            step += warmup_steps
        for k in range(snapshots):
            tgt = torch.from_numpy(wl.rejitter_targets(w, rng)).to(device)
            md.md_step(ctx, st, tgt, False, None, 0, every, step)
            step += every
            md.md_datagen(ctx, st, 7, X[k * n:(k + 1) * n], Y[k * n:(k + 1) * n])
        torch.cuda.synchronize()
    finally:
        md.md_destroy(ctx)
    return X, Y


def dataset(total_log2=22, seed=3, every=30, device="cuda"):
    """Half the samples from 2x2x2 lattices, half from 4x4x2 lattices."""
    import torch
    half = 1 << (total_log2 - 1)
    parts = []
    for shape, s in (((2, 2, 2), seed), ((4, 4, 2), seed + 1)):
        m = shape[0] * shape[1] * shape[2]
        snaps = 32 if half >= 32 * m else max(1, half // m)
        n_envs = max(1, half // (snaps * m))
        parts.append(generate(n_envs, shape, snaps, every, s, device=device))
    X = torch.cat([p[0] for p in parts])
    Y = torch.cat([p[1] for p in parts])
    return X, Y


def fit_norm(X, Y, max_rows=1 << 18):
    """Per-feature standardisation (mean, 1/std; constant features get 1) and
    per-output scales (std, floored at 1e-6 of the largest force scale),
    estimated on the host from an evenly strided subsample of the data."""
    stride = max(1, X.shape[0] // max_rows)
    x = X[::stride].cpu().numpy().astype(np.float64)
    y = Y[::stride].cpu().numpy().astype(np.float64)
    xm, xs = x.mean(0), x.std(0)
    xinv = np.where(xs > 1e-8, 1.0 / np.maximum(xs, 1e-8), 1.0)
    ym, ys = y.mean(0), y.std(0)
    floor = 1e-6 * max(float(ys[:3].max()), 1e-12)
    ys = np.where(ys > floor, ys, floor)
    return np.concatenate([xm, xinv, ym, ys]).astype(np.float32)


def init_params(seed):
    rng = np.random.default_rng(seed)
    parts = []
    for sh in md.MLP_SHAPES:
        if len(sh) == 2:
            parts.append(rng.normal(size=sh) * math.sqrt(2.0 / sh[1]))
        else:
            parts.append(np.zeros(sh))
    return md.mlp_flatten(parts)


def train(X, Y, norm, epochs=20, batch=4096, lr=2e-3, lr_final=2e-5, seed=0, log=None):
    """Adam on the mean squared standardised error; cosine learning-rate
    decay.  Returns (md_mlp handle, history)."""
    import torch
    N = X.shape[0]
    m = md.md_mlp_create(max(batch, 4096))  # predict() runs batches of 4096
    md.md_mlp_set_params(m, init_params(seed))
    md.md_mlp_set_norm(m, norm)
    gen = torch.Generator(device=X.device)
    gen.manual_seed(seed)
    steps_per_epoch = N // batch
    total = epochs * steps_per_epoch
    hist = []
    it = 0
    t0 = time.time()
    for ep in range(epochs):
        perm = torch.randperm(N, device=X.device, generator=gen)
        Xp, Yp = X[perm], Y[perm]
        for b in range(steps_per_epoch):
            cur = lr_final + 0.5 * (lr - lr_final) * (1 + math.cos(math.pi * it / max(1, total)))
            xb = Xp[b * batch:(b + 1) * batch]
            yb = Yp[b * batch:(b + 1) * batch]
            md.md_mlp_forward(m, xb)
            md.md_mlp_backward(m, yb)
            md.md_mlp_adam(m, cur)
            it += 1
        loss = md.md_mlp_loss(m)
        hist.append({"epoch": ep, "loss": loss, "lr": cur, "seconds": time.time() - t0})
        if log:
            log("epoch %d loss %.4e lr %.2e (%.1fs)" % (ep, loss, cur, time.time() - t0))
    return m, hist


def predict(m, X, batch=None):
    """Network outputs (de-standardised) for X through the training forward."""
    import torch
    B = batch or 4096
    Y = torch.empty((X.shape[0], 6), dtype=torch.float32, device=X.device)
    for o in range(0, X.shape[0], B):
        nb = min(B, X.shape[0] - o)
        md.md_mlp_forward(m, X[o:o + nb], nb, Y[o:o + nb])
    torch.cuda.synchronize()
    return Y


def force_error(Yhat, Y):
    """eps = sqrt(sum |F_hat - F|^2 / sum |F|^2) over the force block."""
    d = (Yhat[:, :3] - Y[:, :3]).double()
    return float(d.pow(2).sum().sqrt() / Y[:, :3].double().pow(2).sum().sqrt())


def save(path, flat, norm, meta):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    hdr = json.dumps(dict(meta, n_params=md.MLP_NPARAMS, n_norm=md.MLP_NORM,
                          layers=[64, 128, 128, 128, 6], activation="silu")).encode()
    with open(path, "wb") as f:
        f.write(MAGIC)
        f.write(struct.pack("<I", len(hdr)))
        f.write(hdr)
        f.write(np.asarray(flat, dtype="<f4").tobytes())
        f.write(np.asarray(norm, dtype="<f4").tobytes())


def load(path=DEFAULT_WEIGHTS):
    with open(path, "rb") as f:
        if f.read(8) != MAGIC:
            raise ValueError("not a surrogate weights file: " + path)
        (hl,) = struct.unpack("<I", f.read(4))
        meta = json.loads(f.read(hl).decode())
        flat = np.frombuffer(f.read(4 * md.MLP_NPARAMS), dtype="<f4").astype(np.float32)
        norm = np.frombuffer(f.read(4 * md.MLP_NORM), dtype="<f4").astype(np.float32)
    if flat.size != md.MLP_NPARAMS or norm.size != md.MLP_NORM:
        raise ValueError("truncated surrogate weights file: " + path)
    return flat, norm, meta


def main():
    import argparse
    ap = argparse.ArgumentParser(description="generate data, train and store the surrogate")
    ap.add_argument("--log2-samples", type=int, default=22)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    args = ap.parse_args()
    import torch
    t0 = time.time()
    X, Y = dataset(args.log2_samples, seed=3)
    Xh, Yh = dataset(args.log2_samples - 4, seed=33)
    print("data: %d train / %d held-out samples in %.1fs" % (X.shape[0], Xh.shape[0], time.time() - t0),
          flush=True)
    norm = fit_norm(X, Y)
    m, hist = train(X, Y, norm, epochs=args.epochs, batch=args.batch, lr=args.lr,
                    log=lambda s: print(s, flush=True))
    eps_train = force_error(predict(m, X[: 1 << 18]), Y[: 1 << 18])
    eps_held = force_error(predict(m, Xh), Yh)
    eps_zero = force_error(torch.zeros_like(Yh), Yh)
    flat = md.md_mlp_get_params(m)
    meta = {"samples": int(X.shape[0]), "held_out": int(Xh.shape[0]), "epochs": args.epochs,
            "batch": args.batch, "lr": args.lr, "eps_train": eps_train, "eps_held_out": eps_held,
            "eps_no_aero": eps_zero, "history": hist}
    save(args.out, flat, norm, meta)
    md.md_mlp_destroy(m)
    print(json.dumps({"eps_train": eps_train, "eps_held_out": eps_held, "eps_no_aero": eps_zero,
                      "out": args.out, "seconds": time.time() - t0}), flush=True)


if __name__ == "__main__":
    main()
