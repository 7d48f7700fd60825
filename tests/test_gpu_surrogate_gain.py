"""What the learned residual gains over the method without it.

* The committed trained network on held-out samples (fresh seeds): its
  force error eps = sqrt(sum |F_hat - F|^2 / sum |F|^2) against the plain
  Eq. 4-6 residual, versus eps = 1 for the aero-free step (F_hat = 0).
* In-step: rollouts with the surrogate, with the plain terms and with no
  aerodynamic terms from one initial state; the surrogate trajectory must stay
  much closer to the plain one than the aero-free trajectory does.
* The training pipeline end to end on a small budget (data generation,
  forward/backward/Adam kernels) beats the aero-free baseline by a wide margin.
"""
import os

import numpy as np
import pytest

from paper_2606_08039_amd import md, surrogate, workloads as wl

pytestmark = pytest.mark.gpu

WEIGHTS = surrogate.DEFAULT_WEIGHTS


def _held_out():
    import torch
    X1, Y1 = surrogate.generate(512, (2, 2, 2), 4, 30, seed=133)
    X2, Y2 = surrogate.generate(128, (4, 4, 2), 4, 30, seed=134)
    return torch.cat([X1, X2]), torch.cat([Y1, Y2])


@pytest.mark.skipif(not os.path.exists(WEIGHTS), reason="no trained weights committed")
def test_trained_network_on_held_out_samples():
    import torch
    flat, norm, meta = surrogate.load(WEIGHTS)
    X, Y = _held_out()
    m = md.md_mlp_create(4096)
    md.md_mlp_set_params(m, flat)
    md.md_mlp_set_norm(m, norm)
    eps = surrogate.force_error(surrogate.predict(m, X), Y)
    md.md_mlp_destroy(m)
    eps_none = surrogate.force_error(torch.zeros_like(Y), Y)
    print("held-out force error: surrogate %.4f, no aero %.4f (training record %s)"
          % (eps, eps_none, meta.get("eps_held_out")))
    assert eps_none == pytest.approx(1.0)
    assert eps <= 0.02  # the <= 2 % residual-force error of the surrogate's contract


# Fallback bounds of the trained network's region (lattice flights: speeds
# below 1 m/s, neighbour relative speeds below 1.2 m/s, tilts below half a
# degree, column partners 0.8-1.45 m apart vertically, same-layer neighbours
# at least 0.9 m apart laterally), with margin: world speed 1.5 m/s, relative
# speed 2 m/s, tilt 2 degrees; a neighbour inside |dz| < 0.75 m, dxy < 0.85 m
# or beyond |dz| > 3 m; and the downwash singularity below 10 um.
DZ_OOD, OOD, REGION = 1e-5, (1.5, 2.0, float(np.radians(2.0))), (0.75, 0.85, 3.0)


def _rollout(w, mask, flat=None, norm=None, steps=480, warm=60):
    """steps PID steps from the workload's initial state; the judge counts
    the steps after the first `warm` (the start-up transient, whose first
    corrections drive rotor speeds outside the range the network was trained
    on, as the bench's warm-up launches do)."""
    import torch
    p = md.md_default_params_cf2x()
    ctx = md.md_create(p, w["dt"], mask, md.MD_ACT_PID, w["ctrl_decim"])
    md.md_bind_layout(ctx, w["env_offsets"])
    if mask & md.MD_AERO_SURROGATE:
        md.md_load_surrogate(ctx, flat, norm, DZ_OOD, 16)
        md.md_set_surrogate_ood(ctx, *OOD)
        md.md_set_surrogate_region(ctx, *REGION)
    st = md.DeviceState.from_numpy(w["state"])
    act = torch.from_numpy(w["action"]).cuda()
    md.md_step(ctx, st, act, False, None, 0, warm, 0)
    if mask & md.MD_AERO_SURROGATE:
        md.md_judge_reset(ctx)
    md.md_step(ctx, st, act, False, None, 0, steps - warm, warm)
    torch.cuda.synchronize()
    j = md.md_judge_stats(ctx) if mask & md.MD_AERO_SURROGATE else None
    md.md_destroy(ctx)
    return st.to_numpy(), j


@pytest.mark.skipif(not os.path.exists(WEIGHTS), reason="no trained weights committed")
def test_in_step_surrogate_tracks_the_plain_model():
    flat, norm, _ = surrogate.load(WEIGHTS)
    w = wl.subset_envs(wl.lattice(n_envs=16384, shape=(2, 2, 2), seed=233), 512)
    plain, _ = _rollout(w, 7)
    sur, judge = _rollout(w, md.MD_AERO_SURROGATE, flat, norm)
    none, _ = _rollout(w, 0)
    lower = w["state"]["p"][2] < np.median(w["state"]["p"][2])  # drones under a wake
    rms = lambda a: float(np.sqrt(np.mean(np.sum((a["p"] - plain["p"]) ** 2, axis=0)[lower])))
    e_sur, e_none = rms(sur), rms(none)
    print("2 s rollouts, RMS position gap to plain aero (lower layer): surrogate %.4g m, "
          "no aero %.4g m; judge eps %.4f over %d samples, %.2f %% of drone-steps on the fallback"
          % (e_sur, e_none, judge["force_rel_err"], judge["n_judged"],
             100.0 * judge["n_fallback"] / judge["n_drone_steps"]))
    assert e_sur < 0.2 * e_none
    assert judge["force_rel_err"] <= 0.02


def test_training_pipeline_beats_the_aero_free_baseline():
    import torch
    X, Y = surrogate.generate(256, (2, 2, 2), 16, 30, seed=333)  # 32768 samples
    Xh, Yh = surrogate.generate(64, (2, 2, 2), 4, 30, seed=334)
    norm = surrogate.fit_norm(X, Y)
    m, hist = surrogate.train(X, Y, norm, epochs=6, batch=1024, lr=3e-3, seed=1)
    eps = surrogate.force_error(surrogate.predict(m, Xh), Yh)
    md.md_mlp_destroy(m)
    print("small training run: held-out eps %.4f, losses %s" % (eps, [round(h["loss"], 5) for h in hist]))
    assert hist[-1]["loss"] < hist[0]["loss"]
    assert eps < 0.5
