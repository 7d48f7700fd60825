#!/usr/bin/env python3
"""Throughput of the batched explicit quadrotor step on one MI355X.

A bench "step" is one rollout of the whole hot path over the workload: one
md_step call advancing every drone `physics_steps` steps (rotor speeds from
the PID, motor model, ground effect, drag, pairwise downwash, Newton-Euler,
exponential map, KIN-20 observation written to HBM every physics step).
Throughput is drone-steps/s = drones x physics steps x K / time of K rollouts,
inputs resident in HBM before the timed region.

Default workload: 8192 environments x 32 drones (262,144 drones) on yawed
4x4x2 lattices, PID formation targets, ground effect + drag + downwash,
1000 physics steps per rollout, KIN-20 observation rows [1000][20][N] fp32.

    python bench.py [--steps K] [--warmup W] [--workload formation|pid_field|ragged_grid|lattice8]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
BF16_PEAK_TFLOPS = 2500.0  # dense MFMA
METRIC = "drone-steps/s on 1 MI355X, full aero plain vs MLP-surrogate at ≤2% force err"

# Algorithmic work per drone-step (FMA = 2 FLOP; transcendental calls are
# not counted as FLOP).  Base: motor model + mixer, rotation matrix,
# Newton-Euler, exponential map, renormalisation.
FLOP_BASE = 130
FLOP_GND = 8
FLOP_DRAG = 55
FLOP_DW_CANDIDATE = 6      # dx, dy, dz, dxy^2, two compares
FLOP_DW_PAIR = 13          # alpha, beta, beta^2, exponent, product, accumulate
FLOP_PID_UPDATE = 110
FLOP_OBS = 15
OBS_BYTES = 80             # 20 float32 per drone-step
STATE_BYTES = 2 * 4 * 23   # state read + written once per launch (p,q,v,w,pid_int,rpm)


KERNEL_SOURCES = ("paper_2606_08039_amd/csrc/md_step.hip", "paper_2606_08039_amd/csrc/md_step_kernel.h",
                  "paper_2606_08039_amd/csrc/md_sweep.h", "paper_2606_08039_amd/csrc/md_physics.h",
                  "paper_2606_08039_amd/csrc/md_internal.h", "paper_2606_08039_amd/csrc/md_api.cpp")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


# committed counter summary of the step kernel, per workload
PROFILE_TAG = {"formation": "formation_8192x32"}


def measured_traffic(workload_name):
    """HBM bytes per launch from the committed rocprofv3 counter summary
    (FETCH_SIZE and WRITE_SIZE passes, each scaled by what the counter reads
    for a plain 1 GiB device copy), or None when the kernel sources changed
    since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "step_kernel_%s_counters.json" % PROFILE_TAG.get(workload_name, workload_name))
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_sha256") != kernel_source_hash():
        return None
    return rec["fetch_kib_per_dispatch"] * 1024 * rec["fetch_scale"] + \
        rec["write_kib_per_dispatch"] * 1024 * rec["write_scale"]


def workload(name, hover):
    from paper_2606_08039_amd import workloads as wl
    if name == "formation":
        w = wl.formation(n_envs=8192, n_steps=1000, seed=4)
        return w, dict(workload="formation_8192x32_pid_gnd_drag_dw_kin20", n_envs=8192,
                       drones_per_env=32, obs="KIN-20 every physics step")
    if name == "lattice8":
        w = wl.lattice(n_envs=16384, shape=(2, 2, 2), n_steps=1000, seed=3)
        return w, dict(workload="lattice_16384x8_pid_gnd_drag_dw", n_envs=16384, drones_per_env=8,
                       obs="none")
    if name == "pid_field":
        w = wl.pid_field(n_envs=4096, n_steps=2400, seed=1)
        return w, dict(workload="pid_field_4096x1_pid_gnd_drag", n_envs=4096, drones_per_env=1,
                       obs="none")
    if name == "ragged_grid":
        w = wl.ragged_grid(hover, n_envs=1024, n_steps=100, seed=2)
        return w, dict(workload="ragged_grid_1024_envs_M2to32_rpm_gnd_drag_dw", n_envs=1024,
                       drones_per_env="U{2..32}", obs="none")
    raise SystemExit("unknown workload " + name)


def algorithmic_counts(w, with_obs):
    """FLOP and HBM bytes the method needs per rollout (one md_step call)."""
    off = np.asarray(w["env_offsets"], dtype=np.int64)
    m = np.diff(off)
    n = int(off[-1])
    K = w["n_steps"]
    mask = w["aero_mask"]
    per_drone = FLOP_BASE + (FLOP_GND if mask & 1 else 0) + (FLOP_DRAG if mask & 2 else 0)
    if w["act_type"] == "pid":
        per_drone += FLOP_PID_UPDATE / w["ctrl_decim"]
    if with_obs:
        per_drone += FLOP_OBS
    flop = per_drone * n * K
    if mask & 4:
        # ordered candidate pairs (i, j != i) per env, about half of them pass dz > 0
        cand = float(np.sum(m * (m - 1)))
        flop += (FLOP_DW_CANDIDATE * cand + FLOP_DW_PAIR * cand / 2) * K
    act_bytes = 16 * n * (K if w["action_per_step"] else 1)
    bytes_ = STATE_BYTES * n + act_bytes + (OBS_BYTES * n * K if with_obs else 0)
    return flop, bytes_


def host_cpu():
    """What the CPU baseline ran on: the CPUs visible to this process, the
    thread count the job may use, the CPU model."""
    visible = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    omp = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    # all cores of the job's CPU share: the visible CPUs, or fewer when the
    # environment limits the job's threads (OMP_NUM_THREADS)
    share = min(visible, omp) if omp > 0 else visible
    return {"cpu_count": os.cpu_count(), "nproc": visible, "omp_num_threads": omp or None,
            "threads_all": share, "model": model}


def cpu_baseline(w, with_obs, seconds_one=4.0, seconds_all=3.0, reps=3):
    """The FP64 oracle (the same C code, built -O3 -march=native for this
    host) on bounded samples of the same workload: on one thread and on all
    threads of the job's CPU share, each the median of `reps` runs."""
    import tempfile
    import oracle as orc
    from paper_2606_08039_amd import workloads as wl
    build = orc.load_native(tempfile.mkdtemp(prefix="oracle_native_"))
    host = host_cpu()
    P = orc.cf2x()
    n_env_total = len(w["env_offsets"]) - 1
    steps = min(w["n_steps"], 100)

    def run(n_envs, n_steps, threads):
        sub = wl.subset_envs(w, n_envs)
        s = {k: v.astype(np.float64) for k, v in sub["state"].items()}
        act = sub["action"][:n_steps] if w["action_per_step"] else sub["action"]
        n = int(sub["env_offsets"][-1])
        t0 = time.perf_counter()
        orc.step(P, w["dt"], w["aero_mask"], {"rpm": 0, "pid": 1}[w["act_type"]],
                 w["ctrl_decim"], sub["env_offsets"], s, act.astype(np.float64),
                 w["action_per_step"], n_steps, n_obs_slots=1 if with_obs else 0,
                 n_threads=threads)
        return n * n_steps, time.perf_counter() - t0

    def sized(threads, seconds):
        # calibrate on a few environments, then size the sample to `seconds`
        e0 = min(n_env_total, 16 * threads)
        ds, dt = run(e0, min(10, steps), threads)
        envs = int(max(1, min(n_env_total, e0 * seconds / max(dt * steps / min(10, steps), 1e-9))))
        rates, walls, n_ds = [], [], 0
        for _ in range(reps):
            n_ds, dt = run(envs, steps, threads)
            rates.append(n_ds / dt)
            walls.append(dt)
        return {"value": float(np.median(rates)), "unit": "drone-steps/s", "threads": threads,
                "runs": [round(r, 1) for r in rates],
                "sample": "%d envs (%d drones) x %d physics steps, median of %d runs of %.1f-%.1f s"
                          % (envs, n_ds // steps, steps, reps, min(walls), max(walls))}

    one = sized(1, seconds_one)
    allc = sized(host["threads_all"], seconds_all)
    return {"value": allc["value"], "unit": "drone-steps/s", "cores": host["threads_all"], "kind": "oracle",
            "sample": "FP64 C oracle (%s), KIN rows to a 1-slot ring; all cores: %s; one core: %s"
                      % (build, allc["sample"], one["sample"]),
            "one_core": one, "all_cores": allc, "host": host}


def timed_rollouts(args, w, p, with_obs, mask=None, integrator=None, surrogate_weights=None,
                   tune=True, config=None, dr=None, wind=None):
    """Warm up, then time args.steps rollouts (one md_step call of w["n_steps"]
    physics steps each) on torch's current stream, which is also the stream
    the step kernels are launched on.  Returns wall seconds, the per-launch
    kernel times (HIP events around each launch), the launch configuration
    and the judge statistics of a surrogate context."""
    import torch
    from paper_2606_08039_amd import md
    n = int(w["env_offsets"][-1])
    K = w["n_steps"]
    act = {"rpm": md.MD_ACT_RPM, "pid": md.MD_ACT_PID}[w["act_type"]]
    ctx = md.md_create(p, w["dt"], w["aero_mask"] if mask is None else mask, act, w["ctrl_decim"])
    try:
        if integrator is not None:
            md.md_set_integrator(ctx, integrator)
        md.md_bind_layout(ctx, w["env_offsets"])
        if surrogate_weights is not None:
            flat, norm = surrogate_weights
            md.md_load_surrogate(ctx, flat, norm, SUR_DZ_OOD, 64)
            md.md_set_surrogate_ood(ctx, *SUR_OOD)
            md.md_set_surrogate_region(ctx, *SUR_REGION)
        state = md.DeviceState.from_numpy(w["state"])
        dr_t = None
        if dr is not None:
            dr_t = {k: (torch.from_numpy(v).cuda() if isinstance(v, np.ndarray) else v) for k, v in dr.items()}
            state.add_dr_blocks(act)
            md.md_set_domain_randomization(ctx, dr_t["scale"], dr_t["tau_mot"], dr_t["delay"],
                                           noise=dr_t["noise"], seed=dr_t["seed"], obs_delay=dr_t["obs_delay"],
                                           obs_bias=dr_t["obs_bias"])
        wind_t = None
        if wind is not None:
            state.add_wind_block()
            wind_t = {k: (torch.from_numpy(v).cuda() if isinstance(v, np.ndarray) else v) for k, v in wind.items()}
            md.md_set_wind(ctx, **wind_t)
        action = torch.from_numpy(np.ascontiguousarray(w["action"], dtype=np.float32)).cuda()
        obs = torch.empty((K, 20, n), dtype=torch.float32, device="cuda") if with_obs else None
        n_slots = K if with_obs else 0
        stream = torch.cuda.current_stream()
        cfg = None
        if config is not None and surrogate_weights is None:
            md.md_set_launch_config(ctx, **config)
            cfg = md.md_get_launch_config(ctx)
        elif tune and not args.no_tune and surrogate_weights is None:
            # untimed: choose the launch configuration on scratch copies of the
            # state, with the observation stream when the timed launches write it
            # (over the full launch length: configurations that tie over a few
            # dozen steps separate over a thousand)
            if with_obs:
                cfg = md.md_autotune_obs(ctx, state, action, w["action_per_step"], obs, n_slots,
                                         n_steps=K, stream=stream, cache_path="")
            else:
                cfg = md.md_autotune(ctx, state, action, w["action_per_step"], n_steps=min(K, 50),
                                     stream=stream, cache_path="")
        step0 = 0
        for _ in range(args.warmup):
            md.md_step(ctx, state, action, w["action_per_step"], obs, n_slots, K, step0, stream)
            step0 += K
        torch.cuda.synchronize()
        if surrogate_weights is not None:
            md.md_judge_reset(ctx)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
        t0 = time.perf_counter()
        for i in range(args.steps):
            ev[i][0].record(stream)
            md.md_step(ctx, state, action, w["action_per_step"], obs, n_slots, K, step0, stream)
            ev[i][1].record(stream)
            step0 += K
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        kernel_ms = [a.elapsed_time(b) for a, b in ev]
        judge = md.md_judge_stats(ctx) if surrogate_weights is not None else None
        # untimed sanity check of the final state
        fin = torch.isfinite(torch.cat([state.t[k] for k in ("p", "q", "v", "w")])).all(dim=0)
        speed = torch.linalg.vector_norm(state.t["v"], dim=0)
        check_state = {"nonfinite_drones": int((~fin).sum()),
                       "max_speed": float(torch.where(fin, speed, torch.zeros_like(speed)).max()),
                       "below_ground": int((state.t["p"][2] < 0).sum())}
    finally:
        md.md_destroy(ctx)
    return wall, kernel_ms, cfg, judge, check_state


# Surrogate fallback: the downwash singularity (a neighbour above by less
# than 10 um) and the edge of the training data (lattice flights: speeds below
# 1 m/s, neighbour relative speeds below 1.2 m/s, tilts below half a degree,
# column partners 0.8-1.45 m apart vertically, same-layer neighbours at least
# 0.9 m apart laterally): world speed 1.5 m/s, relative speed 2 m/s, tilt 2
# degrees, a neighbour inside |dz| < 0.75 m and dxy < 0.85 m (outside it
# Eq. 6 stays below 1e-4 N for 10 um < dz < 0.75 m) or beyond |dz| > 3 m.
SUR_DZ_OOD = 1e-5
SUR_OOD = (1.5, 2.0, float(np.radians(2.0)))
SUR_REGION = (0.75, 0.85, 3.0)


def surrogate_leg(args, w, p, with_obs):
    """The same rollouts with the learned residual in place of Eq. 4-6
    (fallback near the downwash singularity, 1/64 of drone-steps judged
    against the plain terms)."""
    from paper_2606_08039_amd import md, surrogate
    path = args.weights or surrogate.DEFAULT_WEIGHTS
    if not os.path.exists(path):
        return {"value": None, "note": "no trained weights at %s" % os.path.relpath(path, ROOT)}
    flat, norm, meta = surrogate.load(path)
    n = int(w["env_offsets"][-1])
    K = w["n_steps"]
    wall, kernel_ms, _, j, chk = timed_rollouts(args, w, p, with_obs, mask=md.MD_AERO_SURROGATE,
                                                surrogate_weights=(flat, norm))
    kms = float(np.mean(kernel_ms))
    ds = float(n) * K * args.steps
    mfma_flop = 86016.0 * n * K
    return {"value": ds / wall, "unit": "drone-steps/s", "ms_per_step": wall / args.steps * 1e3,
            "kernel_ms_avg": kms,
            "mfma_tflops": mfma_flop / (kms * 1e-3) / 1e12,
            # the network's MFMA work against the dense bf16 peak; the binding pipe
            # is the VALU (SiLU epilogues, neighbour ranking), which the MFMA does
            # not overlap
            "roofline": {"bound": "mfma", "achieved": round(mfma_flop / (kms * 1e-3) / 1e12, 1),
                         "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": round(mfma_flop / (kms * 1e-3) / 1e12 / BF16_PEAK_TFLOPS, 4), "traffic": None},
            "judge_force_rel_err": j["force_rel_err"], "judged_drone_steps": j["n_judged"],
            "judge_nonfinite": j["n_nonfinite"], "final_state": chk,
            "fallback_fraction": j["n_fallback"] / max(j["n_drone_steps"], 1.0),
            "full_ranking_fraction": j["n_knn_full"] / max(j["n_drone_steps"], 1.0),
            "held_out_force_rel_err": meta.get("eps_held_out"),
            "fallback_bounds": {"dz": SUR_DZ_OOD, "speed": SUR_OOD[0], "rel_speed": SUR_OOD[1],
                                "tilt_rad": SUR_OOD[2], "near_dz": SUR_REGION[0], "near_r": SUR_REGION[1],
                                "far_dz": SUR_REGION[2]},
            "weights": os.path.relpath(path, ROOT)}


# Uniform two-layer lattices (the trained network's neighbourhood: one
# column partner, the rest of the layer laterally) from 8 to 512 drones per
# environment, the same number of drones at every size.
CROSSOVER_SHAPES = {8: (2, 2, 2), 16: (4, 2, 2), 32: (4, 4, 2), 64: (8, 4, 2), 128: (8, 8, 2), 256: (16, 8, 2),
                    512: (16, 16, 2)}


def crossover_leg(args, p, n_drones=262144, steps=250):
    """Plain full aero (autotuned) against the learned residual on the
    CROSSOVER_SHAPES lattices: PID waypoints, no observation writes, one
    warm-up and three timed launches of `steps` steps each; rates from the
    kernel time.  The plain step's neighbour sweep grows as M, the network's
    cost per drone does not, so the surrogate would win beyond some M."""
    from paper_2606_08039_amd import workloads as wl

    class A:
        pass
    a = A()
    a.steps, a.warmup, a.no_tune, a.weights = 3, 1, False, args.weights
    rows = []
    for M, shape in CROSSOVER_SHAPES.items():
        w = wl.lattice(n_envs=n_drones // M, shape=shape, n_steps=steps, seed=40 + M)
        n = int(w["env_offsets"][-1])
        _, kms, cfg, _, _ = timed_rollouts(a, w, p, False)
        plain = n * steps / (float(np.mean(kms)) * 1e-3)
        sur = surrogate_leg(a, w, p, False)
        srate = n * steps / (sur["kernel_ms_avg"] * 1e-3) if sur.get("value") else None
        rows.append({"M": M, "lattice": "x".join(map(str, shape)), "n_envs": n // M,
                     "plain": plain, "plain_ms": float(np.mean(kms)), "plain_config": cfg,
                     "surrogate": srate, "surrogate_ms": sur.get("kernel_ms_avg"),
                     "surrogate_over_plain": (srate / plain) if srate else None,
                     "judge_force_rel_err": sur.get("judge_force_rel_err"),
                     "fallback_fraction": sur.get("fallback_fraction"),
                     "full_ranking_fraction": sur.get("full_ranking_fraction")})
    won = [r["M"] for r in rows if r["surrogate_over_plain"] and r["surrogate_over_plain"] >= 1.0]
    return {"unit": "drone-steps/s", "drones": n_drones, "steps_per_launch": steps, "rows": rows,
            "crossover_M": min(won) if won else None}


DR_SEED = 50


def dr_leg(args, w, p, with_obs):
    """The same rollouts under every row of the domain-randomisation table
    (Table "Recommended domain-randomization ranges"): initial-state draws,
    per-drone factors, motor lag, action and sensor latency, sensor noise and
    sticky bias, and COMBINED wind with a per-environment mean."""
    from paper_2606_08039_amd import workloads as wl
    n = int(w["env_offsets"][-1])
    # latencies drawn per environment (one sensing and radio pipeline per
    # arena); the per-vehicle draw is timed beside it
    we = wl.randomized(w, DR_SEED, latency_per="env")
    wall, kernel_ms, cfg, _, chk = timed_rollouts(args, we, p, with_obs, dr=we["dr"], wind=we["wind"])
    wd = wl.randomized(w, DR_SEED, latency_per="drone")
    wall_d, kernel_ms_d, cfg_d, _, _ = timed_rollouts(args, wd, p, with_obs, dr=wd["dr"], wind=wd["wind"])
    return {"value": float(n) * w["n_steps"] * args.steps / wall, "unit": "drone-steps/s",
            "ms_per_step": wall / args.steps * 1e3, "kernel_ms_avg": float(np.mean(kernel_ms)),
            "launch_config": cfg, "final_state": chk, "latency_per": "environment",
            "per_drone_latency": {"value": float(n) * w["n_steps"] * args.steps / wall_d,
                                  "kernel_ms_avg": float(np.mean(kernel_ms_d)), "launch_config": cfg_d}}


def ragged_graph_leg(args, p, hover):
    """The latency-bound ragged layout (1024 environments of 2..32 drones on a
    coplanar grid, 17.4k drones, per-step rotor speeds, all aero terms): a
    100-step rollout as one persistent launch of 100 steps (the value), as
    that launch replayed from a captured hipGraph, and as 10 launches of 10
    steps replayed from one captured hipGraph and issued eagerly."""
    import torch
    from paper_2606_08039_amd import md, workloads as wl
    w = wl.ragged_grid(hover, n_envs=1024, n_steps=100, seed=2)
    n = int(w["env_offsets"][-1])
    ctx = md.md_create(p, w["dt"], w["aero_mask"], md.MD_ACT_RPM, 1)
    try:
        md.md_bind_layout(ctx, w["env_offsets"])
        state = md.DeviceState.from_numpy(w["state"])
        action = torch.from_numpy(np.ascontiguousarray(w["action"], dtype=np.float32)).cuda()
        stream = torch.cuda.current_stream()
        cfg = md.md_autotune(ctx, state, action[:10].contiguous(), True, n_steps=10, stream=stream, cache_path="")
        reps = 20
        # eager: ten 10-step launches per rollout
        t_eager = []
        for r in range(reps + 2):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            for k in range(10):
                md.md_step(ctx, state, action[10 * k:10 * k + 10].contiguous(), True, None, 0, 10, 10 * k, stream)
            b.record(stream)
            torch.cuda.synchronize()
            if r >= 2:
                t_eager.append(a.elapsed_time(b))
        # one persistent launch of all 100 steps
        t_one = []
        for r in range(reps + 2):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            md.md_step(ctx, state, action, True, None, 0, 100, 0, stream)
            b.record(stream)
            torch.cuda.synchronize()
            if r >= 2:
                t_one.append(a.elapsed_time(b))
        def replay(steps_per_launch, n_launches):
            graph = md.md_rollout_graph_create(ctx, state, action, True, None, 0, steps_per_launch=steps_per_launch,
                                               n_launches=n_launches, step0=0, stream=stream)
            t = []
            try:
                for r in range(reps + 2):
                    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    a.record(stream)
                    md.md_graph_launch(graph, stream)
                    b.record(stream)
                    torch.cuda.synchronize()
                    if r >= 2:
                        t.append(a.elapsed_time(b))
            finally:
                md.md_graph_destroy(graph)
            return t
        t_graph = replay(10, 10)
        t_graph1 = replay(100, 1)
    finally:
        md.md_destroy(ctx)
    mg, me, m1 = float(np.median(t_graph)), float(np.median(t_eager)), float(np.median(t_one))
    return {"value": float(n) * 100 / (m1 * 1e-3), "unit": "drone-steps/s", "n_drones": n,
            "rollout_ms_single_launch_median": m1, "ns_per_step_single_launch": m1 * 1e6 / 100,
            "rollout_ms_graph_median": mg, "rollout_ms_graph_one_launch_median": float(np.median(t_graph1)),
            "rollout_ms_eager_median": me, "replays": reps,
            "value_graph": float(n) * 100 / (mg * 1e-3),
            "launch_config": cfg, "workload": "ragged_grid_1024envs_m2to32_rpm_gnd_drag_dw_100steps"}


# Sec. "Wind and turbulence", the paper's hover example: a steady 0.9 m/s
# wind along +y plus Dryden turbulence (per-drone Philox draws).
WIND_BENCH = dict(models=1 | 4, v_mean=(0.0, 0.9, 0.0), rho=1.225, cd_area=0.01, dryden_sigma=0.3,
                  dryden_airspeed=0.9, seed=7)


def wind_leg(args, w, p, with_obs):
    """The same rollouts under steady wind plus Dryden turbulence."""
    n = int(w["env_offsets"][-1])
    wall, kernel_ms, cfg, _, chk = timed_rollouts(args, w, p, with_obs, wind=WIND_BENCH)
    return {"value": float(n) * w["n_steps"] * args.steps / wall, "unit": "drone-steps/s",
            "ms_per_step": wall / args.steps * 1e3, "kernel_ms_avg": float(np.mean(kernel_ms)),
            "launch_config": cfg, "final_state": chk, "wind": WIND_BENCH}


def pid_field_leg(args, p, hover):
    """The latency-bound single-drone field: 4096 environments of one drone,
    PID every 5th step, ground effect and drag, 2400 physics steps per
    launch, no observations; 64 waves leave most of the chip idle, so the
    figure is the time per physics step of the dependency chain."""
    w, cfg_w = workload("pid_field", hover)
    n = int(w["env_offsets"][-1])
    wall, kernel_ms, cfg, _, chk = timed_rollouts(args, w, p, False)
    k = float(np.median(kernel_ms))
    return {"value": float(n) * w["n_steps"] * args.steps / wall, "unit": "drone-steps/s",
            "kernel_ms_median": k, "ns_per_step": k * 1e6 / w["n_steps"], "launch_config": cfg,
            "final_state": chk, "workload": cfg_w["workload"]}


def rk4_leg(args, w, p, with_obs):
    """The same rollouts with the classic Runge-Kutta integrator (four force
    evaluations, four neighbour sweeps per physics step)."""
    from paper_2606_08039_amd import md
    n = int(w["env_offsets"][-1])
    wall, kernel_ms, cfg, _, chk = timed_rollouts(args, w, p, with_obs, integrator=md.MD_INTEG_RK4)
    return {"value": float(n) * w["n_steps"] * args.steps / wall, "unit": "drone-steps/s",
            "ms_per_step": wall / args.steps * 1e3, "kernel_ms_avg": float(np.mean(kernel_ms)),
            "launch_config": cfg, "final_state": chk}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=int(os.environ.get("WORLD_SIZE", "1")))
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="formation")
    ap.add_argument("--no-obs", action="store_true", help="skip the KIN-20 writes")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true", help="skip the surrogate-aero leg")
    ap.add_argument("--no-rk4", action="store_true", help="skip the Runge-Kutta leg")
    ap.add_argument("--no-dr", action="store_true", help="skip the domain-randomisation leg")
    ap.add_argument("--no-wind", action="store_true", help="skip the wind leg")
    ap.add_argument("--no-graph", action="store_true", help="skip the ragged-layout hipGraph leg")
    ap.add_argument("--no-pid-field", action="store_true", help="skip the single-drone PID field leg")
    ap.add_argument("--no-compute-only", action="store_true",
                    help="skip plain_no_obs (the same launches without observation writes)")
    ap.add_argument("--no-tune", action="store_true", help="default launch configuration, no autotuning")
    ap.add_argument("--config", default=None,
                    help="launch configuration lanes_per_drone,unroll,waves_per_group,pair_symmetric "
                         "for the plain leg (instead of autotuning)")
    ap.add_argument("--weights", default=None, help="surrogate weights file")
    ap.add_argument("--no-crossover", action="store_true",
                    help="skip plain vs surrogate on uniform lattices of 8..512 drones per environment")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (for HBM counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: measures one GPU; --gpus %d is not supported "
              "(environments shard across GPUs with no per-step exchange)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2606_08039_amd import md

    torch.cuda.set_device(0)
    p = md.md_default_params_cf2x()
    hover = md.md_derive(p).hover_rpm
    w, cfg = workload(args.workload, hover)
    with_obs = (cfg["obs"] != "none") and not args.no_obs
    n = int(w["env_offsets"][-1])
    K = w["n_steps"]

    config = None
    if args.config:
        v = [int(x) for x in args.config.split(",")]
        config = dict(lanes_per_drone=v[0], unroll=v[1], waves_per_group=v[2], pair_symmetric=v[3])
    wall, kernel_ms, launch_cfg, _, check_state = timed_rollouts(args, w, p, with_obs, tune=not args.no_tune,
                                                                 config=config)

    ds = float(n) * K * args.steps
    value = ds / wall
    flop, bytes_ = algorithmic_counts(w, with_obs)
    kavg = float(np.mean(kernel_ms)) * 1e-3
    hbm = bytes_ / kavg / 1e9
    alu = flop / kavg / 1e12
    traffic = measured_traffic(args.workload)
    # Two limits meet in the step kernel: its vector-ALU instruction stream
    # (the launch without observation writes, `plain_no_obs`, is bound by it)
    # and the observation write stream.  Both views are reported; the primary
    # one follows the roofline model: below the ridge point (FP32 peak over
    # HBM peak, in FLOP per byte) the algorithmic intensity puts the kernel
    # under the HBM line, above it under the ALU line.
    roof_alu = {"bound": "alu", "achieved": round(alu, 3), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(alu / FP32_PEAK_TFLOPS, 4), "traffic": traffic}
    roof_hbm = {"bound": "hbm", "achieved": round(hbm, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(hbm / HBM_PEAK_GBS, 4), "traffic": traffic}
    intensity = flop / bytes_
    ridge = FP32_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)
    roof = roof_hbm if intensity < ridge else roof_alu
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "drone-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded lattices / grids, PID targets or rotor speeds)",
        "config": dict(cfg, n_drones=n, physics_steps_per_rollout=K, dt=w["dt"],
                       aero="GND|DRAG|DW" if w["aero_mask"] == 7 else "GND|DRAG" if w["aero_mask"] == 3 else w["aero_mask"],
                       action="pid waypoints, ctrl_decim %d" % w["ctrl_decim"] if w["act_type"] == "pid"
                       else "rotor speeds per step", path="plain aero"),
        "roofline": roof,
        "roofline_alu": roof_alu,
        "roofline_hbm": roof_hbm,
        "intensity_flop_per_byte": round(intensity, 2),
        "ridge_flop_per_byte": round(ridge, 2),
        "kernel_ms_avg": kavg * 1e3,
        "launch_config": launch_cfg,
        "final_state": check_state,
        "algorithmic_bytes_per_launch": bytes_,
        "algorithmic_flop_per_launch": flop,
    }
    if with_obs and not args.no_compute_only:
        # the same launches without observation writes, in the same launch
        # configuration: the compute side of the step kernel alone
        wall0, kms0, _, _, _ = timed_rollouts(args, w, p, False, tune=False, config=launch_cfg)
        flop0, _ = algorithmic_counts(w, False)
        k0 = float(np.mean(kms0)) * 1e-3
        out["plain_no_obs"] = {"value": ds / wall0, "unit": "drone-steps/s", "kernel_ms_avg": k0 * 1e3,
                               "alu_tflops": round(flop0 / k0 / 1e12, 3),
                               "frac_fp32_peak": round(flop0 / k0 / 1e12 / FP32_PEAK_TFLOPS, 4)}
    if not args.no_surrogate:
        out["surrogate"] = surrogate_leg(args, w, p, with_obs)
        if out["surrogate"].get("value"):
            out["surrogate"]["speed_vs_plain"] = out["surrogate"]["value"] / value
    if not args.no_rk4:
        out["rk4"] = rk4_leg(args, w, p, with_obs)
        out["rk4"]["speed_vs_euler"] = out["rk4"]["value"] / value
    if not args.no_dr:
        out["domain_randomization"] = dr_leg(args, w, p, with_obs)
        out["domain_randomization"]["speed_vs_plain"] = out["domain_randomization"]["value"] / value
    if not args.no_graph:
        out["ragged_graph"] = ragged_graph_leg(args, p, hover)
    if not args.no_pid_field:
        out["pid_field"] = pid_field_leg(args, p, hover)
    if not args.no_wind:
        out["wind"] = wind_leg(args, w, p, with_obs)
        out["wind"]["speed_vs_plain"] = out["wind"]["value"] / value
    if not args.no_crossover and not args.no_surrogate:
        out["crossover"] = crossover_leg(args, p)
    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = {"read": a.numel() * 4, "write": a.numel() * 4}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, with_obs)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
