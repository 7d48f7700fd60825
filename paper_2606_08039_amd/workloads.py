"""Seeded synthetic inputs for the batched quadrotor step.

This module only draws inputs: initial states, rotor-speed or waypoint
actions and ragged environment layouts.  It holds none of the method's
arithmetic -- quantities such as the hover rotor speed are passed in by the
caller -- and it imports nothing else from this package, so both the HIP path
and the CPU oracle consume exactly the same float32 buffers.

State arrays are float32, component-major ``[c][N]``:
``p[3], q[4] (w,x,y,z), v[3], w[3], pid_int[6], rpm[4], ctl[4]``.

Workloads (dt = 1/240 s):

* ``single``       1 env x 1 drone at (0,0,1), level, at rest; rotor speeds
                   hover*(1+u), u ~ U[-0.05, 0.05] per step and motor;
                   no aerodynamic terms; ``jitter=0`` gives the pure hover run.
* ``pid_field``    E envs x 1 drone, xy ~ U[-1,1]^2, z ~ U[0.05,1.5], random
                   yaw, at rest; waypoints U[-2,2]^2 x U[0.2,2], yaw 0;
                   PID every 5 steps; ground effect + drag.
* ``ragged_grid``  E envs with M ~ U{2..32} drones on distinct cells of a
                   4x4x4 grid of 0.15 m pitch (origin (-0.225,-0.225,0.5)),
                   level, at rest; per-step rotor speeds hover*(1+U[-0.1,0.1]);
                   ground effect + drag + downwash.
* ``lattice``      E envs x (nx*ny*nz) drones on a yawed lattice with lateral
                   pitch U[1.0,1.3] m, vertical pitch U[0.9,1.0] m, lower layer
                   at z ~ U[0.3,0.5]; PID waypoints = lattice point +
                   U[-0.05,0.05]^3, start = waypoint + U[-0.1,0.1]^3.
                   2x2x2 / 16384 envs is the surrogate workload, 4x4x2 / 8192
                   envs the formation workload.
"""
import numpy as np

STATE_ROWS = (("p", 3), ("q", 4), ("v", 3), ("w", 3), ("pid_int", 6), ("rpm", 4), ("ctl", 4))
DT = 1.0 / 240.0


def empty_state(n):
    s = {k: np.zeros((r, n), dtype=np.float32) for k, r in STATE_ROWS}
    s["q"][0] = 1.0
    return s


def _yaw_quat(yaw):
    # A rotation by `yaw` about world z, as a [w, x, y, z] unit quaternion.
    return np.cos(0.5 * yaw), np.sin(0.5 * yaw)


def single(hover_rpm, n_steps=240, jitter=0.05, seed=0):
    rng = np.random.default_rng(seed)
    s = empty_state(1)
    s["p"][2, 0] = 1.0
    u = rng.uniform(-jitter, jitter, size=(n_steps, 4, 1)) if jitter > 0 else np.zeros((n_steps, 4, 1))
    act = (hover_rpm * (1.0 + u)).astype(np.float32)
    return dict(name="single", env_offsets=np.array([0, 1], dtype=np.int32), state=s,
                action=act, action_per_step=True, aero_mask=0, act_type="rpm",
                ctrl_decim=1, n_steps=n_steps, dt=DT)


def pid_field(n_envs=4096, n_steps=2400, seed=1):
    rng = np.random.default_rng(seed)
    n = n_envs
    s = empty_state(n)
    s["p"][0:2] = rng.uniform(-1.0, 1.0, size=(2, n))
    s["p"][2] = rng.uniform(0.05, 1.5, size=n)
    yaw = rng.uniform(-np.pi, np.pi, size=n)
    cw, sz = _yaw_quat(yaw)
    s["q"][0], s["q"][3] = cw, sz
    tgt = np.zeros((4, n), dtype=np.float32)
    tgt[0:2] = rng.uniform(-2.0, 2.0, size=(2, n))
    tgt[2] = rng.uniform(0.2, 2.0, size=n)
    return dict(name="pid_field", env_offsets=np.arange(n + 1, dtype=np.int32), state=s,
                action=tgt[None], action_per_step=False, aero_mask=1 | 2, act_type="pid",
                ctrl_decim=5, n_steps=n_steps, dt=DT)


def ragged_grid(hover_rpm, n_envs=1024, n_steps=100, m_lo=2, m_hi=32, pitch=0.15, seed=2):
    rng = np.random.default_rng(seed)
    m = rng.integers(m_lo, m_hi + 1, size=n_envs)
    off = np.zeros(n_envs + 1, dtype=np.int32)
    off[1:] = np.cumsum(m)
    n = int(off[-1])
    s = empty_state(n)
    g = np.arange(4)
    cells = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
    origin = np.array([-0.225, -0.225, 0.5])
    for e in range(n_envs):
        pick = rng.permutation(64)[: m[e]]
        pos = origin + pitch * cells[pick]
        s["p"][:, off[e]:off[e + 1]] = pos.T
    u = rng.uniform(-0.1, 0.1, size=(n_steps, 4, n))
    act = (hover_rpm * (1.0 + u)).astype(np.float32)
    return dict(name="ragged_grid", env_offsets=off, state=s, action=act, action_per_step=True,
                aero_mask=1 | 2 | 4, act_type="rpm", ctrl_decim=1, n_steps=n_steps, dt=DT)


def lattice(n_envs=16384, shape=(2, 2, 2), n_steps=1000, seed=3, target_jitter=0.05,
            start_jitter=0.1):
    rng = np.random.default_rng(seed)
    nx, ny, nz = shape
    m = nx * ny * nz
    n = n_envs * m
    off = (np.arange(n_envs + 1) * m).astype(np.int32)
    sxy = rng.uniform(1.0, 1.3, size=n_envs)
    szz = rng.uniform(0.9, 1.0, size=n_envs)
    yaw = rng.uniform(0.0, 2.0 * np.pi, size=n_envs)
    z0 = rng.uniform(0.3, 0.5, size=n_envs)
    ix, iy, iz = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    lx = (ix.ravel() - 0.5 * (nx - 1))
    ly = (iy.ravel() - 0.5 * (ny - 1))
    lz = iz.ravel().astype(np.float64)
    c, sn = np.cos(yaw)[:, None], np.sin(yaw)[:, None]
    X = sxy[:, None] * (c * lx[None] - sn * ly[None])
    Y = sxy[:, None] * (sn * lx[None] + c * ly[None])
    Z = z0[:, None] + szz[:, None] * lz[None]
    base = np.stack([X.ravel(), Y.ravel(), Z.ravel()])  # [3][n], env-major
    tgt = np.zeros((4, n), dtype=np.float32)
    tgt[0:3] = base + rng.uniform(-target_jitter, target_jitter, size=(3, n))
    s = empty_state(n)
    s["p"][:] = tgt[0:3].astype(np.float64) + rng.uniform(-start_jitter, start_jitter, size=(3, n))
    return dict(name="lattice%dx%dx%d" % shape, env_offsets=off, state=s, action=tgt[None],
                action_per_step=False, aero_mask=1 | 2 | 4, act_type="pid", ctrl_decim=5,
                n_steps=n_steps, dt=DT, lattice_points=base.astype(np.float32),
                target_jitter=target_jitter)


def rejitter_targets(w, rng):
    """New PID waypoints for a lattice workload: its lattice points plus a
    fresh U[-j, j]^3 jitter (the same draw as at creation), yaw 0."""
    base = w["lattice_points"]
    j = w["target_jitter"]
    tgt = np.zeros((1, 4, base.shape[1]), dtype=np.float32)
    tgt[0, 0:3] = base + rng.uniform(-j, j, size=base.shape)
    return tgt


def formation(n_envs=8192, n_steps=1000, seed=4):
    w = lattice(n_envs=n_envs, shape=(4, 4, 2), n_steps=n_steps, seed=seed)
    w["name"] = "formation"
    return w


def commanded(kind, hover_thrust, n_envs=1024, n_steps=480, seed=5):
    """E envs x 1 drone placed and oriented as in pid_field, with held
    commands for the VEL, ATTITUDE or DSL action types (ground effect + drag):
      vel       heading-frame velocity U[-1,1]^2 x U[-0.5,0.5] m/s, yaw rate U[-1,1] rad/s;
      attitude  thrust hover_thrust*(1+U[-0.2,0.2]) N, roll and pitch U[-0.3,0.3] rad,
                yaw rate U[-1,1] rad/s;
      dsl       waypoints U[-2,2]^2 x U[0.2,2] m, yaw U[-pi,pi), feed-forward
                acceleration U[-0.5,0.5]^3 m/s^2; the setpoint block starts at the
                drone's position and yaw."""
    rng = np.random.default_rng(seed)
    n = n_envs
    s = empty_state(n)
    s["p"][0:2] = rng.uniform(-1.0, 1.0, size=(2, n))
    s["p"][2] = rng.uniform(0.3, 1.5, size=n)
    yaw = rng.uniform(-np.pi, np.pi, size=n)
    cw, sz = _yaw_quat(yaw)
    s["q"][0], s["q"][3] = cw, sz
    if kind == "vel":
        cmd = np.stack([rng.uniform(-1, 1, n), rng.uniform(-1, 1, n), rng.uniform(-0.5, 0.5, n),
                        rng.uniform(-1, 1, n)])
    elif kind == "attitude":
        cmd = np.stack([hover_thrust * (1 + rng.uniform(-0.2, 0.2, n)), rng.uniform(-0.3, 0.3, n),
                        rng.uniform(-0.3, 0.3, n), rng.uniform(-1, 1, n)])
    elif kind == "dsl":
        cmd = np.stack([rng.uniform(-2, 2, n), rng.uniform(-2, 2, n), rng.uniform(0.2, 2, n),
                        rng.uniform(-np.pi, np.pi, n), rng.uniform(-0.5, 0.5, n),
                        rng.uniform(-0.5, 0.5, n), rng.uniform(-0.5, 0.5, n)])
        s["ctl"][0:3] = s["p"]
        s["ctl"][3] = yaw
    else:
        raise ValueError(kind)
    return dict(name="commanded_" + kind, env_offsets=np.arange(n + 1, dtype=np.int32), state=s,
                action=cmd.astype(np.float32)[None], action_per_step=False, aero_mask=1 | 2,
                act_type=kind, ctrl_decim=5, n_steps=n_steps, dt=DT)


def permute_envs(w, perm):
    """Same workload with its environments stored in the order ``perm``."""
    off = w["env_offsets"]
    idx = np.concatenate([np.arange(off[e], off[e + 1]) for e in perm]) if len(perm) else \
        np.zeros(0, dtype=np.int64)
    m = np.diff(off)[perm]
    noff = np.zeros(len(perm) + 1, dtype=np.int32)
    noff[1:] = np.cumsum(m)
    out = dict(w)
    out["env_offsets"] = noff
    out["state"] = {k: np.ascontiguousarray(v[:, idx]) for k, v in w["state"].items()}
    out["action"] = np.ascontiguousarray(w["action"][:, :, idx])
    if "lattice_points" in w:
        out["lattice_points"] = np.ascontiguousarray(w["lattice_points"][:, idx])
    out["drone_index"] = idx
    return out


def subset_envs(w, n_envs):
    """The first n_envs environments of a workload."""
    off = w["env_offsets"][: n_envs + 1].copy()
    n = int(off[-1])
    out = dict(w)
    out["env_offsets"] = off
    out["state"] = {k: np.ascontiguousarray(v[:, :n]) for k, v in w["state"].items()}
    out["action"] = np.ascontiguousarray(w["action"][:, :, :n])
    if "lattice_points" in w:
        out["lattice_points"] = np.ascontiguousarray(w["lattice_points"][:, :n])
    return out


def thin_envs(w, seed, m_lo=2):
    """Ragged environments from a uniform workload: each environment keeps a
    random subset of U{m_lo..M} of its drones (in their original order)."""
    rng = np.random.default_rng(seed)
    off = np.asarray(w["env_offsets"], dtype=np.int64)
    keep = []
    for e in range(len(off) - 1):
        m = int(off[e + 1] - off[e])
        k = int(rng.integers(min(m_lo, m), m + 1))
        keep.append(np.sort(rng.choice(m, size=k, replace=False)) + off[e])
    sizes = np.array([len(k) for k in keep])
    idx = np.concatenate(keep) if keep else np.zeros(0, dtype=np.int64)
    out = dict(w)
    out["env_offsets"] = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
    out["state"] = {k: np.ascontiguousarray(v[:, idx]) for k, v in w["state"].items()}
    out["action"] = np.ascontiguousarray(w["action"][:, :, idx])
    if "lattice_points" in w:
        out["lattice_points"] = np.ascontiguousarray(w["lattice_points"][:, idx])
    return out


# Table "Recommended domain-randomization ranges": half-widths a of the
# multiplicative factors U(1 - a, 1 + a), the motor time constant and the
# action latency ranges.
DR_HALF_WIDTH = {"m": 0.2, "J": 0.2, "L": 0.02, "kf": 0.15, "km": 0.15, "drag": 0.3, "C_gnd": 0.3,
                 "C1": 0.3, "max_rpm": 0.05, "g": 0.02, "bias": 0.05}
DR_TAU_MOT = (0.005, 0.050)   # s
DR_LATENCY = (0.0, 0.050)     # s
# sensors: noise sigmas of position (m), velocity (m/s), roll/pitch/yaw
# (rad), body rates (rad/s), and the sensor latency range (s)
DR_NOISE = (0.01, 0.05, float(np.radians(1.0)), 0.05)
DR_SENSOR_LATENCY = (0.0, 0.020)


def domain_randomization(w, seed, lag=True, latency=True, sensors=True, latency_per="drone"):
    """Seeded draws for the workload's drones: one vehicle per drone (mass,
    inertia, arm, kf, km, drag, C_gnd, C1, MAX_RPM, four motor biases, motor
    time constant, action latency rounded to whole steps), gravity per
    environment, and with sensors the table's noise levels, a noise seed and
    a sensor latency per drone rounded to whole steps.  Returns float32 scale
    [14][N], float32 tau_mot [N] (None without lag), int32 delay [N] (None
    without latency), noise (4 sigmas, zeros without sensors), seed and int32
    obs_delay [N] (None without sensors).  latency_per "env" draws the two
    latencies once per environment (one sensing and radio pipeline per
    arena) instead of once per drone."""
    rng = np.random.default_rng(seed)
    off = np.asarray(w["env_offsets"], dtype=np.int64)
    n = int(off[-1])
    rows = ("m", "J", "L", "kf", "km", "drag", "C_gnd", "C1", "max_rpm")
    scale = np.ones((14, n))
    for r, k in enumerate(rows):
        a = DR_HALF_WIDTH[k]
        scale[r] = rng.uniform(1 - a, 1 + a, size=n)
    a = DR_HALF_WIDTH["g"]
    scale[9] = np.repeat(rng.uniform(1 - a, 1 + a, size=len(off) - 1), np.diff(off))
    a = DR_HALF_WIDTH["bias"]
    scale[10:14] = rng.uniform(1 - a, 1 + a, size=(4, n))
    tau = rng.uniform(*DR_TAU_MOT, size=n).astype(np.float32) if lag else None
    assert latency_per in ("drone", "env")
    per_env = latency_per == "env"

    def steps(rng_range):
        x = rng.uniform(*rng_range, size=len(off) - 1 if per_env else n)
        x = np.repeat(x, np.diff(off)) if per_env else x
        return np.rint(x / w["dt"]).astype(np.int32)

    delay = steps(DR_LATENCY) if latency else None
    noise, nseed, obs_delay, obs_bias = (0.0, 0.0, 0.0, 0.0), 0, None, None
    if sensors:
        noise = DR_NOISE
        nseed = int(rng.integers(0, 2 ** 63))
        obs_delay = steps(DR_SENSOR_LATENCY)
        # sticky bias: one draw per drone and episode, with the noise levels
        sig = np.repeat(np.asarray(DR_NOISE), 3)[:, None]
        obs_bias = (sig * rng.standard_normal((12, n))).astype(np.float32)
    return dict(scale=scale.astype(np.float32), tau_mot=tau, delay=delay, noise=noise, seed=nseed,
                obs_delay=obs_delay, obs_bias=obs_bias)


# Table "Recommended domain-randomization ranges", initial state: position,
# roll/pitch/yaw and velocity offsets (uniform half-widths, m / rad / m/s).
DR_INIT = (0.2, 0.1, 0.5)
# COMBINED wind for randomisation: the mean wind of each environment has a
# uniform magnitude in [0, 1] m/s and a uniform horizontal heading; gusts,
# Dryden turbulence and the sinusoid keep fixed levels.
DR_WIND = dict(models=15, rho=1.225, cd_area=0.01, gust_prob=0.002, gust_duration=0.5, gust_amp=0.02,
               dryden_sigma=0.3, dryden_airspeed=0.9, sin_amp=0.005, sin_omega=1.0)


def perturb_initial_state(w, seed):
    """The table's initial-state draws on a workload whose drones start level
    (yaw-only attitudes): per drone, position, roll, pitch, yaw and velocity
    offsets uniform within DR_INIT."""
    rng = np.random.default_rng(seed)
    s = {k: v.copy() for k, v in w["state"].items()}
    n = s["p"].shape[1]
    assert np.all(s["q"][1:3] == 0), "level start expected"
    dp, da, dv = DR_INIT
    s["p"] += rng.uniform(-dp, dp, (3, n)).astype(np.float32)
    s["v"] += rng.uniform(-dv, dv, (3, n)).astype(np.float32)
    roll, pitch, dyaw = rng.uniform(-da, da, (3, n))
    yaw = 2.0 * np.arctan2(s["q"][3].astype(np.float64), s["q"][0].astype(np.float64)) + dyaw
    cr, sr = np.cos(0.5 * roll), np.sin(0.5 * roll)
    cp, sp = np.cos(0.5 * pitch), np.sin(0.5 * pitch)
    cy, sy = np.cos(0.5 * yaw), np.sin(0.5 * yaw)
    # q = q_z(yaw) q_y(pitch) q_x(roll), the ZYX convention of the observation
    s["q"] = np.stack([cr * cp * cy + sr * sp * sy, sr * cp * cy - cr * sp * sy,
                       cr * sp * cy + sr * cp * sy, cr * cp * sy - sr * sp * cy]).astype(np.float32)
    return dict(w, state=s)


def dr_wind(w, seed):
    """COMBINED wind with a per-environment mean wind (DR_WIND), as the
    keyword arguments of md_set_wind plus the per-drone array
    v_mean_drone [3][N] float32."""
    rng = np.random.default_rng(seed)
    off = np.asarray(w["env_offsets"], dtype=np.int64)
    m = np.diff(off)
    mag = rng.uniform(0.0, 1.0, len(m))
    head = rng.uniform(0.0, 2.0 * np.pi, len(m))
    vm = np.stack([np.repeat(mag * np.cos(head), m), np.repeat(mag * np.sin(head), m),
                   np.zeros(int(off[-1]))]).astype(np.float32)
    return dict(DR_WIND, seed=int(rng.integers(0, 2 ** 63)), v_mean_drone=vm)


def randomized(w, seed, latency_per="env"):
    """The workload under every row of the domain-randomisation table: the
    initial-state draws, the per-drone factors, motor lag, latencies,
    sensor noise and bias (domain_randomization) and the COMBINED wind with
    a per-environment mean (dr_wind).  Returns the workload dict with "dr"
    and "wind" entries."""
    out = perturb_initial_state(w, seed)
    out["dr"] = domain_randomization(w, seed + 1, latency_per=latency_per)
    out["wind"] = dr_wind(w, seed + 2)
    return out
