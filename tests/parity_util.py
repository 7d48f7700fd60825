"""Helpers shared by the GPU parity tests: run a workload through libmd and
the same seeded inputs through the FP64 oracle, and compare block by block.

Per-step criterion (written here once): for every drone and every state block
(p, q, v, w, applied rotor speeds), ||gpu - oracle||_inf <= TOL *
max(||oracle||_inf, 1), the oracle having been stepped once in FP64 from the
GPU's own float32 pre-step state.
"""
import numpy as np

import oracle as orc
from paper_2606_08039_amd import md

TOL = 1e-5
BLOCKS = ("p", "q", "v", "w", "rpm")
ACT = {"rpm": md.MD_ACT_RPM, "pid": md.MD_ACT_PID, "vel": md.MD_ACT_VEL,
       "attitude": md.MD_ACT_ATTITUDE, "dsl": md.MD_ACT_DSL}
ORC_ACT = {"rpm": orc.ACT_RPM, "pid": orc.ACT_PID, "vel": orc.ACT_VEL,
           "attitude": orc.ACT_ATTITUDE, "dsl": orc.ACT_DSL}


def params():
    return md.md_default_params_cf2x()


def oracle_params():
    return orc.cf2x()


def hover_rpm():
    return md.md_derive(md.md_default_params_cf2x()).hover_rpm


class DeviceRun:
    """A libmd context plus device buffers for one workload dict."""

    def __init__(self, w, p=None, mask=None, cfg=None):
        import torch
        self.w = w
        self.p = p or params()
        self.mask = w["aero_mask"] if mask is None else mask
        self.ctx = md.md_create(self.p, w["dt"], self.mask, ACT[w["act_type"]], w["ctrl_decim"])
        if w.get("integrator", "euler") == "rk4":
            md.md_set_integrator(self.ctx, md.MD_INTEG_RK4)
        md.md_bind_layout(self.ctx, w["env_offsets"])
        if cfg is not None:
            md.md_set_launch_config(self.ctx, **cfg)
        self.n = int(w["env_offsets"][-1])
        self.state = md.DeviceState.from_numpy(w["state"])
        self.dr = None
        if w.get("dr") is not None:
            dr = w["dr"]
            self.dr = {k: (torch.from_numpy(dr[k]).cuda() if dr.get(k) is not None else None)
                       for k in ("scale", "tau_mot", "delay", "obs_delay", "obs_bias")}
            self.state.add_dr_blocks(ACT[w["act_type"]], w["state"])
            md.md_set_domain_randomization(self.ctx, self.dr["scale"], self.dr["tau_mot"], self.dr["delay"],
                                           noise=dr.get("noise", (0.0, 0.0, 0.0, 0.0)), seed=dr.get("seed", 0),
                                           obs_delay=self.dr["obs_delay"], obs_bias=self.dr["obs_bias"])
        self.wind_arrays = None
        if w.get("wind") is not None:
            self.state.add_wind_block(w["state"])
            wk = dict(w["wind"])
            if wk.get("v_mean_drone") is not None:
                self.wind_arrays = torch.from_numpy(np.ascontiguousarray(wk["v_mean_drone"], dtype=np.float32)).cuda()
                wk["v_mean_drone"] = self.wind_arrays
            md.md_set_wind(self.ctx, **wk)
        self.action = torch.from_numpy(np.ascontiguousarray(w["action"], dtype=np.float32)).cuda()
        self.step_index = 0

    def action_slice(self, k0, k):
        if self.w["action_per_step"]:
            return self.action[k0:k0 + k].contiguous()
        return self.action

    def run(self, k, obs_slots=0):
        import torch
        obs = torch.zeros((obs_slots, 20, self.n), dtype=torch.float32, device="cuda") \
            if obs_slots > 0 else None
        md.md_step(self.ctx, self.state, self.action_slice(self.step_index, k),
                   self.w["action_per_step"], obs, obs_slots, k, self.step_index)
        torch.cuda.synchronize()
        self.step_index += k
        return obs.cpu().numpy() if obs is not None else None

    def snapshot(self):
        return self.state.to_numpy()

    def close(self):
        md.md_destroy(self.ctx)


def to_oracle_state(s32):
    return {k: np.ascontiguousarray(v, dtype=np.int32 if k in ("act_count", "obs_count") else np.float64)
            for k, v in s32.items()}


def obs_to_state(o, prev=None):
    """State blocks carried by a KIN observation [20][N] (p, q, v, w, rpm)."""
    s = {"p": o[0:3], "q": o[3:7], "v": o[10:13], "w": o[13:16], "rpm": o[16:20]}
    n = o.shape[1]
    s["pid_int"] = prev["pid_int"] if prev is not None else np.zeros((6, n), dtype=o.dtype)
    s["ctl"] = prev["ctl"] if prev is not None and "ctl" in prev else np.zeros((4, n), dtype=o.dtype)
    return s


def oracle_one_step(w, s32, k, env_subset=None, mask=None, n_steps=1, obs_slots=0):
    """Step the oracle from a float32 GPU state for n_steps starting at global
    step k (action row k when actions are per step).  env_subset restricts the
    run to some environments (they are independent)."""
    P = oracle_params()
    off = np.asarray(w["env_offsets"], dtype=np.int64)
    act = w["action"]
    s = to_oracle_state(s32)
    if env_subset is not None:
        idx = np.concatenate([np.arange(off[e], off[e + 1]) for e in env_subset])
        m = np.array([off[e + 1] - off[e] for e in env_subset])
        sub_off = np.concatenate([[0], np.cumsum(m)]).astype(np.int32)
        s = {kk: np.ascontiguousarray(v[..., idx]) for kk, v in s.items()}
        act = act[:, :, idx]
    else:
        idx = None
        sub_off = np.asarray(off, dtype=np.int32)
    a = act[k:k + n_steps] if w["action_per_step"] else act[0:1]
    dr = None
    if w.get("dr") is not None:
        pick = (lambda v: v) if idx is None else (lambda v: v[..., idx])
        dr = {kk: (np.ascontiguousarray(pick(v)) if isinstance(v, np.ndarray) else v)
              for kk, v in w["dr"].items()}
        dr["scale"] = dr["scale"].astype(np.float64)
        # the GPU takes float32 noise levels; the draws of a sub-batch keep
        # the drones' indices in the whole batch
        dr["noise"] = tuple(float(np.float32(x)) for x in dr.get("noise", (0.0, 0.0, 0.0, 0.0)))
        if idx is not None:
            dr["drone_id"] = idx.astype(np.int32)
        if dr.get("tau_mot") is not None:
            dr["tau_mot"] = dr["tau_mot"].astype(np.float64)
    wind = None
    if w.get("wind") is not None:
        wk = dict(w["wind"])
        # the GPU takes float32 parameters; hand the oracle the same values
        f32 = lambda x: float(np.float32(x))
        for key in ("rho", "cd_area", "gust_prob", "gust_duration", "gust_amp", "dryden_sigma",
                    "dryden_airspeed", "sin_amp", "sin_omega"):
            if key in wk:
                wk[key] = f32(wk[key])
        if "v_mean" in wk:
            wk["v_mean"] = tuple(f32(x) for x in wk["v_mean"])
        if wk.get("v_mean_drone") is not None:
            vmd = np.asarray(wk["v_mean_drone"], dtype=np.float32).astype(np.float64)
            wk["v_mean_drone"] = vmd if idx is None else np.ascontiguousarray(vmd[:, idx])
        wind = orc.make_wind(**wk, drone_id=idx.astype(np.int32) if idx is not None else None)
    obs = orc.step(P, w["dt"], w["aero_mask"] if mask is None else mask,
                   ORC_ACT[w["act_type"]], w["ctrl_decim"],
                   sub_off, s, np.ascontiguousarray(a, dtype=np.float64), w["action_per_step"],
                   n_steps, step0=k, n_obs_slots=obs_slots,
                   integrator=w.get("integrator", "euler"), dr=dr, wind=wind)
    return s, obs, idx


def block_errors(gpu, ref, idx=None, blocks=BLOCKS):
    """Worst per-drone scaled error of each block."""
    out = {}
    for k in blocks:
        a = np.asarray(gpu[k], dtype=np.float64)
        if idx is not None:
            a = a[:, idx]
        b = np.asarray(ref[k], dtype=np.float64)
        scale = np.maximum(np.max(np.abs(b), axis=0), 1.0)
        err = np.max(np.abs(a - b), axis=0) / scale
        out[k] = float(err.max()) if err.size else 0.0
    return out


def assert_blocks(gpu, ref, idx=None, tol=TOL, blocks=BLOCKS, what=""):
    e = block_errors(gpu, ref, idx, blocks)
    bad = {k: v for k, v in e.items() if not v <= tol}
    assert not bad, "%s per-step error above %g: %s (all %s)" % (what, tol, bad, e)
    return e
