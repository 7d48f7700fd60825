"""FP64 CPU oracle for the batched explicit quadrotor step -- TEST INFRASTRUCTURE.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``md_oracle.c`` (plain FP64
C, built with gcc) through ctypes and shares no code with the HIP library.
Each wrapper states the passage of the paper it follows; the readings of
silent passages are documented in ``md_oracle.c``.

Arrays are numpy float64 in the component-major SoA layout ``[c][N]``.
"""
import ctypes
import os

import numpy as np

from . import build_oracle

_HERE = os.path.dirname(os.path.abspath(__file__))

AERO_GND, AERO_DRAG, AERO_DW, AERO_SURROGATE = 1, 2, 4, 8
ACT_RPM, ACT_PID, ACT_VEL, ACT_ATTITUDE, ACT_DSL = 0, 1, 2, 3, 4
ACTION_ROWS = {ACT_RPM: 4, ACT_PID: 4, ACT_VEL: 4, ACT_ATTITUDE: 4, ACT_DSL: 7}
N_FEAT, K_NN = 64, 8


_D_T = ctypes.POINTER(ctypes.c_double)


class Params(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in (
        "m", "L", "kf", "km", "Ixx", "Iyy", "Izz", "thrust2weight", "r_p", "g",
        "C_gnd", "c_xy", "c_z", "C1", "C2", "C3", "dw_dz_min")] + [
        ("pos_kp", ctypes.c_double * 3), ("pos_ki", ctypes.c_double * 3),
        ("pos_kd", ctypes.c_double * 3), ("pos_i_clamp", ctypes.c_double),
        ("att_kp", ctypes.c_double * 3), ("att_ki", ctypes.c_double * 3),
        ("att_kd", ctypes.c_double * 3), ("att_i_clamp", ctypes.c_double),
        ("dsl_pos_kp", ctypes.c_double * 3), ("dsl_pos_ki", ctypes.c_double * 3),
        ("dsl_pos_kd", ctypes.c_double * 3), ("dsl_pos_i_clamp", ctypes.c_double),
        ("dsl_att_kp", ctypes.c_double * 3), ("dsl_att_ki", ctypes.c_double * 3),
        ("dsl_att_kd", ctypes.c_double * 3), ("dsl_att_i_clamp", ctypes.c_double),
        ("dsl_max_speed", ctypes.c_double), ("dsl_max_yaw_rate", ctypes.c_double)]

    def copy(self):
        o = Params()
        ctypes.memmove(ctypes.byref(o), ctypes.byref(self), ctypes.sizeof(Params))
        return o


class Derived(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("hover_rpm", "max_rpm", "max_thrust", "h_clip")]


class Net(ctypes.Structure):
    _fields_ = [("W", _D_T * 4), ("b", _D_T * 4), ("norm", _D_T), ("dz_ood", ctypes.c_double),
                ("ood_speed", ctypes.c_double), ("ood_rel_speed", ctypes.c_double), ("ood_tilt", ctypes.c_double),
                ("near_dz", ctypes.c_double), ("near_r", ctypes.c_double), ("far_dz", ctypes.c_double)]


class _CState(ctypes.Structure):
    _fields_ = [(n, ctypes.POINTER(ctypes.c_double)) for n in ("p", "q", "v", "w", "pid_int", "rpm", "ctl",
                                                               "rpm_cmd", "act_hist")] + \
        [("act_count", ctypes.POINTER(ctypes.c_int32)), ("wind", ctypes.POINTER(ctypes.c_double)),
         ("obs_hist", ctypes.POINTER(ctypes.c_double)), ("obs_count", ctypes.POINTER(ctypes.c_int32))]


class _CWind(ctypes.Structure):
    _fields_ = [("models", ctypes.c_uint32), ("v_mean", ctypes.c_double * 3), ("rho", ctypes.c_double),
                ("cd_area", ctypes.c_double), ("gust_prob", ctypes.c_double),
                ("gust_duration", ctypes.c_double), ("gust_amp", ctypes.c_double),
                ("dryden_sigma", ctypes.c_double), ("dryden_airspeed", ctypes.c_double),
                ("sin_amp", ctypes.c_double), ("sin_omega", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("drone_id", ctypes.POINTER(ctypes.c_int32)), ("v_mean_drone", ctypes.POINTER(ctypes.c_double))]


WIND_CONSTANT, WIND_GUST, WIND_DRYDEN, WIND_SINUSOIDAL = 1, 2, 4, 8
WIND_COMBINED = 15


class _CDr(ctypes.Structure):
    _fields_ = [("scale", ctypes.POINTER(ctypes.c_double)), ("tau_mot", ctypes.POINTER(ctypes.c_double)),
                ("delay", ctypes.POINTER(ctypes.c_int32)), ("noise_p", ctypes.c_double),
                ("noise_v", ctypes.c_double), ("noise_rpy", ctypes.c_double), ("noise_w", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("obs_delay", ctypes.POINTER(ctypes.c_int32)),
                ("drone_id", ctypes.POINTER(ctypes.c_int32)), ("obs_bias", ctypes.POINTER(ctypes.c_double))]


# Domain randomisation factor rows (orc_dr.scale) and the latency ring depth.
DR_ROWS = ("m", "J", "L", "kf", "km", "drag", "C_gnd", "C1", "max_rpm", "g",
           "bias0", "bias1", "bias2", "bias3")
DR_HIST = 32
DR_OBS_HIST = 8


_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_I32 = ctypes.POINTER(ctypes.c_int32)


_native_path = None


def load_native(directory):
    """Build the oracle with -march=native for this host into directory and
    use that build for every later call of this process (the CPU baseline of
    bench.py: the same C code, compiled for the CPU it is timed on).  Must
    run before any other oracle call.  Returns the command line's flags."""
    global _native_path
    if _lib is not None:
        raise RuntimeError("oracle already loaded")
    os.makedirs(directory, exist_ok=True)
    _native_path = build_oracle.build(native=True, dst=os.path.join(directory, "liboracle_native.so"))
    return " ".join(["gcc"] + build_oracle.FLAGS + ["-march=native"])


def _load():
    global _lib
    if _lib is not None:
        return _lib
    path = _native_path or build_oracle.LIB
    src = os.path.join(_HERE, "md_oracle.c")
    if _native_path is None and ((not os.path.exists(path)) or os.path.getmtime(path) < os.path.getmtime(src)):
        build_oracle.build()
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER(Params)
    lib.orc_params_cf2x.argtypes = [P]
    lib.orc_derive.argtypes = [P, ctypes.POINTER(Derived)]
    lib.orc_quat_to_rot.argtypes = [_D, _D]
    lib.orc_quat_mul.argtypes = [_D, _D, _D]
    lib.orc_euler_zyx.argtypes = [_D, _D]
    lib.orc_motor.argtypes = [P, _D, _D, _D, _D]
    lib.orc_ground_effect.argtypes = [P, ctypes.POINTER(Derived), _D, ctypes.c_double, _D]
    lib.orc_ground_effect.restype = ctypes.c_double
    lib.orc_drag.argtypes = [P, _D, _D, _D, _D]
    lib.orc_downwash_pair.argtypes = [P, _D, _D]
    lib.orc_downwash_pair.restype = ctypes.c_double
    lib.orc_pid.argtypes = [P, ctypes.POINTER(Derived), ctypes.c_double, _D, _D, _D, _D, _D, _D, _D]
    lib.orc_integrate.argtypes = [P, ctypes.c_double, _D, _D, _D, _D, _D, _D]
    lib.orc_vel_ctrl.argtypes = [P, ctypes.POINTER(Derived), ctypes.c_double, _D, _D, _D, _D, _D, _D]
    lib.orc_att_ctrl.argtypes = [P, ctypes.POINTER(Derived), ctypes.c_double, _D, _D, _D, _D, _D]
    lib.orc_dsl_pid.argtypes = [P, ctypes.POINTER(Derived), ctypes.c_double, _D, _D, _D, _D, _D,
                                _D, _D, _D]
    lib.orc_step.argtypes = [P, ctypes.c_double, ctypes.c_uint32, ctypes.c_int, ctypes.c_int,
                             ctypes.c_int, _I32, ctypes.c_int, ctypes.POINTER(_CState), _D,
                             ctypes.c_int, _D, ctypes.c_int, ctypes.c_int, ctypes.c_int64,
                             ctypes.c_int]
    lib.orc_step.restype = ctypes.c_int
    lib.orc_step_rk4.argtypes = lib.orc_step.argtypes
    lib.orc_step_dr.argtypes = lib.orc_step.argtypes + [ctypes.POINTER(_CDr)]
    lib.orc_step_dr.restype = ctypes.c_int
    lib.orc_step_disturbed.argtypes = lib.orc_step_dr.argtypes + [ctypes.POINTER(_CWind)]
    lib.orc_step_disturbed.restype = ctypes.c_int
    lib.orc_philox4x32.argtypes = [ctypes.POINTER(ctypes.c_uint32)] * 3
    lib.orc_philox4x32.restype = None
    lib.orc_step_rk4.restype = ctypes.c_int
    lib.orc_knn.argtypes = [ctypes.c_int, _I32, ctypes.c_int, _D, ctypes.c_int, _I32]
    lib.orc_features.argtypes = [P, ctypes.c_int, _I32, ctypes.c_int, ctypes.POINTER(_CState),
                                 _I32, ctypes.c_int, ctypes.c_int, _D]
    lib.orc_aero_residual.argtypes = [P, ctypes.c_uint32, ctypes.c_int, _I32, ctypes.c_int,
                                      ctypes.POINTER(_CState), _D, _D]
    lib.orc_mlp_forward.argtypes = [ctypes.c_int, _I32, ctypes.POINTER(_D), ctypes.POINTER(_D),
                                    ctypes.c_int, _D, _D, _D, ctypes.c_int]
    lib.orc_mlp_backward.argtypes = [ctypes.c_int, _I32, ctypes.POINTER(_D), ctypes.POINTER(_D),
                                     ctypes.c_int, _D, _D, _D, ctypes.POINTER(_D),
                                     ctypes.POINTER(_D), _D]
    lib.orc_adam.argtypes = [ctypes.c_int, _D, _D, _D, _D, ctypes.c_double, ctypes.c_double,
                             ctypes.c_double, ctypes.c_double, ctypes.c_int64]
    lib.orc_step_surrogate.argtypes = [P, ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                       _I32, ctypes.c_int, ctypes.POINTER(_CState), _D, ctypes.c_int,
                                       _D, ctypes.c_int, ctypes.c_int, ctypes.c_int64,
                                       ctypes.POINTER(Net), _D, _I32, ctypes.c_int]
    lib.orc_step_surrogate.restype = ctypes.c_int
    lib.orc_bf16_round.argtypes = [ctypes.c_double]
    lib.orc_bf16_round.restype = ctypes.c_double
    _lib = lib
    return lib


def _dp(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def _ip(a):
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(_I32)


def _vec(x, n):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(n))
    return a


# --------------------------------------------------------------------------
# Constants (Table "Drone model parameters", Eq. (6) coefficients, Table
# "Default PIDControl gains"; readings in md_oracle.c).
# --------------------------------------------------------------------------

def cf2x():
    P = Params()
    _load().orc_params_cf2x(ctypes.byref(P))
    return P


def derive(P):
    D = Derived()
    _load().orc_derive(ctypes.byref(P), ctypes.byref(D))
    return D


# --------------------------------------------------------------------------
# Per-drone building blocks.
# --------------------------------------------------------------------------

def quat_to_rot(q):
    q = _vec(q, 4)
    R = np.zeros(9)
    _load().orc_quat_to_rot(_dp(q), _dp(R))
    return R.reshape(3, 3)


def quat_mul(a, b):
    a, b = _vec(a, 4), _vec(b, 4)
    o = np.zeros(4)
    _load().orc_quat_mul(_dp(a), _dp(b), _dp(o))
    return o


def euler_zyx(q):
    q = _vec(q, 4)
    o = np.zeros(3)
    _load().orc_euler_zyx(_dp(q), _dp(o))
    return o


def motor(P, n):
    """Eq. (1)-(3): returns (F[4], T, tau_body[3])."""
    n = _vec(n, 4)
    F, T, tau = np.zeros(4), ctypes.c_double(0.0), np.zeros(3)
    _load().orc_motor(ctypes.byref(P), _dp(n), _dp(F), ctypes.byref(T), _dp(tau))
    return F, T.value, tau


def ground_effect(P, n, pz, q):
    """Eq. (4): extra world +z force."""
    D = derive(P)
    n, q = _vec(n, 4), _vec(q, 4)
    return _load().orc_ground_effect(ctypes.byref(P), ctypes.byref(D), _dp(n), float(pz), _dp(q))


def drag(P, n, q, v):
    """Eq. (5): drag force in the world frame."""
    n, q, v = _vec(n, 4), _vec(q, 4), _vec(v, 3)
    F = np.zeros(3)
    _load().orc_drag(ctypes.byref(P), _dp(n), _dp(q), _dp(v), _dp(F))
    return F


def downwash_pair(P, p_low, p_other):
    """Eq. (6): world-z force on the drone at p_low from the drone at p_other."""
    a, b = _vec(p_low, 3), _vec(p_other, 3)
    return _load().orc_downwash_pair(ctypes.byref(P), _dp(a), _dp(b))


def pid(P, dt_c, p, q, v, w, target, integ):
    """Sec. "Control": cascaded PID; returns (rpm[4], new integrals[6])."""
    D = derive(P)
    p, q, v, w, t = _vec(p, 3), _vec(q, 4), _vec(v, 3), _vec(w, 3), _vec(target, 4)
    I = _vec(integ, 6).copy()
    n = np.zeros(4)
    _load().orc_pid(ctypes.byref(P), ctypes.byref(D), float(dt_c), _dp(p), _dp(q), _dp(v),
                    _dp(w), _dp(t), _dp(I), _dp(n))
    return n, I


def vel_ctrl(P, dt_c, q, v, w, cmd, integ):
    """VEL action controller (readings in md_oracle.c); returns (rpm, integrals)."""
    D = derive(P)
    q, v, w, c = _vec(q, 4), _vec(v, 3), _vec(w, 3), _vec(cmd, 4)
    I = _vec(integ, 6).copy()
    n = np.zeros(4)
    _load().orc_vel_ctrl(ctypes.byref(P), ctypes.byref(D), float(dt_c), _dp(q), _dp(v), _dp(w),
                         _dp(c), _dp(I), _dp(n))
    return n, I


def att_ctrl(P, dt_c, q, w, cmd, integ):
    """ATTITUDE action controller; returns (rpm, integrals)."""
    D = derive(P)
    q, w, c = _vec(q, 4), _vec(w, 3), _vec(cmd, 4)
    I = _vec(integ, 6).copy()
    n = np.zeros(4)
    _load().orc_att_ctrl(ctypes.byref(P), ctypes.byref(D), float(dt_c), _dp(q), _dp(w), _dp(c),
                         _dp(I), _dp(n))
    return n, I


def dsl_pid(P, dt_c, p, q, v, w, cmd, integ, sp):
    """DSL-style PID; returns (rpm, integrals, setpoint)."""
    D = derive(P)
    p, q, v, w, c = _vec(p, 3), _vec(q, 4), _vec(v, 3), _vec(w, 3), _vec(cmd, 7)
    I = _vec(integ, 6).copy()
    S = _vec(sp, 4).copy()
    n = np.zeros(4)
    _load().orc_dsl_pid(ctypes.byref(P), ctypes.byref(D), float(dt_c), _dp(p), _dp(q), _dp(v),
                        _dp(w), _dp(c), _dp(I), _dp(S), _dp(n))
    return n, I, S


def integrate(P, dt, Fw, tau, p, q, v, w):
    """Sec. "Physics Modes": semi-implicit Euler + exponential map."""
    Fw, tau = _vec(Fw, 3), _vec(tau, 3)
    p, q, v, w = _vec(p, 3).copy(), _vec(q, 4).copy(), _vec(v, 3).copy(), _vec(w, 3).copy()
    _load().orc_integrate(ctypes.byref(P), float(dt), _dp(Fw), _dp(tau), _dp(p), _dp(q),
                          _dp(v), _dp(w))
    return p, q, v, w


# --------------------------------------------------------------------------
# Batched step.
# --------------------------------------------------------------------------

STATE_ROWS = {"p": 3, "q": 4, "v": 3, "w": 3, "pid_int": 6, "rpm": 4, "ctl": 4}


def new_state(n):
    s = {k: np.zeros((r, n)) for k, r in STATE_ROWS.items()}
    s["q"][0] = 1.0
    return s


def _cstate(s):
    for k in STATE_ROWS:
        if k == "ctl" and k not in s:
            continue
        assert s[k].dtype == np.float64 and s[k].flags.c_contiguous, k
    for k in ("rpm_cmd", "act_hist", "wind", "obs_hist"):
        if k in s:
            assert s[k].dtype == np.float64 and s[k].flags.c_contiguous, k
    for k in ("act_count", "obs_count"):
        if k in s:
            assert s[k].dtype == np.int32 and s[k].flags.c_contiguous, k
    return _CState(*([s[k].ctypes.data_as(_D) if k in s else None
                      for k in ("p", "q", "v", "w", "pid_int", "rpm", "ctl", "rpm_cmd", "act_hist")] +
                     [s["act_count"].ctypes.data_as(_I32) if "act_count" in s else None,
                      s["wind"].ctypes.data_as(_D) if "wind" in s else None,
                      s["obs_hist"].ctypes.data_as(_D) if "obs_hist" in s else None,
                      s["obs_count"].ctypes.data_as(_I32) if "obs_count" in s else None]))


def dr_state(state, act_type):
    """Add the blocks the randomised step needs to a state dict: the held
    controller command (= the state's rotor speeds), an empty action ring and
    zero counts."""
    n = state["p"].shape[1]
    state["rpm_cmd"] = state["rpm"].copy()
    state["act_hist"] = np.zeros((DR_HIST, ACTION_ROWS[act_type], n))
    state["act_count"] = np.zeros(n, dtype=np.int32)
    state["obs_hist"] = np.zeros((DR_OBS_HIST, 20, n))
    state["obs_count"] = np.zeros(n, dtype=np.int32)
    return state


def wind_state(state):
    """Add the wind block to a state dict: Dryden velocity 0, gusts idle."""
    n = state["p"].shape[1]
    state["wind"] = np.zeros((5, n))
    state["wind"][3] = -1.0
    return state


def philox4x32(ctr, key):
    c = (ctypes.c_uint32 * 4)(*[int(x) & 0xffffffff for x in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(x) & 0xffffffff for x in key])
    o = (ctypes.c_uint32 * 4)()
    _load().orc_philox4x32(c, k, o)
    return [o[i] for i in range(4)]


def make_wind(models, v_mean=(0.0, 0.0, 0.0), rho=1.225, cd_area=0.01, gust_prob=0.0, gust_duration=0.5,
              gust_amp=0.0, dryden_sigma=0.0, dryden_airspeed=1.0, sin_amp=0.0, sin_omega=0.0, seed=0,
              drone_id=None, v_mean_drone=None):
    """drone_id: optional int32 [N], the first Philox counter word of each
    drone (default its index), so that a sub-batch keeps its drones' draws;
    v_mean_drone: optional [3][N] per-drone mean wind (default v_mean)."""
    ids = np.ascontiguousarray(drone_id, dtype=np.int32) if drone_id is not None else None
    vmd = np.ascontiguousarray(v_mean_drone, dtype=np.float64) if v_mean_drone is not None else None
    w = _CWind(int(models), (ctypes.c_double * 3)(*v_mean), rho, cd_area, gust_prob, gust_duration,
               gust_amp, dryden_sigma, dryden_airspeed, sin_amp, sin_omega, int(seed),
               ids.ctypes.data_as(_I32) if ids is not None else None,
               vmd.ctypes.data_as(_D) if vmd is not None else None)
    w._keep = (ids, vmd)
    return w


def step(P, dt, aero_mask, act_type, ctrl_decim, env_offsets, state, action,
         action_per_step, n_steps, step0=0, n_obs_slots=0, n_threads=0, integrator="euler",
         dr=None, wind=None):
    """Advance ``state`` (dict of [c][N] float64 arrays, updated in place) by
    n_steps with the semi-implicit Euler step or classic RK4; returns the
    observation array [slots][20][N] or None.  dr: None, or a dict with
    "scale" [len(DR_ROWS)][N] and optional "tau_mot" [N] (s), "delay" [N]
    (int steps), "noise" (sigma_p, sigma_v, sigma_rpy, sigma_w), "seed",
    "obs_delay" [N] (int steps), "drone_id" [N] (Philox counter word) and
    "obs_bias" [12][N] (sticky bias on the p, v, rpy, w rows) for the
    domain-randomised Euler step."""
    off = np.ascontiguousarray(np.asarray(env_offsets, dtype=np.int32))
    n_envs = len(off) - 1
    n = int(off[-1])
    act = np.ascontiguousarray(np.asarray(action, dtype=np.float64))
    need = (n_steps if action_per_step else 1) * ACTION_ROWS[act_type] * n
    assert act.size == need, (act.size, need)
    obs = np.zeros((n_obs_slots, 20, n)) if n_obs_slots > 0 else None
    cs = _cstate(state)
    args = (ctypes.byref(P), float(dt), int(aero_mask), int(act_type),
            int(ctrl_decim), n_envs, _ip(off), n, ctypes.byref(cs), _dp(act),
            int(bool(action_per_step)), _dp(obs) if obs is not None else None,
            int(n_obs_slots), int(n_steps), int(step0), int(n_threads))
    if dr is not None or wind is not None:
        assert integrator == "euler"
        cdr = None
        if dr is not None:
            sc = np.ascontiguousarray(dr["scale"], dtype=np.float64)
            assert sc.shape == (len(DR_ROWS), n), sc.shape
            tau = np.ascontiguousarray(dr["tau_mot"], dtype=np.float64) if dr.get("tau_mot") is not None else None
            dl = np.ascontiguousarray(dr["delay"], dtype=np.int32) if dr.get("delay") is not None else None
            od = np.ascontiguousarray(dr["obs_delay"], dtype=np.int32) if dr.get("obs_delay") is not None else None
            ids = np.ascontiguousarray(dr["drone_id"], dtype=np.int32) if dr.get("drone_id") is not None else None
            bias = np.ascontiguousarray(dr["obs_bias"], dtype=np.float64) if dr.get("obs_bias") is not None else None
            assert bias is None or bias.shape == (12, n), bias.shape
            nz = tuple(float(x) for x in (dr.get("noise") or (0.0, 0.0, 0.0, 0.0)))
            cdr = _CDr(_dp(sc), _dp(tau) if tau is not None else None,
                       dl.ctypes.data_as(_I32) if dl is not None else None, nz[0], nz[1], nz[2], nz[3],
                       int(dr.get("seed", 0)), od.ctypes.data_as(_I32) if od is not None else None,
                       ids.ctypes.data_as(_I32) if ids is not None else None,
                       _dp(bias) if bias is not None else None)
        rc = _load().orc_step_disturbed(*args, ctypes.byref(cdr) if cdr is not None else None,
                                        ctypes.byref(wind) if wind is not None else None)
    else:
        fn = _load().orc_step if integrator == "euler" else _load().orc_step_rk4
        rc = fn(*args)
    if rc != 0:
        raise ValueError("orc_step failed (%d)" % rc)
    return obs


# --------------------------------------------------------------------------
# Surrogate support.
# --------------------------------------------------------------------------

def knn(env_offsets, p, k=K_NN):
    off = np.ascontiguousarray(np.asarray(env_offsets, dtype=np.int32))
    n = int(off[-1])
    p = np.ascontiguousarray(p, dtype=np.float64)
    nbr = np.full((n, k), -1, dtype=np.int32)
    rc = _load().orc_knn(len(off) - 1, _ip(off), n, _dp(p), int(k), _ip(nbr))
    if rc != 0:
        raise MemoryError("orc_knn")
    return nbr


def features(P, env_offsets, state, nbr, n_feat=N_FEAT):
    off = np.ascontiguousarray(np.asarray(env_offsets, dtype=np.int32))
    n = int(off[-1])
    k = nbr.shape[1]
    X = np.zeros((n, n_feat))
    cs = _cstate(state)
    rc = _load().orc_features(ctypes.byref(P), len(off) - 1, _ip(off), n, ctypes.byref(cs),
                              _ip(np.ascontiguousarray(nbr, dtype=np.int32)), int(k),
                              int(n_feat), _dp(X))
    if rc != 0:
        raise ValueError("orc_features")
    return X


def aero_residual(P, aero_mask, env_offsets, state, rpm=None):
    off = np.ascontiguousarray(np.asarray(env_offsets, dtype=np.int32))
    n = int(off[-1])
    rpm = state["rpm"] if rpm is None else np.ascontiguousarray(rpm, dtype=np.float64)
    Y = np.zeros((n, 6))
    cs = _cstate(state)
    _load().orc_aero_residual(ctypes.byref(P), int(aero_mask), len(off) - 1, _ip(off), n,
                              ctypes.byref(cs), _dp(rpm), _dp(Y))
    return Y


def _ptrs(arrs):
    return (_D * len(arrs))(*[_dp(a) for a in arrs])


def mlp_forward(Ws, bs, X, bf16_acts=False):
    """Ws[l]: [out][in] float64; returns (Y, acts)."""
    dims = np.array([Ws[0].shape[1]] + [W.shape[0] for W in Ws], dtype=np.int32)
    Ws = [np.ascontiguousarray(W, dtype=np.float64) for W in Ws]
    bs = [np.ascontiguousarray(b, dtype=np.float64) for b in bs]
    X = np.ascontiguousarray(X, dtype=np.float64)
    B = X.shape[0]
    Y = np.zeros((B, dims[-1]))
    acts = np.zeros(int(sum(2 * B * d for d in dims[1:])))
    rc = _load().orc_mlp_forward(len(Ws), _ip(dims), _ptrs(Ws), _ptrs(bs), B, _dp(X), _dp(Y),
                                 _dp(acts), int(bool(bf16_acts)))
    if rc != 0:
        raise MemoryError("orc_mlp_forward")
    return Y, acts


def mlp_backward(Ws, bs, X, acts, dY, want_dx=False):
    dims = np.array([Ws[0].shape[1]] + [W.shape[0] for W in Ws], dtype=np.int32)
    Ws = [np.ascontiguousarray(W, dtype=np.float64) for W in Ws]
    bs = [np.ascontiguousarray(b, dtype=np.float64) for b in bs]
    X = np.ascontiguousarray(X, dtype=np.float64)
    dY = np.ascontiguousarray(dY, dtype=np.float64)
    B = X.shape[0]
    dWs = [np.zeros_like(W) for W in Ws]
    dbs = [np.zeros_like(b) for b in bs]
    dX = np.zeros_like(X) if want_dx else None
    rc = _load().orc_mlp_backward(len(Ws), _ip(dims), _ptrs(Ws), _ptrs(bs), B, _dp(X),
                                  _dp(acts), _dp(dY), _ptrs(dWs), _ptrs(dbs),
                                  _dp(dX) if dX is not None else None)
    if rc != 0:
        raise MemoryError("orc_mlp_backward")
    return dWs, dbs, dX


def adam(param, grad, m1, m2, lr, beta1, beta2, eps, t):
    for a in (param, grad, m1, m2):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    _load().orc_adam(param.size, _dp(param), _dp(grad), _dp(m1), _dp(m2), float(lr),
                     float(beta1), float(beta2), float(eps), int(t))


def bf16_round(x):
    f = _load().orc_bf16_round
    return np.vectorize(f, otypes=[np.float64])(np.asarray(x, dtype=np.float64))


def make_net(flat_params, norm, dz_ood, ood_speed=0.0, ood_rel_speed=0.0, ood_tilt=0.0,
             near_dz=0.0, near_r=0.0, far_dz=0.0):
    """The surrogate as the oracle evaluates it: weight matrices rounded to
    bfloat16 (as the in-step network stores them), biases and normalisation
    as given (float32 values), fallback thresholds as float32 values.
    Returns (Net, keepalive)."""
    flat = np.asarray(flat_params, dtype=np.float32).astype(np.float64)
    shapes = ((128, 64), (128,), (128, 128), (128,), (128, 128), (128,), (6, 128), (6,))
    parts, o = [], 0
    for sh in shapes:
        k = int(np.prod(sh))
        parts.append(flat[o:o + k].reshape(sh))
        o += k
    Ws = [np.ascontiguousarray(bf16_round(parts[2 * l])) for l in range(4)]
    bs = [np.ascontiguousarray(parts[2 * l + 1]) for l in range(4)]
    nrm = np.ascontiguousarray(np.asarray(norm, dtype=np.float32).astype(np.float64))
    net = Net()
    for l in range(4):
        net.W[l] = _dp(Ws[l])
        net.b[l] = _dp(bs[l])
    net.norm = _dp(nrm)
    net.dz_ood = float(np.float32(dz_ood))
    net.ood_speed = float(np.float32(ood_speed))
    net.ood_rel_speed = float(np.float32(ood_rel_speed))
    net.ood_tilt = float(ood_tilt)
    net.near_dz = float(np.float32(near_dz))
    net.near_r = float(np.float32(near_r))
    net.far_dz = float(np.float32(far_dz))
    return net, (Ws, bs, nrm)


def step_surrogate(P, dt, act_type, ctrl_decim, env_offsets, state, action, action_per_step,
                   n_steps, net, step0=0, n_obs_slots=0, n_threads=0):
    """Step with the learned residual (see orc_step_surrogate); returns
    (obs, aero_body[N][6] of the last step, fallback[N])."""
    off = np.ascontiguousarray(np.asarray(env_offsets, dtype=np.int32))
    n = int(off[-1])
    act = np.ascontiguousarray(np.asarray(action, dtype=np.float64))
    obs = np.zeros((n_obs_slots, 20, n)) if n_obs_slots > 0 else None
    aero = np.zeros((n, 6))
    fb = np.zeros(n, dtype=np.int32)
    cs = _cstate(state)
    rc = _load().orc_step_surrogate(ctypes.byref(P), float(dt), int(act_type), int(ctrl_decim),
                                    len(off) - 1, _ip(off), n, ctypes.byref(cs), _dp(act),
                                    int(bool(action_per_step)),
                                    _dp(obs) if obs is not None else None, int(n_obs_slots),
                                    int(n_steps), int(step0), ctypes.byref(net), _dp(aero),
                                    _ip(fb), int(n_threads))
    if rc != 0:
        raise ValueError("orc_step_surrogate failed (%d)" % rc)
    return obs, aero, fb
