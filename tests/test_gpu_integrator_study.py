"""Euler against RK4, error per cost (the study that goes with the RK4 variant
of Table "Physics modes"): 0.5 s of PID flight of 64 two-layer lattices
(2x2x2, the surrogate's training geometry), on the GPU in float32 with the
semi-implicit Euler step at dt, dt/2, dt/4 and the classic RK4 step at dt,
each against the FP64 oracle's RK4 at dt/16.  The controller updates at the
same instants in every run (ctrl_decim scaled with the step).

With ground effect and drag the right-hand side is smooth: Euler converges
at first order and RK4 at dt is down to float32 rounding.  With the literal
downwash its gates (strict dz > 0, dxy < 10 m) make it discontinuous, so RK4
loses its order, yet it stays well below Euler at dt/4, which costs more
than RK4 at dt (the bench times the RK4 step at about three Euler steps)."""
import numpy as np
import pytest

import oracle as orc
import parity_util as pu
from paper_2606_08039_amd import workloads as wl

pytestmark = pytest.mark.gpu

T_END = 0.5


def _base():
    return wl.subset_envs(wl.lattice(n_envs=16384, shape=(2, 2, 2), seed=3), 64)


def _oracle_rk4(w, mask, k):
    P = pu.oracle_params()
    dt = w["dt"] / k
    s = pu.to_oracle_state(w["state"])
    orc.step(P, dt, mask, pu.ORC_ACT[w["act_type"]], w["ctrl_decim"] * k, w["env_offsets"], s,
             np.ascontiguousarray(w["action"][0:1], dtype=np.float64), False, int(round(T_END / dt)),
             integrator="rk4")
    return s["p"]


def _gpu(w, mask, integrator, k):
    wk = dict(w, dt=w["dt"] / k, ctrl_decim=w["ctrl_decim"] * k, integrator=integrator)
    g = pu.DeviceRun(wk, mask=mask)
    try:
        g.run(int(round(T_END / wk["dt"])))
        return g.snapshot()["p"].astype(np.float64)
    finally:
        g.close()


def _rms(p, ref):
    return float(np.sqrt(np.mean(np.sum((p - ref) ** 2, axis=0))))


@pytest.mark.parametrize("mask", [3, 7], ids=["gnd_drag", "gnd_drag_dw"])
def test_euler_first_order_and_rk4_more_accurate_per_cost(mask):
    w = _base()
    assert not w["action_per_step"]
    ref = _oracle_rk4(w, mask, 16)
    e = {("euler", k): _rms(_gpu(w, mask, "euler", k), ref) for k in (1, 2, 4)}
    e[("rk4", 1)] = _rms(_gpu(w, mask, "rk4", 1), ref)
    print("mask %d, rms position error after %.1f s against FP64 RK4 at dt/16: %s" % (
        mask, T_END, ", ".join("%s dt/%d %.2e m" % (i, k, v) for (i, k), v in e.items())))
    # semi-implicit Euler: first order
    for k in (1, 2):
        ratio = e[("euler", k)] / e[("euler", 2 * k)]
        assert 1.6 < ratio < 2.4, (k, ratio)
    # RK4 at dt (about three Euler steps of work) well below Euler at dt/4 (four)
    assert e[("rk4", 1)] < 0.25 * e[("euler", 4)], e
