"""Seeded synthetic workloads: controller configurations and tick inputs.

This module holds parameters and random draws only -- no step of the
controller's arithmetic -- so that the HIP path and the FP64 oracle can be
driven with identical inputs.

Model and workloads (the paper's MuJoCo/Aliengo runs are not reproducible
here; a single-rigid-body quadruped with these constants stands in for them):

* mass 21.5 kg, diagonal inertia (0.07, 0.26, 0.24) kg m^2, g = 9.81 m/s^2,
  hips at (+-0.24, +-0.13, 0) m in the body frame, feet on flat ground at
  z = 0 (the CoM starts 0.35 m above it), trot (FL/RR in phase, FR/RL half a
  cycle later), duty factor 0.5, dt = 0.02 s, Q = I (C1 and the disturbance
  study: Q_STIFF), R = 1e-4 I (quadratic cost of Sec. V with positive
  diagonal weights).
* ``c0``  plain MPPI, FP64, N=256, H=25, fixed trot 1.4 Hz, GRF noise 20 N,
  lambda = 1, no friction clip, reference velocity 0.3 m/s.
* ``c1``  MPPI with per-sample gait frequency ~ U[1.0, 2.5] Hz, FP32,
  N=10240, H=50, noise 10 N, lambda = 30, the stiff weights Q_STIFF,
  friction cone mu = 0.5, 100 receding-horizon ticks, 40 N lateral push from
  tick 30 (the shape of the paper's push test).
* ``c2``  elite (CEM-style) sampler, FP32, N=16384, H=50, 3 iterations per
  tick, top 10 %, Gaussian frequency (mean 1.4 Hz, std 0.4), reference
  velocity ~ U[-0.5, 0.5] m/s, 100 ticks.
* ``c3``  64 independent controllers, N log-uniform in [1024, 16384],
  H ~ U{20..60}, MPPI or elite by a fair coin, FP32.
* ``c4``  256 robots at 50 Hz Poisson arrivals, N in {2048, 4096, 8192},
  H in {25, 50}, MPPI with gait-frequency sampling, FP32, 10 s.
"""
from __future__ import annotations

import numpy as np

MASS = 21.5
GRAVITY = 9.81
INERTIA = (0.07, 0.26, 0.24)
HIP = ((0.24, 0.13, 0.0),    # FL, body-frame hip offsets from the CoM
       (0.24, -0.13, 0.0),   # FR
       (-0.24, 0.13, 0.0),   # RL
       (-0.24, -0.13, 0.0))  # RR
TROT_OFFSETS = (0, 1 << 31, 1 << 31, 0)
PACE_OFFSETS = (0, 1 << 31, 0, 1 << 31)
HEIGHT = 0.35
DT = 0.02
# state weights [p, Phi, v, omega] that hold the plant up in closed loop:
# height and attitude stiff (1000) against R = 1e-4 on the GRFs
Q_STIFF = (10.0, 10.0, 1000.0, 1000.0, 1000.0, 100.0, 10.0, 10.0, 10.0, 1.0, 1.0, 1.0)


def base_model() -> dict:
    return {
        "mass": MASS, "gravity": GRAVITY, "inertia": list(INERTIA),
        "hip": [list(h) for h in HIP], "phase_offset": list(TROT_OFFSETS),
        "duty": 0.5, "dt": DT, "Q": [1.0] * 12, "R": [1e-4] * 12,
        "sigma_min_grf": 1.0, "sigma_min_f": 0.05, "f_min": 1.0, "f_max": 2.5,
        "f_nominal": 1.4, "f_fixed": 1.4, "lambda": 1.0, "elite_frac": 0.1,
        "mu_fric": 0.5, "friction_on": False, "rho": 0.0, "sigma_f": 0.0,
        "iterations": 1, "method": "mppi", "freq_mode": "fixed", "precision": "fp32",
        "mu_f0": 1.4,
    }


def config(name: str, **over) -> dict:
    """Controller configuration of workload ``name`` (c0..c4) as a plain dict."""
    c = base_model()
    if name == "c0":
        c.update(N=256, H=25, precision="fp64", method="mppi", freq_mode="fixed",
                 sigma_grf=20.0, friction_on=False, rho=0.0, seed=0)
    elif name == "c1":
        # the closed loop's weights: height and attitude stiff against the GRF
        # effort, 10 N noise, lambda = 30 (with Q = I and 25 N the plant is not
        # held up and most benchmark episodes end in a fall)
        c.update(N=10240, H=50, precision="fp32", method="mppi", freq_mode="uniform",
                 sigma_grf=10.0, friction_on=True, mu_fric=0.5, rho=1.0, seed=1,
                 Q=list(Q_STIFF), **{"lambda": 30.0})
    elif name == "c2":
        c.update(N=16384, H=50, precision="fp32", method="elite", iterations=3,
                 elite_frac=0.1, freq_mode="gaussian", mu_f0=1.4, sigma_f=0.4,
                 sigma_grf=25.0, friction_on=True, mu_fric=0.5, rho=1.0, seed=2)
    elif name in ("c3", "c4"):
        c.update(N=2048, H=25, precision="fp32", method="mppi", freq_mode="uniform",
                 sigma_grf=25.0, friction_on=True, mu_fric=0.5, rho=1.0,
                 seed=3000 if name == "c3" else 4000)
    else:
        raise KeyError(name)
    c.update(over)
    return c


def initial_state(rng: np.random.Generator) -> list:
    """x0 = [p, Phi, v, omega]: standing at 0.35 m, level, and every velocity
    component uniform in [-0.3, 0.3]."""
    v = rng.uniform(-0.3, 0.3, size=3)
    w = rng.uniform(-0.3, 0.3, size=3)
    return [0.0, 0.0, HEIGHT, 0.0, 0.0, 0.0, *v.tolist(), *w.tolist()]


def feet_under_hips(x0) -> list:
    """World footholds straight below the hips of a level body at x0."""
    return [[float(x0[0]) + h[0], float(x0[1]) + h[1], 0.0] for h in HIP]


def tick_input(x0, v_ref=(0.3, 0.0, 0.0), p_ref0=None, phase_robot=0, yaw_ref=0.0,
               foot_pos=None) -> dict:
    if p_ref0 is None:
        p_ref0 = (float(x0[0]), float(x0[1]), HEIGHT)
    if foot_pos is None:
        foot_pos = feet_under_hips(x0)
    return {"x0": [float(v) for v in x0], "v_ref": [float(v) for v in v_ref],
            "p_ref0": [float(v) for v in p_ref0], "yaw_ref": float(yaw_ref),
            "phase_robot": int(phase_robot) & 0xFFFFFFFF,
            "foot_pos": [[float(c) for c in f] for f in foot_pos]}


def c0_input() -> dict:
    return tick_input(initial_state(np.random.default_rng(0)))


def c2_episode_vref(seed: int = 2) -> tuple:
    rng = np.random.default_rng(seed)
    return (float(rng.uniform(-0.5, 0.5)), 0.0, 0.0)


def c3_controllers(seed: int = 3, count: int = 64) -> list:
    """64 uneven controllers: N log-uniform on [1024, 16384], H ~ U{20..60},
    MPPI (1 iteration) or elite (3 iterations) by a fair coin."""
    rng = np.random.default_rng(seed)
    out = []
    for c in range(count):
        n = int(np.floor(np.exp(rng.uniform(np.log(1024), np.log(16384)))))
        h = int(rng.integers(20, 61))
        elite = bool(rng.integers(0, 2))
        cfg = config("c3", N=n, H=h, seed=3000 + c)
        if elite:
            cfg.update(method="elite", iterations=3, freq_mode="gaussian", sigma_f=0.4)
        out.append(cfg)
    return out


def c3_inputs(seed: int = 3, count: int = 64) -> list:
    rng = np.random.default_rng(seed + 1)
    return [tick_input(initial_state(rng)) for _ in range(count)]


def c4_fleet(seed: int = 4, robots: int = 256) -> list:
    rng = np.random.default_rng(seed)
    out = []
    for r in range(robots):
        n = int(rng.choice([2048, 4096, 8192]))
        h = int(rng.choice([25, 50]))
        out.append(config("c4", N=n, H=h, seed=4000 + r))
    return out


def c4_arrivals(seed: int = 4, robots: int = 256, rate_hz: float = 50.0,
                duration_s: float = 10.0) -> list:
    """Per-robot Poisson arrival times (exponential gaps with mean 1/rate)."""
    rng = np.random.default_rng(seed + 7)
    out = []
    for _ in range(robots):
        t, ts = 0.0, []
        while True:
            t += float(rng.exponential(1.0 / rate_hz))
            if t >= duration_s:
                break
            ts.append(t)
        out.append(ts)
    return out


# Closed-loop disturbance study in the shape of the paper's gait-adaptation
# test (Sec. V-C, Fig. 4): the robot trots with a lateral velocity command of
# 0.1 m/s; from 2 s a 40 N lateral push acts on the CoM for 3 s; an episode
# lasts 8 s (400 control ticks at 50 Hz).  The paper's cost weights are not
# given, so the study weights stiffen height and attitude against the GRF
# effort (a 5 cm height error then costs as much as a 158 N error in one GRF
# component).
STUDY_Q = list(Q_STIFF)
STUDY_TICKS = 400
STUDY_PUSH = (100, 250, 40.0)  # first tick, end tick, lateral force [N]
STUDY_VREF = (0.0, 0.1, 0.0)
STUDY_FSET = [1.4, 2.0, 2.4]   # f_n, 2.0, 2.4 Hz (Sec. V)


def study_config(method: str = "naive", adapt: bool = True, rho: float = 1.0,
                 **over) -> dict:
    """Controller of the disturbance study: best-sample (Alg. 3) or MPPI, one
    iteration per tick, N = 10240, H = 25 (0.5 s), 10 N GRF noise; with gait
    adaptation the frequency is drawn from the paper's set, without it the
    trot runs at f_n = 1.4 Hz."""
    c = config("c1", N=10240, H=25, sigma_grf=10.0, method=method, iterations=1, rho=rho,
               **{"lambda": 30.0})
    c["Q"] = list(STUDY_Q)
    c["R"] = [1e-4] * 12
    if adapt:
        c.update(freq_mode="set", f_set=list(STUDY_FSET))
    else:
        c.update(freq_mode="fixed", f_fixed=STUDY_FSET[0])
    c.update(over)
    return c


def fallen(x) -> bool:
    """Fall criterion of every closed-loop run: roll or pitch beyond 0.8 rad,
    CoM height outside (0.2, 0.6) m, or a non-finite state."""
    return not (abs(x[3]) < 0.8 and abs(x[4]) < 0.8 and 0.2 < x[2] < 0.6)  # NaN fails too


def study_wrench(t: int) -> np.ndarray:
    """External wrench [Fx, Fy, Fz, Tx, Ty, Tz] on the CoM at tick t."""
    w = np.zeros(6)
    if STUDY_PUSH[0] <= t < STUDY_PUSH[1]:
        w[1] = STUDY_PUSH[2]
    return w
