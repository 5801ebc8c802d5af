"""Python view of the FP64 CPU oracle (test infrastructure only).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  It compiles ``oracle.c`` with gcc into ``liboracle.so``
next to this file and exposes thin numpy wrappers.  It imports nothing from the
HIP product package; configurations arrive as plain dicts.

Parity pins and the one unpinned area are listed in ``oracle.h``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "oracle.c")

MPPI, ELITE, NAIVE = 0, 1, 2
FREQ_FIXED, FREQ_UNIFORM, FREQ_GAUSSIAN, FREQ_SET = 0, 1, 2, 3
FLAG_NONFINITE = 1
METHODS = {"mppi": MPPI, "elite": ELITE, "naive": NAIVE}
FREQ_MODES = {"fixed": FREQ_FIXED, "uniform": FREQ_UNIFORM, "gaussian": FREQ_GAUSSIAN,
              "set": FREQ_SET}


def build() -> str:
    """Compile the oracle (always; a stale library is never reused)."""
    tmp = LIB_PATH + ".tmp"
    cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
           "-shared", "-pthread", "-Wall", "-Wextra", "-Wno-unused-parameter",
           SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


class Cfg(C.Structure):
    _fields_ = [
        ("N", C.c_int32), ("H", C.c_int32), ("iterations", C.c_int32),
        ("method", C.c_int32), ("freq_mode", C.c_int32), ("friction_on", C.c_int32),
        ("knots", C.c_int32),
        ("dt", C.c_double), ("lam", C.c_double), ("elite_frac", C.c_double),
        ("mu_fric", C.c_double), ("rho", C.c_double), ("f_nominal", C.c_double),
        ("sigma_grf", C.c_double), ("sigma_f", C.c_double),
        ("sigma_min_grf", C.c_double), ("sigma_min_f", C.c_double),
        ("f_min", C.c_double), ("f_max", C.c_double), ("f_fixed", C.c_double),
        ("duty", C.c_double), ("mass", C.c_double), ("gravity", C.c_double),
        ("inertia", C.c_double * 3), ("hip", C.c_double * 12),
        ("Q", C.c_double * 12), ("R", C.c_double * 12),
        ("phase_offset", C.c_uint32 * 4), ("seed", C.c_uint64),
        ("f_set", C.c_double * 4), ("n_fset", C.c_int32),
    ]


class Input(C.Structure):
    _fields_ = [
        ("x0", C.c_double * 12), ("foot_pos", C.c_double * 12), ("p_ref0", C.c_double * 3), ("v_ref", C.c_double * 3),
        ("yaw_ref", C.c_double), ("phase_robot", C.c_uint32),
    ]


class Action(C.Structure):
    _fields_ = [
        ("grf", C.c_double * 12), ("contact", C.c_int32 * 4), ("freq_hz", C.c_double),
        ("q", C.c_uint32), ("best_cost", C.c_double), ("flags", C.c_int32),
    ]


_lib = None
_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_fp = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        L.orc_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
        L.orc_gauss_pair.argtypes = [C.c_uint32, C.c_uint32, _fp]
        L.orc_noise_step.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32,
                                     C.c_uint32, _fp]
        L.orc_q_of_freq.argtypes = [C.c_double, C.c_double]
        L.orc_q_of_freq.restype = C.c_uint32
        L.orc_freq_of_q.argtypes = [C.c_uint32, C.c_double]
        L.orc_freq_of_q.restype = C.c_double
        L.orc_freq_q.argtypes = [C.POINTER(Cfg), C.c_double, C.c_double, C.c_uint32,
                                 C.c_uint32, C.c_uint32]
        L.orc_freq_q.restype = C.c_uint32
        L.orc_contact.argtypes = [C.POINTER(Cfg), C.c_uint32, C.c_uint32, C.c_int32, _i32p]
        L.orc_contact.restype = C.c_int
        L.orc_friction_clip.argtypes = [_dp, C.c_double, _dp]
        L.orc_rotation.argtypes = [_dp, _dp]
        L.orc_euler_rate_matrix.argtypes = [_dp, _dp]
        L.orc_srbd_deriv.argtypes = [C.POINTER(Cfg), _dp, _dp, _dp, _dp]
        L.orc_foothold.argtypes = [C.POINTER(Cfg), _dp, C.c_uint32, _dp, C.c_int32, _dp]
        L.orc_knot_time.argtypes = [C.POINTER(Cfg), C.c_int32]
        L.orc_knot_time.restype = C.c_double
        L.orc_spline_eval.argtypes = [C.POINTER(Cfg), _dp, C.c_double, _dp]
        L.orc_rollout.argtypes = [C.POINTER(Cfg), C.POINTER(Input), _dp, C.c_uint32,
                                  C.c_void_p, C.c_void_p]
        L.orc_rollout.restype = C.c_double
        L.orc_mppi_weights.argtypes = [C.c_int32, _dp, C.c_double, _dp,
                                       C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.orc_mppi_weights.restype = C.c_int
        L.orc_weighted_mean.argtypes = [C.c_int32, C.c_int32, _dp, _dp, _dp]
        L.orc_elite_count.argtypes = [C.c_int32, C.c_double]
        L.orc_elite_count.restype = C.c_int32
        L.orc_elite_select.argtypes = [C.c_int32, _dp, C.c_int32, _i32p]
        L.orc_elite_moments.argtypes = [C.c_int32, C.c_int32, _i32p, _dp, _dp, _dp]
        L.orc_tick.argtypes = [C.POINTER(Cfg), _dp, C.POINTER(C.c_double), C.c_uint32,
                               C.POINTER(Input), C.POINTER(Action), C.c_void_p, C.c_void_p,
                               C.c_void_p, C.c_void_p, C.c_int32]
        L.orc_tick.restype = C.c_int
        _lib = L
    return _lib


# --------------------------------------------------------------------------
# marshalling from plain dicts
# --------------------------------------------------------------------------
def make_cfg(d: dict) -> Cfg:
    c = Cfg()
    c.N, c.H, c.iterations = int(d["N"]), int(d["H"]), int(d.get("iterations", 1))
    c.method = METHODS[d.get("method", "mppi")]
    c.freq_mode = FREQ_MODES[d.get("freq_mode", "fixed")]
    c.friction_on = 1 if d.get("friction_on", False) else 0
    c.knots = int(d.get("knots", 0))
    c.dt, c.lam = float(d["dt"]), float(d.get("lambda", 1.0))
    c.elite_frac, c.mu_fric = float(d.get("elite_frac", 0.1)), float(d.get("mu_fric", 0.5))
    c.rho, c.f_nominal = float(d.get("rho", 0.0)), float(d.get("f_nominal", 1.4))
    c.sigma_grf, c.sigma_f = float(d["sigma_grf"]), float(d.get("sigma_f", 0.0))
    c.sigma_min_grf = float(d.get("sigma_min_grf", 1.0))
    c.sigma_min_f = float(d.get("sigma_min_f", 0.05))
    c.f_min, c.f_max = float(d.get("f_min", 1.0)), float(d.get("f_max", 2.5))
    c.f_fixed, c.duty = float(d.get("f_fixed", 1.4)), float(d.get("duty", 0.5))
    c.mass, c.gravity = float(d["mass"]), float(d["gravity"])
    c.inertia[:] = [float(v) for v in d["inertia"]]
    c.hip[:] = [float(v) for v in np.asarray(d["hip"], dtype=np.float64).reshape(12)]
    c.Q[:] = [float(v) for v in d["Q"]]
    c.R[:] = [float(v) for v in d["R"]]
    c.phase_offset[:] = [int(v) & 0xFFFFFFFF for v in d["phase_offset"]]
    c.seed = int(d.get("seed", 0)) & 0xFFFFFFFFFFFFFFFF
    fs = [float(v) for v in d.get("f_set", ())]
    c.n_fset = len(fs)
    c.f_set[:] = (fs + [0.0] * 4)[:4]
    return c


def make_input(d: dict) -> Input:
    i = Input()
    i.x0[:] = [float(v) for v in d["x0"]]
    i.foot_pos[:] = [float(v) for v in np.asarray(d["foot_pos"], dtype=np.float64).reshape(12)]
    i.p_ref0[:] = [float(v) for v in d.get("p_ref0", (0.0, 0.0, 0.35))]
    i.v_ref[:] = [float(v) for v in d.get("v_ref", (0.0, 0.0, 0.0))]
    i.yaw_ref = float(d.get("yaw_ref", 0.0))
    i.phase_robot = int(d.get("phase_robot", 0)) & 0xFFFFFFFF
    return i


# --------------------------------------------------------------------------
# numpy wrappers
# --------------------------------------------------------------------------
def philox(ctr, key):
    out = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(np.asarray(ctr, np.uint32), np.asarray(key, np.uint32), out)
    return out


def gauss_pair(w0: int, w1: int):
    out = np.zeros(2, np.float32)
    lib().orc_gauss_pair(w0 & 0xFFFFFFFF, w1 & 0xFFFFFFFF, out)
    return out


def noise_step(seed, tick, r, k, j):
    z = np.zeros(12, np.float32)
    lib().orc_noise_step(seed, tick, r, k, j, z)
    return z


def noise_block(seed, tick, r, n, h):
    """z[k][j][d] for k < n, j < h (slow; small sizes only)."""
    z = np.zeros((n, h, 12), np.float32)
    for k in range(n):
        for j in range(h):
            z[k, j] = noise_step(seed, tick, r, k, j)
    return z


def q_of_freq(f, dt):
    return int(lib().orc_q_of_freq(f, dt))


def freq_of_q(q, dt):
    return float(lib().orc_freq_of_q(q, dt))


def freq_q(cfg: dict, mu_f, sigma_f, tick, r, k):
    c = make_cfg(cfg)
    return int(lib().orc_freq_q(C.byref(c), mu_f, sigma_f, tick, r, k))


def contact(cfg: dict, phase_robot, q, j):
    c = make_cfg(cfg)
    d = np.zeros(4, np.int32)
    n = lib().orc_contact(C.byref(c), phase_robot & 0xFFFFFFFF, q & 0xFFFFFFFF, j, d)
    return d, n


def friction_clip(f, mu):
    out = np.zeros(3)
    lib().orc_friction_clip(np.ascontiguousarray(f, np.float64), mu, out)
    return out


def rotation(phi):
    R = np.zeros(9)
    lib().orc_rotation(np.ascontiguousarray(phi, np.float64), R)
    return R.reshape(3, 3)


def euler_rate_matrix(phi):
    E = np.zeros(9)
    lib().orc_euler_rate_matrix(np.ascontiguousarray(phi, np.float64), E)
    return E.reshape(3, 3)


def srbd_deriv(cfg: dict, x, u, lever):
    c = make_cfg(cfg)
    xd = np.zeros(12)
    lib().orc_srbd_deriv(C.byref(c), np.ascontiguousarray(x, np.float64),
                         np.ascontiguousarray(u, np.float64).reshape(12),
                         np.ascontiguousarray(lever, np.float64).reshape(12), xd)
    return xd


def foothold(cfg: dict, x, q, v_ref, leg):
    c = make_cfg(cfg)
    out = np.zeros(3)
    lib().orc_foothold(C.byref(c), np.ascontiguousarray(x, np.float64), q & 0xFFFFFFFF,
                       np.ascontiguousarray(v_ref, np.float64), leg, out)
    return out


def rows(cfg: dict) -> int:
    """Rows of the GRF decision variable: the knot count, else H."""
    k = int(cfg.get("knots", 0))
    return k if k > 0 else int(cfg["H"])


def knot_time(cfg: dict, p: int) -> float:
    return float(lib().orc_knot_time(C.byref(make_cfg(cfg)), p))


def spline_eval(cfg: dict, theta, t: float):
    """The 12 GRFs of the spline through the knots theta [P][12] at time t."""
    out = np.zeros(12)
    lib().orc_spline_eval(C.byref(make_cfg(cfg)),
                          np.ascontiguousarray(theta, np.float64).reshape(-1), float(t), out)
    return out


def rollout(cfg: dict, inp: dict, theta, q, return_states=False):
    """J, or (J, states[H+1][12], footholds[H][4][3]) with return_states.
    theta is [H][12], or [P][12] knots for a spline configuration."""
    c, i = make_cfg(cfg), make_input(inp)
    th = np.ascontiguousarray(theta, np.float64).reshape(-1)
    assert th.size == 12 * rows(cfg)
    xs = np.zeros((c.H + 1, 12)) if return_states else None
    feet = np.zeros((c.H, 4, 3)) if return_states else None
    J = lib().orc_rollout(C.byref(c), C.byref(i), th, q & 0xFFFFFFFF,
                          xs.ctypes.data if xs is not None else None,
                          feet.ctypes.data if feet is not None else None)
    return (J, xs, feet) if return_states else J


def mppi_weights(J, lam):
    J = np.ascontiguousarray(J, np.float64)
    w = np.zeros_like(J)
    beta, Om = C.c_double(), C.c_double()
    flags = lib().orc_mppi_weights(J.size, J, lam, w, C.byref(beta), C.byref(Om))
    return w, beta.value, Om.value, flags


def weighted_mean(omega, theta):
    theta = np.ascontiguousarray(theta, np.float64)
    n, d = theta.shape
    out = np.zeros(d)
    lib().orc_weighted_mean(n, d, np.ascontiguousarray(omega, np.float64), theta, out)
    return out


def elite_count(n, frac):
    return int(lib().orc_elite_count(n, frac))


def elite_select(J, ke):
    J = np.ascontiguousarray(J, np.float64)
    idx = np.zeros(ke, np.int32)
    lib().orc_elite_select(J.size, J, ke, idx)
    return idx


def elite_moments(idx, theta):
    theta = np.ascontiguousarray(theta, np.float64)
    idx = np.ascontiguousarray(idx, np.int32)
    d = theta.shape[1]
    mean, var = np.zeros(d), np.zeros(d)
    lib().orc_elite_moments(idx.size, d, idx, theta, mean, var)
    return mean, var


def tick(cfg: dict, mu, mu_f, tick_no, inp: dict, nthreads=1, costs_override=None):
    """One control step.  Returns a dict with the action, the warm-started
    mean, the updated frequency mean, all costs and sampled increments."""
    c, i = make_cfg(cfg), make_input(inp)
    N, H, R = c.N, rows(cfg), c.iterations  # H: rows of the mean
    mu = np.array(mu, dtype=np.float64).reshape(-1).copy()
    assert mu.size == 12 * H
    mf = C.c_double(float(mu_f))
    act = Action()
    costs = np.zeros(R * N)
    mean = np.zeros(12 * H)
    qs = np.zeros(R * N, np.uint32)
    ov = None
    if costs_override is not None:
        ov = np.ascontiguousarray(costs_override, np.float64).reshape(-1)
        assert ov.size == R * N
    rc = lib().orc_tick(C.byref(c), mu, C.byref(mf), tick_no & 0xFFFFFFFF, C.byref(i),
                        C.byref(act), costs.ctypes.data,
                        ov.ctypes.data if ov is not None else None,
                        mean.ctypes.data, qs.ctypes.data, nthreads)
    if rc != 0:
        raise ValueError(f"oracle tick rejected its input (rc={rc})")
    return {
        "grf": np.array(act.grf[:]), "contact": np.array(act.contact[:], np.int32),
        "freq_hz": act.freq_hz, "q": act.q, "best_cost": act.best_cost,
        "flags": act.flags, "mu_next": mu.reshape(H, 12), "mu_f_next": mf.value,
        "mean": mean.reshape(H, 12), "costs": costs.reshape(R, N),
        "q_samples": qs.reshape(R, N),
    }
