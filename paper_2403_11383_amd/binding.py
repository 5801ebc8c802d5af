"""ctypes binding of libsbs.so (include/sbs.h), argument marshalling only.

Every step of a control tick runs in the HIP kernels of the library; this
module converts dicts and numpy arrays to the C structs, lends the library a
torch-allocated device arena and torch streams, and turns status codes into
exceptions.  If the library is not built, loading fails loudly: there is no
other execution path.
"""
from __future__ import annotations

import ctypes as C
import time
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsbs.so")

MPPI, ELITE, NAIVE = 0, 1, 2
METHODS = {"mppi": MPPI, "elite": ELITE, "naive": NAIVE}
FREQ_MODES = {"fixed": 0, "uniform": 1, "gaussian": 2, "set": 3}
PRECISIONS = {"fp32": 0, "fp64": 1}
MODES = {"direct": 0, "serving": 1}
FLAG_NONFINITE = 1

OK, EINVAL, ENOMEM, EAGAIN, ETIMEDOUT, EDEVICE, ECANCELED, ENOENT = 0, -1, -2, -3, -4, -5, -6, -7

EXPORTED = [
    "sbs_runtime_create", "sbs_runtime_destroy", "sbs_init_controller",
    "sbs_destroy_controller", "sbs_submit_tick", "sbs_submit_tick_noalloc", "sbs_submit_batch", "sbs_fetch_action", "sbs_fetch_actions", "sbs_fetch_ready",
    "sbs_plan_create", "sbs_plan_submit", "sbs_plan_destroy", "sbs_plan_set_tune",
    "sbs_plan_autotune", "sbs_get_state",
    "sbs_set_state", "sbs_export_state", "sbs_import_state", "sbs_set_debug", "sbs_debug_fetch",
    "sbs_debug_costs", "sbs_debug_noise", "sbs_stats",
    "sbs_set_timing", "sbs_timing", "sbs_timing_rollout", "sbs_timing_overhead", "sbs_set_rollout_lanes", "sbs_set_rollout_pairs", "sbs_set_rollout_noise", "sbs_set_serving_depth", "sbs_set_prefetch", "sbs_plant_step", "sbs_plant_step_wrench", "sbs_closed_loop_step", "sbs_last_error", "sbs_abi_version",
]


class SBSError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"sbs error {code}: {msg}")
        self.code = code


class ControllerCfg(C.Structure):
    _fields_ = [
        ("N", C.c_int32), ("H", C.c_int32), ("iterations", C.c_int32), ("method", C.c_int32),
        ("freq_mode", C.c_int32), ("friction_on", C.c_int32), ("precision", C.c_int32),
        ("knots", C.c_int32),
        ("dt", C.c_double), ("lam", C.c_double), ("elite_frac", C.c_double),
        ("mu_fric", C.c_double), ("rho", C.c_double), ("f_nominal", C.c_double),
        ("sigma_grf", C.c_double), ("sigma_f", C.c_double), ("sigma_min_grf", C.c_double),
        ("sigma_min_f", C.c_double), ("f_min", C.c_double), ("f_max", C.c_double),
        ("f_fixed", C.c_double), ("duty", C.c_double), ("mu_f0", C.c_double),
        ("mass", C.c_double), ("gravity", C.c_double), ("inertia", C.c_double * 3),
        ("hip", C.c_double * 12), ("Q", C.c_double * 12), ("R", C.c_double * 12),
        ("phase_offset", C.c_uint32 * 4), ("seed", C.c_uint64),
        ("f_set", C.c_double * 4), ("n_fset", C.c_int32), ("reserved1", C.c_int32),
    ]


class TickInput(C.Structure):
    _fields_ = [
        ("x0", C.c_double * 12), ("foot_pos", C.c_double * 12), ("p_ref0", C.c_double * 3),
        ("v_ref", C.c_double * 3), ("yaw_ref", C.c_double), ("phase_robot", C.c_uint32),
        ("reserved0", C.c_uint32),
    ]


class Action(C.Structure):
    _fields_ = [
        ("grf", C.c_double * 12), ("contact", C.c_int32 * 4), ("freq_hz", C.c_double),
        ("best_cost", C.c_double), ("q", C.c_uint32), ("flags", C.c_int32),
        ("tick", C.c_uint32), ("controller", C.c_int32), ("t_submit_ns", C.c_int64),
        ("t_launch_ns", C.c_int64), ("t_done_ns", C.c_int64), ("n_active", C.c_uint32),
        ("reserved0", C.c_uint32),
    ]


class Tune(C.Structure):
    _fields_ = [("lanes", C.c_int32), ("block", C.c_int32), ("unroll", C.c_int32),
                ("reserved", C.c_int32), ("tick_us", C.c_double)]


class PlantState(C.Structure):
    _fields_ = [
        ("x", C.c_double * 12), ("foot_pos", C.c_double * 12), ("contact", C.c_int32 * 4),
        ("phase", C.c_uint32), ("reserved0", C.c_uint32),
    ]


_lib = None


def lib():
    """Load the in-tree library; raise if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run paper_2403_11383_amd/build.py")
        L = C.CDLL(LIB_PATH)
        vp, u64, i32, u32 = C.c_void_p, C.c_uint64, C.c_int32, C.c_uint32
        L.sbs_runtime_create.argtypes = [vp, u64, vp, vp, i32, C.POINTER(vp)]
        L.sbs_runtime_destroy.argtypes = [vp]
        L.sbs_init_controller.argtypes = [vp, C.POINTER(ControllerCfg), C.POINTER(i32)]
        L.sbs_destroy_controller.argtypes = [vp, i32]
        L.sbs_submit_tick.argtypes = [vp, i32, C.POINTER(TickInput), C.POINTER(u64)]
        L.sbs_submit_tick_noalloc.argtypes = [vp, i32, C.POINTER(TickInput), C.POINTER(u64)]
        L.sbs_submit_batch.argtypes = [vp, i32, C.POINTER(i32), C.POINTER(TickInput), C.POINTER(u64)]
        L.sbs_fetch_action.argtypes = [vp, u64, C.POINTER(Action), C.c_int64]
        L.sbs_fetch_actions.argtypes = [vp, i32, vp, C.POINTER(Action), C.c_int64]
        L.sbs_fetch_ready.argtypes = [vp, i32, vp, C.POINTER(Action), C.POINTER(i32), C.c_int64]
        L.sbs_plan_create.argtypes = [vp, i32, C.POINTER(i32), i32, C.POINTER(i32)]
        L.sbs_plan_submit.argtypes = [vp, i32, C.POINTER(TickInput), C.POINTER(u64)]
        L.sbs_plan_destroy.argtypes = [vp, i32]
        L.sbs_plan_set_tune.argtypes = [vp, i32, C.POINTER(Tune)]
        L.sbs_plan_autotune.argtypes = [vp, i32, C.POINTER(TickInput), i32, C.POINTER(Tune)]
        L.sbs_get_state.argtypes = [vp, i32, vp, C.POINTER(C.c_double), C.POINTER(u32)]
        L.sbs_set_state.argtypes = [vp, i32, vp, C.c_double, u32]
        L.sbs_export_state.argtypes = [vp, i32, vp, C.POINTER(C.c_double), C.POINTER(u32)]
        L.sbs_import_state.argtypes = [vp, i32, vp, C.c_double, u32]
        L.sbs_set_debug.argtypes = [vp, i32, i32]
        L.sbs_debug_costs.argtypes = [vp, i32, vp, vp, vp]
        L.sbs_timing_rollout.argtypes = [vp, i32, C.POINTER(C.c_double), C.POINTER(u64),
                                         C.POINTER(C.c_double)]
        L.sbs_debug_fetch.argtypes = [vp, i32, vp, vp, vp]
        L.sbs_debug_noise.argtypes = [vp, i32, u32, u32, vp, vp]
        L.sbs_stats.argtypes = [vp, C.POINTER(u64), C.POINTER(u64), C.POINTER(u64)]
        L.sbs_set_timing.argtypes = [vp, i32]
        L.sbs_timing.argtypes = [vp, vp, vp]
        L.sbs_timing_overhead.argtypes = [vp, i32, C.POINTER(C.c_double)]
        L.sbs_set_rollout_lanes.argtypes = [vp, i32]
        L.sbs_set_rollout_pairs.argtypes = [vp, i32]
        L.sbs_set_rollout_noise.argtypes = [vp, i32]
        L.sbs_set_serving_depth.argtypes = [vp, i32]
        L.sbs_set_prefetch.argtypes = [vp, i32, i32]
        L.sbs_plant_step.argtypes = [C.POINTER(ControllerCfg), C.POINTER(PlantState),
                                     C.POINTER(Action), vp, vp]
        L.sbs_plant_step_wrench.argtypes = [C.POINTER(ControllerCfg), C.POINTER(PlantState),
                                     C.POINTER(Action), vp, vp]
        L.sbs_closed_loop_step.argtypes = [vp, i32, C.POINTER(ControllerCfg), C.POINTER(PlantState),
                                           vp, vp, C.c_double, C.c_double, C.POINTER(Action)]
        L.sbs_last_error.restype = C.c_char_p
        L.sbs_abi_version.restype = i32
        for name in EXPORTED:
            if name not in ("sbs_last_error", "sbs_abi_version"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(rc: int):
    if rc != OK:
        raise SBSError(rc, lib().sbs_last_error().decode(errors="replace"))


def rows(d: dict) -> int:
    """Rows of the mean: the spline knot count, else the horizon."""
    k = int(d.get("knots", 0))
    return k if k > 0 else int(d["H"])


def make_cfg(d: dict) -> ControllerCfg:
    c = ControllerCfg()
    c.N, c.H, c.iterations = int(d["N"]), int(d["H"]), int(d.get("iterations", 1))
    c.method = METHODS[d.get("method", "mppi")]
    c.freq_mode = FREQ_MODES[d.get("freq_mode", "fixed")]
    c.friction_on = 1 if d.get("friction_on", False) else 0
    c.precision = PRECISIONS[d.get("precision", "fp32")]
    c.knots = int(d.get("knots", 0))
    c.dt, c.lam = float(d["dt"]), float(d.get("lambda", 1.0))
    c.elite_frac, c.mu_fric = float(d.get("elite_frac", 0.1)), float(d.get("mu_fric", 0.5))
    c.rho, c.f_nominal = float(d.get("rho", 0.0)), float(d.get("f_nominal", 1.4))
    c.sigma_grf, c.sigma_f = float(d["sigma_grf"]), float(d.get("sigma_f", 0.0))
    c.sigma_min_grf = float(d.get("sigma_min_grf", 1.0))
    c.sigma_min_f = float(d.get("sigma_min_f", 0.05))
    c.f_min, c.f_max = float(d.get("f_min", 1.0)), float(d.get("f_max", 2.5))
    c.f_fixed, c.duty = float(d.get("f_fixed", 1.4)), float(d.get("duty", 0.5))
    c.mu_f0 = float(d.get("mu_f0", 1.4))
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


def make_input(d: dict) -> TickInput:
    i = TickInput()
    i.x0[:] = [float(v) for v in d["x0"]]
    i.foot_pos[:] = [float(v) for v in np.asarray(d["foot_pos"], dtype=np.float64).reshape(12)]
    i.p_ref0[:] = [float(v) for v in d.get("p_ref0", (0.0, 0.0, 0.35))]
    i.v_ref[:] = [float(v) for v in d.get("v_ref", (0.0, 0.0, 0.0))]
    i.yaw_ref = float(d.get("yaw_ref", 0.0))
    i.phase_robot = int(d.get("phase_robot", 0)) & 0xFFFFFFFF
    return i


def action_dict(a: Action) -> dict:
    return {
        "grf": np.array(a.grf[:]), "contact": np.array(a.contact[:], np.int32),
        "freq_hz": a.freq_hz, "best_cost": a.best_cost, "q": int(a.q), "flags": int(a.flags),
        "tick": int(a.tick), "controller": int(a.controller),
        "t_submit_ns": int(a.t_submit_ns), "t_launch_ns": int(a.t_launch_ns),
        "t_done_ns": int(a.t_done_ns), "n_active": int(a.n_active),
    }


class Runtime:
    """A runtime on one GPU.  The device arena is a torch uint8 tensor and
    the streams are torch streams; both stay alive as long as this object."""

    def __init__(self, arena_bytes: int = 1 << 30, mode: str = "direct", device: str = "cuda:0",
                 two_streams: bool = False):
        import torch
        self._torch = torch
        self.device = torch.device(device)
        torch.cuda.set_device(self.device)
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.Stream(self.device)
        self.stream2 = torch.cuda.Stream(self.device) if two_streams else None
        self.cfgs = {}
        self._plan_cfgs = {}
        h = C.c_void_p()
        _check(lib().sbs_runtime_create(
            C.c_void_p(self.arena.data_ptr()), C.c_uint64(self.arena.numel()),
            C.c_void_p(self.stream.cuda_stream),
            C.c_void_p(self.stream2.cuda_stream) if self.stream2 is not None else None,
            MODES[mode], C.byref(h)))
        self._h = h

    # -- lifecycle -----------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            _check(lib().sbs_runtime_destroy(self._h))
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- controllers -----------------------------------------------------------
    def init_controller(self, cfg: dict) -> int:
        c = make_cfg(cfg)
        i = C.c_int32()
        _check(lib().sbs_init_controller(self._h, C.byref(c), C.byref(i)))
        self.cfgs[i.value] = dict(cfg)
        return i.value

    def destroy_controller(self, cid: int):
        _check(lib().sbs_destroy_controller(self._h, cid))
        self.cfgs.pop(cid, None)

    # -- ticks -----------------------------------------------------------------
    def submit_tick(self, cid: int, inp: dict) -> int:
        t = C.c_uint64()
        i = make_input(inp)
        _check(lib().sbs_submit_tick(self._h, cid, C.byref(i), C.byref(t)))
        return t.value

    def submit_tick_noalloc(self, cid: int, inp: dict) -> int:
        """sbs_submit_tick with the step workspace in the library's static
        device scratch array (no arena memory, no allocation)."""
        t = C.c_uint64()
        i = make_input(inp)
        _check(lib().sbs_submit_tick_noalloc(self._h, cid, C.byref(i), C.byref(t)))
        return t.value

    def submit_batch(self, cids, inputs) -> list:
        n = len(cids)
        ids = (C.c_int32 * n)(*cids)
        ins = (TickInput * n)(*[make_input(x) for x in inputs])
        tks = (C.c_uint64 * n)()
        _check(lib().sbs_submit_batch(self._h, n, ids, ins, tks))
        return list(tks)

    def fetch(self, ticket: int, timeout_us: int = -1):
        a = Action()
        rc = lib().sbs_fetch_action(self._h, C.c_uint64(ticket), C.byref(a), timeout_us)
        if rc in (EAGAIN, ETIMEDOUT):
            return None
        _check(rc)
        return action_dict(a)

    def tick(self, cid: int, inp: dict) -> dict:
        return self.fetch(self.submit_tick(cid, inp))

    # -- plans -----------------------------------------------------------------
    def plan_create(self, cids, use_graph: bool = True) -> int:
        n = len(cids)
        ids = (C.c_int32 * n)(*cids)
        p = C.c_int32()
        _check(lib().sbs_plan_create(self._h, n, ids, 1 if use_graph else 0, C.byref(p)))
        self._plan_cfgs[p.value] = [self.cfgs[c] for c in cids]
        return p.value

    def plan_submit(self, plan: int, inputs) -> list:
        n = len(inputs)
        ins = (TickInput * n)(*[make_input(x) for x in inputs])
        tks = (C.c_uint64 * n)()
        self.plan_submit_raw(plan, ins, tks)
        return list(tks)

    def plan_submit_raw(self, plan: int, ins, tickets):
        """plan_submit with caller-built ctypes arrays (TickInput * n inputs,
        c_uint64 * n tickets), for loops that resubmit the same inputs; waits
        (on the host) while the previous replay is still finishing."""
        L = lib()
        while True:
            rc = L.sbs_plan_submit(self._h, plan, ins, tickets)
            if rc != EAGAIN:
                break
            time.sleep(0)
        _check(rc)

    def fetch_many(self, tickets, out, timeout_us: int = -1):
        """Fetch len(tickets) actions in one call into out (Action * n)."""
        n = len(tickets)
        rc = lib().sbs_fetch_actions(self._h, n, C.cast(tickets, C.c_void_p), out, timeout_us)
        _check(rc)
        return out

    def fetch_ready(self, max_n: int = 1024, timeout_us: int = 0):
        """Every completed tick at once: a list of (ticket, action dict)."""
        tks = (C.c_uint64 * max_n)()
        acts = (Action * max_n)()
        n = C.c_int32()
        _check(lib().sbs_fetch_ready(self._h, max_n, tks, acts, C.byref(n), int(timeout_us)))
        return [(int(tks[i]), action_dict(acts[i])) for i in range(n.value)]

    def plan_destroy(self, plan: int):
        _check(lib().sbs_plan_destroy(self._h, plan))

    def plan_set_tune(self, plan: int, lanes: int, block: int = 64, unroll: int = 1):
        t = Tune(lanes, block, unroll, 0, 0.0)
        _check(lib().sbs_plan_set_tune(self._h, plan, C.byref(t)))

    def plan_autotune(self, plan: int, inputs, reps: int = 3, cache_path: str | None = None):
        """Pick the fastest rollout form for the plan (device-timed trials that
        restore every controller's state).  With cache_path, a JSON file keyed
        by device, kernel build and the plan's (N, H, iterations, method,
        precision) multiset is consulted first and updated after tuning."""
        import json
        key = self._plan_key(plan)
        if cache_path and os.path.exists(cache_path):
            try:
                ent = json.load(open(cache_path)).get(key)
            except (OSError, ValueError):
                ent = None
            if ent:
                self.plan_set_tune(plan, ent["lanes"], ent["block"], ent["unroll"])
                return dict(ent, cached=True)
        n = len(inputs)
        ins = (TickInput * n)(*[make_input(x) for x in inputs])
        t = Tune()
        _check(lib().sbs_plan_autotune(self._h, plan, ins, int(reps), C.byref(t)))
        res = {"lanes": t.lanes, "block": t.block, "unroll": t.unroll, "tick_us": t.tick_us}
        if cache_path:
            doc = {}
            if os.path.exists(cache_path):
                try:
                    doc = json.load(open(cache_path))
                except (OSError, ValueError):
                    doc = {}
            doc[key] = res
            with open(cache_path, "w") as f:
                json.dump(doc, f, indent=1, sort_keys=True)
        return dict(res, cached=False)

    def _plan_key(self, plan: int) -> str:
        import hashlib
        members = sorted((int(c["N"]), int(c["H"]), rows(c), int(c.get("iterations", 1)),
                          str(c.get("method", "mppi")), str(c.get("precision", "fp32")))
                         for c in self._plan_cfgs[plan])
        h = hashlib.sha256(open(LIB_PATH, "rb").read()).hexdigest()[:12]
        dev = self._torch.cuda.get_device_name(self.device)
        return f"{dev}|{h}|" + hashlib.sha256(repr(members).encode()).hexdigest()[:16]

    # -- state -----------------------------------------------------------------
    def export_state(self, cid: int):
        mu = np.zeros((rows(self.cfgs[cid]), 12))
        mf = C.c_double()
        tk = C.c_uint32()
        _check(lib().sbs_export_state(self._h, cid, mu.ctypes.data, C.byref(mf), C.byref(tk)))
        return mu, mf.value, tk.value

    def import_state(self, cid: int, mu, mu_f: float, tick: int):
        m = np.ascontiguousarray(mu, dtype=np.float64).reshape(-1)
        assert m.size == 12 * rows(self.cfgs[cid])
        _check(lib().sbs_import_state(self._h, cid, m.ctypes.data, float(mu_f),
                                      int(tick) & 0xFFFFFFFF))

    get_state = export_state   # the C ABI's sbs_get_state / sbs_set_state
    set_state = import_state

    # -- debug taps --------------------------------------------------------------
    def set_debug(self, cid: int, on: bool = True):
        _check(lib().sbs_set_debug(self._h, cid, 1 if on else 0))

    def debug_fetch(self, cid: int):
        c = self.cfgs[cid]
        R, N = int(c.get("iterations", 1)), int(c["N"])
        J = np.zeros((R, N))
        q = np.zeros((R, N), np.uint32)
        mean = np.zeros((rows(c), 12))
        _check(lib().sbs_debug_costs(self._h, cid, J.ctypes.data, q.ctypes.data, mean.ctypes.data))
        return J, q, mean

    debug_costs = debug_fetch

    def debug_noise(self, cid: int, tick: int, r: int = 0):
        c = self.cfgs[cid]
        N = int(c["N"])
        z = np.zeros((N, rows(c), 12), np.float32)
        q = np.zeros(N, np.uint32)
        _check(lib().sbs_debug_noise(self._h, cid, tick, r, z.ctypes.data, q.ctypes.data))
        return z, q

    # -- statistics ----------------------------------------------------------------
    def stats(self):
        a, b, c = C.c_uint64(), C.c_uint64(), C.c_uint64()
        _check(lib().sbs_stats(self._h, C.byref(a), C.byref(b), C.byref(c)))
        return {"ticks": a.value, "batches": b.value, "admit_waits": c.value}

    def set_timing(self, mode: int = 1):
        """0 off; 1 the rollout kernel's own dispatch events on one launch in
        16; 2 event commands around every stage; 3 as 1 on every launch."""
        _check(lib().sbs_set_timing(self._h, int(mode)))

    def set_prefetch(self, cid: int, on: bool = True):
        """Produce each next tick's noise ahead of time on the second stream."""
        _check(lib().sbs_set_prefetch(self._h, cid, 1 if on else 0))

    def set_rollout_lanes(self, lanes: int = 0):
        """0 automatic, 1 one lane per sample, 4 one lane per leg."""
        _check(lib().sbs_set_rollout_lanes(self._h, int(lanes)))

    def set_rollout_pairs(self, on: bool = True):
        """Stance-pair one-lane rollouts for the diagonal trot at duty 1/2."""
        _check(lib().sbs_set_rollout_pairs(self._h, 1 if on else 0))

    def set_rollout_noise(self, mode=2):
        """Where the noise is made (sbs_set_rollout_noise): 0 (or False) a
        separate noise launch, 1 every row in the rollout, 2 (or True, the
        default) the stance legs' only where the form allows."""
        if mode is True:
            mode = 2
        elif mode is False:
            mode = 0
        _check(lib().sbs_set_rollout_noise(self._h, int(mode)))

    def set_serving_depth(self, depth: int):
        """Serving: batches in flight per stream (1 to 4)."""
        _check(lib().sbs_set_serving_depth(self._h, int(depth)))

    def timing(self):
        avg = np.zeros(4)
        n = np.zeros(4, np.uint64)
        _check(lib().sbs_timing(self._h, avg.ctypes.data, n.ctypes.data))
        return {"noise_ns": avg[0], "rollout_ns": avg[1], "select_ns": avg[2],
                "update_ns": avg[3], "launches": n.tolist()}

    def timing_rollout(self, form: int):
        """Timed rollout launches of one form (0 FP32 one lane, 1 FP32 four
        lanes, 2 FP64, 3 FP32 one lane drawing its noise rows, 4 FP32 one
        lane drawing its stance legs' noise) since the last call: average
        device time [ns], number of launches and the rollout-steps they
        covered."""
        avg, n, st = C.c_double(), C.c_uint64(), C.c_double()
        _check(lib().sbs_timing_rollout(self._h, int(form), C.byref(avg), C.byref(n), C.byref(st)))
        return {"avg_ns": avg.value, "launches": n.value, "steps": st.value}

    def timing_overhead_ns(self, reps: int = 64) -> float:
        """Interval that the start/stop events of an empty dispatch span [ns]."""
        v = C.c_double()
        _check(lib().sbs_timing_overhead(self._h, int(reps), C.byref(v)))
        return v.value


class Plant:
    """The simulated robot of closed-loop runs (host FP64, in the library)."""

    def __init__(self, cfg: dict, x0, foot_pos, phase: int = 0):
        self.cfg = make_cfg(cfg)
        self.st = PlantState()
        self.st.x[:] = [float(v) for v in x0]
        self.st.foot_pos[:] = [float(v) for v in np.asarray(foot_pos, np.float64).reshape(12)]
        self.st.phase = int(phase) & 0xFFFFFFFF
        self._ext = np.zeros(6)
        self._vref = np.zeros(3)

    def step(self, act: dict, ext_force=(0.0, 0.0, 0.0), v_ref=(0.0, 0.0, 0.0), ext_torque=None):
        """One plant step; ext_force [N] and ext_torque [N m] act on the CoM in
        the world frame (sbs_plant_step_wrench when a torque is given)."""
        a = Action()
        a.grf[:] = [float(v) for v in act["grf"]]
        a.contact[:] = [int(v) for v in act["contact"]]
        a.q = int(act["q"]) & 0xFFFFFFFF
        self._ext[:3] = ext_force
        self._ext[3:] = 0.0 if ext_torque is None else ext_torque
        self._vref[:] = v_ref
        fn = lib().sbs_plant_step if ext_torque is None else lib().sbs_plant_step_wrench
        _check(fn(C.byref(self.cfg), C.byref(self.st), C.byref(a), self._ext.ctypes.data,
                  self._vref.ctypes.data))

    @property
    def x(self):
        return np.array(self.st.x[:])

    @property
    def foot_pos(self):
        return np.array(self.st.foot_pos[:]).reshape(4, 3)

    @property
    def phase(self):
        return int(self.st.phase)


class ClosedLoop:
    """One controller driving a Plant: each step is one sbs_closed_loop_step
    call (tick input from the plant state, submit, wait for the action, one
    plant step under it and the external wrench), with preallocated C
    structs (for closed-loop runs and benchmarks)."""

    def __init__(self, rt: Runtime, cid: int, plant: Plant, v_ref=(0.0, 0.0, 0.0),
                 z_ref: float = 0.35, yaw_ref: float = 0.0):
        self.rt, self.cid, self.plant = rt, cid, plant
        self.z_ref = float(z_ref)
        self.yaw_ref = float(yaw_ref)
        self.act = Action()
        self.ext = np.zeros(6)
        self.vref = np.array([float(v) for v in v_ref])
        self._L = lib()

    def step(self, ext_force=(0.0, 0.0, 0.0), ext_torque=(0.0, 0.0, 0.0)) -> Action:
        self.ext[:3] = ext_force
        self.ext[3:] = ext_torque
        _check(self._L.sbs_closed_loop_step(
            self.rt._h, self.cid, C.byref(self.plant.cfg), C.byref(self.plant.st),
            self.ext.ctypes.data, self.vref.ctypes.data, self.z_ref, self.yaw_ref,
            C.byref(self.act)))
        return self.act
