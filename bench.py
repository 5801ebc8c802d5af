"""Benchmark of one GPU: closed-loop receding-horizon MPPI with per-sample gait
frequency (N = 10240 samples, H = 50 steps, dt = 0.02 s, GRF noise 25 N,
friction cone mu = 0.5, 40 N lateral push from tick 30), FP32 rollouts.

A step is one control tick: noise, rollouts, selection and mean update on
the GPU (through the C ABI), then one step of the host plant with the
returned action.  The value is rollout-steps per second (N x H x iterations
per tick) over the timed ticks, with the inputs already resident.  One JSON
line is printed.  Its roofline object rates the rollout kernel: algorithmic
FP32 FLOP per launch (FLOP_PER_ROLLOUT_STEP x N x H) over the kernel's
average duration from HIP events on the runtime stream, against the
non-packed FP32 VALU peak.  Its cpu_baseline object times the FP64 oracle on
the host cores over a bounded sample of full-size ticks.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "rollout-steps/sec (N×H per s) + p99 control-tick latency vs plain single MPPI"
# Algorithmic FP32 work of one rollout step, counted with add/sub/mul = 1,
# fma = 2, each sin, cos, sqrt, rcp, rsqrt = 1: policy 24, friction cone 36,
# attitude 24, footholds at touchdown 3 (0.14 touchdowns per step), stage cost
# 94, force and torque 72, R^T tau 15, gyroscopic term 12, Euler-angle rates 11,
# accelerations 10, Euler update and time 25.
FLOP_PER_ROLLOUT_STEP = 326
# With the GRF spline (Sec. IV-B) a step evaluates the spline on four knots
# (12 x (1 mul + 3 fma) = 84) instead of forming mu + sigma z (24); each knot
# of each sample forms mu + sigma z once (24 per knot).
FLOP_PER_SPLINE_STEP = FLOP_PER_ROLLOUT_STEP - 24 + 84
FLOP_PER_SPLINE_KNOT = 24
# Non-packed FP32 VALU peak of MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2 FLOP x 2.4 GHz.
PEAK_FP32_VALU_TFLOPS = 78.6
PEAK_FP32_PUBLISHED_TFLOPS = 157.3


def pct(a, p):
    return float(np.percentile(np.asarray(a, np.float64), p))


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("sbs_kernels.hip", "sbs_device.h"):
        with open(os.path.join(ROOT, "paper_2403_11383_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_traffic(kernel: str, workload: str):
    """HBM bytes per launch from committed rocprofv3 counter summaries, only
    while the kernel source is the one the counters were taken on."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        doc = json.load(open(path))
        ent = doc.get(f"{kernel}/{workload}")
        if ent and ent.get("kernel_source_hash") == kernel_source_hash():
            return ent.get("bytes_per_launch")
    except Exception:
        return None
    return None


def closed_loop(rt, binding, workloads, cfg, ticks, warmup, push_from=30, push=40.0,
                prefetch=True, v_ref=(0.3, 0.0, 0.0), episode=100):
    """Receding-horizon episodes of `episode` ticks (the workload's 100): each
    starts the plant from the seeded initial state (the controller keeps its
    warm start and tick counter); the push acts from tick `push_from` of each
    episode.  An episode also ends when the robot falls (roll or pitch beyond
    1.5 rad, CoM height outside [0.05, 1] m, or a non-finite state).  The
    first `warmup` ticks are untimed."""
    cid = rt.init_controller(cfg)
    if prefetch:
        rt.set_prefetch(cid, True)
    rng = np.random.default_rng(cfg["seed"])
    x0 = workloads.initial_state(rng)
    lat, acts = [], []
    t_start = None
    import torch
    no_push, push_f = (0.0, 0.0, 0.0), (0.0, push, 0.0)
    loop = None
    e, falls = 0, 0
    for t in range(warmup + ticks):
        if t == warmup or e == episode:
            e = 0
        if e == 0:
            plant = binding.Plant(cfg, x0, workloads.feet_under_hips(x0), phase=0)
            loop = binding.ClosedLoop(rt, cid, plant, v_ref=v_ref, z_ref=workloads.HEIGHT)
        if t == warmup:
            torch.cuda.synchronize()
            rt.timing()  # reset the stage-timing accumulators
            t_start = time.perf_counter()
        a = loop.step(push_f if e >= push_from else no_push)
        e += 1
        x = loop.plant.st.x
        if not (abs(x[3]) < 1.5 and abs(x[4]) < 1.5 and 0.05 < x[2] < 1.0):  # NaN fails too
            e = 0
            falls += 1 if t >= warmup else 0
        if t >= warmup:
            # submit-to-visible latency as recorded by the runtime
            lat.append((a.t_done_ns - a.t_submit_ns) * 1e-6)
            acts.append((a.flags, a.freq_hz, a.n_active))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    timing = rt.timing()
    rt.destroy_controller(cid)
    return elapsed, lat, acts, timing, (loop.plant, falls)


def cpu_baseline(cfg, seconds=10.0):
    """The FP64 oracle on the host cores: full-size ticks of the same workload
    from the same initial state until about `seconds` have passed."""
    import oracle
    from paper_2403_11383_amd import workloads
    oracle.build()
    cores = len(os.sched_getaffinity(0))
    rng = np.random.default_rng(cfg["seed"])
    x0 = workloads.initial_state(rng)
    inp = workloads.tick_input(x0, v_ref=(0.3, 0.0, 0.0))
    mu = np.tile([0.0, 0.0, 0.5 * cfg["mass"] * cfg["gravity"]] * 4, (oracle.rows(cfg), 1))
    n = 0
    t0 = time.perf_counter()
    while True:
        out = oracle.tick(cfg, mu, cfg["mu_f0"], n, inp, nthreads=cores)
        mu = out["mu_next"]
        n += 1
        if time.perf_counter() - t0 >= seconds and n >= 2:
            break
    dt = time.perf_counter() - t0
    steps = n * cfg["N"] * cfg["H"] * cfg["iterations"]
    # and on one core, for a few seconds
    n1, t1 = 0, time.perf_counter()
    mu1 = np.tile([0.0, 0.0, 0.5 * cfg["mass"] * cfg["gravity"]] * 4, (oracle.rows(cfg), 1))
    while True:
        mu1 = oracle.tick(cfg, mu1, cfg["mu_f0"], n1, inp, nthreads=1)["mu_next"]
        n1 += 1
        if time.perf_counter() - t1 >= min(3.0, seconds):
            break
    dt1 = time.perf_counter() - t1
    return {"value": steps / dt, "unit": "rollout-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"{n} full ticks (N={cfg['N']}, H={cfg['H']}) from the closed loop's "
                      f"initial state, {dt:.1f} s wall",
            "single_core": {"value": n1 * cfg["N"] * cfg["H"] * cfg["iterations"] / dt1,
                            "sample": f"{n1} full ticks on one thread, {dt1:.1f} s wall"}}


def batched(rt, binding, workloads, steps, warmup, cache_path=None):
    """64 uneven controllers in one fused, graph-replayed tick (autotuned
    rollout form), fixed per-controller inputs, warm-started means."""
    import torch
    cfgs = workloads.c3_controllers()
    inps = workloads.c3_inputs()
    ids = [rt.init_controller(c) for c in cfgs]
    plan = rt.plan_create(ids, use_graph=True)
    tune = rt.plan_autotune(plan, inps, reps=3, cache_path=cache_path)
    # the inputs are fixed per controller: marshalled once, and each tick is
    # one submit and one fetch call for all 64 controllers
    n = len(ids)
    ins = (binding.TickInput * n)(*[binding.make_input(x) for x in inps])
    tks = (binding.C.c_uint64 * n)()
    acts = (binding.Action * n)()
    for _ in range(warmup):
        rt.plan_submit_raw(plan, ins, tks)
        rt.fetch_many(tks, acts)
    torch.cuda.synchronize()
    lat = []
    t0 = time.perf_counter()
    for _ in range(steps):
        a = time.perf_counter_ns()
        rt.plan_submit_raw(plan, ins, tks)
        rt.fetch_many(tks, acts)
        lat.append((time.perf_counter_ns() - a) * 1e-6)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    work = sum(c["N"] * c["H"] * c.get("iterations", 1) for c in cfgs)
    rt.plan_destroy(plan)
    for c in ids:
        rt.destroy_controller(c)
    return elapsed, lat, work, tune, cfgs


def serving_run(binding, workloads, duration, mode, arena_bytes, robots=256):
    """C4: Poisson arrivals (50 Hz per robot) of control ticks from simulated
    robots of different N and H; serving mode batches whatever is admitted,
    direct mode runs every tick as its own launch sequence ("plain single
    MPPI").  Latency is measured from the scheduled arrival to completion."""
    import torch
    fleet = workloads.c4_fleet(robots=robots)
    arrivals = workloads.c4_arrivals(robots=robots, duration_s=duration)
    rt = binding.Runtime(arena_bytes=arena_bytes, mode=mode, two_streams=(mode == "serving"))
    ids = [rt.init_controller(c) for c in fleet]
    rng = np.random.default_rng(5)
    inputs = [binding.make_input(workloads.tick_input(workloads.initial_state(rng))) for _ in fleet]
    events = sorted((t, r) for r, ts in enumerate(arrivals) for t in ts)
    L = binding.lib()
    import ctypes as C
    pending = {}
    lat, done_work = [], 0
    tk = C.c_uint64()
    act = binding.Action()
    torch.cuda.synchronize()
    t_start = time.perf_counter_ns()
    i = 0
    while i < len(events) or pending:
        now = (time.perf_counter_ns() - t_start) * 1e-9
        while i < len(events) and events[i][0] <= now:
            t_arr, r = events[i]
            rc = L.sbs_submit_tick(rt._h, ids[r], C.byref(inputs[r]), C.byref(tk))
            if rc == binding.ENOMEM:  # arena full: retire finished ticks first
                break
            binding._check(rc)
            pending[tk.value] = (t_arr, r)
            i += 1
        for t in list(pending):
            rc = L.sbs_fetch_action(rt._h, t, C.byref(act), 0)
            if rc == binding.OK:
                t_arr, r = pending.pop(t)
                lat.append((act.t_done_ns - t_start) * 1e-6 - t_arr * 1e3)
                c = fleet[r]
                done_work += c["N"] * c["H"]
            elif rc != binding.EAGAIN:
                binding._check(rc)
        if mode == "direct" and pending and i < len(events) and events[i][0] > now:
            time.sleep(0)
    elapsed = (time.perf_counter_ns() - t_start) * 1e-9
    stats = rt.stats()
    rt.close()
    return {"ticks": len(lat), "elapsed_s": elapsed, "rollout_steps_per_s": done_work / elapsed,
            "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99), "max_ms": float(np.max(lat)),
            "batches": stats["batches"], "admit_waits": stats["admit_waits"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000,
                    help="timed ticks (c1/c2: episodes of 100 ticks from the seeded start)")
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--timing", type=int, default=1,
                    help="HIP events: 0 none, 1 the rollout kernel's own dispatch events on "
                         "one tick in 16, 2 event commands around every stage of every tick")
    ap.add_argument("--workload", default="c1", choices=["c1", "c2", "c3", "c4", "copy", "study"],
                    help="c1 closed-loop single MPPI (default); c2 closed-loop elite "
                         "sampler (N=16384, H=50, 3 iterations); c3 batched uneven "
                         "controllers; c4 serving 256 robots vs plain single MPPI; copy: "
                         "a plain 1 GiB device copy, the reference for HBM byte counters; "
                         "study: closed-loop push episodes with and without gait adaptation")
    ap.add_argument("--episodes", type=int, default=20, help="study: seeded episodes per setting")
    ap.add_argument("--duration", type=float, default=10.0, help="c4 stream length [s]")
    ap.add_argument("--arena-gb", type=float, default=4.0)
    ap.add_argument("--no-prefetch", action="store_true",
                    help="c1: generate each tick's noise inside the tick")
    ap.add_argument("--knots", type=int, default=0,
                    help="c1: GRF spline through this many knots (0: one GRF vector per step)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    if args.workload == "copy":
        return main_copy(args)
    if args.workload == "c3":
        return main_c3(args)
    if args.workload == "c4":
        return main_c4(args)
    if args.workload == "study":
        return main_study(args)

    from paper_2403_11383_amd import binding, workloads
    import torch
    c2 = args.workload == "c2"
    cfg = workloads.config(args.workload, knots=args.knots)
    rt = binding.Runtime(arena_bytes=int(args.arena_gb * (1 << 30)), two_streams=True)
    rt.set_timing(args.timing)
    elapsed, lat, acts, timing, plant = closed_loop(
        rt, binding, workloads, cfg, args.steps, args.warmup, prefetch=not args.no_prefetch,
        push=0.0 if c2 else 40.0, v_ref=workloads.c2_episode_vref() if c2 else (0.3, 0.0, 0.0))
    # the events a dispatch carries span its start marker's completion to the
    # kernel's end: a launch that finds its stream idle (the first rollout of
    # a tick; the noise was made ahead) also spans the dispatch's own start-up,
    # measured on an empty kernel bracketed the same way and taken off once
    # per tick; later iterations' rollouts queue behind the previous update
    # and start as soon as it ends
    ev_ovh_ns = rt.timing_overhead_ns(64) if timing["rollout_ns"] > 0 else 0.0
    rt.close()
    N, H, R = cfg["N"], cfg["H"], cfg["iterations"]
    steps_total = N * H * R * args.steps
    value = steps_total / elapsed
    ev_taken_ns = ev_ovh_ns / R if not args.no_prefetch else 0.0
    t_roll = max(timing["rollout_ns"] - ev_taken_ns, 0.0) * 1e-9
    P = args.knots
    flop = N * H * FLOP_PER_ROLLOUT_STEP if P == 0 else \
        N * (H * FLOP_PER_SPLINE_STEP + P * FLOP_PER_SPLINE_KNOT)
    achieved = flop / t_roll / 1e12 if t_roll > 0 else 0.0
    spline_txt = f", GRF spline through {P} knots" if P else ""
    workload_key = args.workload if P == 0 else f"{args.workload}_knots{P}"
    if c2:
        desc = ("c2: closed-loop elite sampler, top 10% of N=16384, H=50, 3 iterations per "
                "tick, Gaussian gait frequency 1.4 +- 0.4 Hz, reference velocity "
                f"{workloads.c2_episode_vref()[0]:+.3f} m/s")
    else:
        desc = ("c1: closed-loop MPPI, gait frequency ~U[1.0,2.5] Hz per sample, "
                "N=10240, H=50, dt=0.02 s, 40 N lateral push from tick 30")
    line = {
        "metric": METRIC, "value": value, "unit": "rollout-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": desc + spline_txt,
                   "N": N, "H": H, "iterations": R, "knots": P, "ticks": args.steps,
                   "noise_prefetch": not args.no_prefetch},
        "latency_ms": {"p50": pct(lat, 50), "p99": pct(lat, 99), "max": float(np.max(lat))},
        "stage_us": {k[:-3]: timing[k] * 1e-3 for k in ("noise_ns", "rollout_ns", "select_ns",
                                                        "update_ns") if timing[k] > 0},
        # the automatic lane policy runs one controller of up to 32768
        # samples with four lanes per sample
        "roofline": {"kernel": "k_rollout_quad" if N <= 32768 else "k_rollout<float>",
                     "launches_per_tick": R,
                     "bound": "alu", "achieved": achieved,
                     "peak": PEAK_FP32_VALU_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_VALU_TFLOPS,
                     "peak_published_packed": PEAK_FP32_PUBLISHED_TFLOPS,
                     "frac_of_published": achieved / PEAK_FP32_PUBLISHED_TFLOPS,
                     "traffic": stored_traffic("k_rollout", workload_key),
                     "flop_per_launch": flop, "duration_us": t_roll * 1e6,
                     # four lanes per sample: waves in flight against the
                     # chip's 1024 SIMDs (one wave per SIMD leaves the
                     # step-to-step dependency chain exposed)
                     "waves": (N * 4 + 63) // 64 if N <= 32768 else (N + 63) // 64,
                     "simds": 1024,
                     "event_interval_us": timing["rollout_ns"] * 1e-3,
                     "event_overhead_us": ev_ovh_ns * 1e-3,
                     "event_overhead_taken_us": ev_taken_ns * 1e-3},
        "closed_loop": {"episodes_ended_by_falls": plant[1],
                        "final_x": [round(float(v), 4) for v in plant[0].x],
                        "nonfinite_ticks": int(sum(a[0] & 1 for a in acts)),
                        "freq_hz_last": acts[-1][1],
                        "active_samples_median": float(np.median([a[2] for a in acts]))},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(cfg, args.cpu_seconds)
    print(json.dumps(line), flush=True)


def main_c3(args):
    from paper_2403_11383_amd import binding, workloads
    rt = binding.Runtime(arena_bytes=int(args.arena_gb * (1 << 30)))
    # the autotuner's choice for this batch, kept between runs on one machine
    cache = os.environ.get("SBS_AUTOTUNE_CACHE",
                           os.path.join(ROOT, ".sbs_cache", "autotune_cache.json"))
    os.makedirs(os.path.dirname(cache), exist_ok=True)
    elapsed, lat, work, tune, cfgs = batched(rt, binding, workloads, args.steps, args.warmup, cache)
    # rollout-kernel timing from a separate pass without the graph: the
    # rollout's own dispatch events on every launch (timing mode 3)
    rt.set_timing(3)
    ids = [rt.init_controller(c) for c in cfgs]
    inps = workloads.c3_inputs()
    plan = rt.plan_create(ids, use_graph=False)
    rt.plan_set_tune(plan, tune["lanes"], tune["block"], tune["unroll"])
    for _ in range(3):
        for t in rt.plan_submit(plan, inps):
            rt.fetch(t)
    rt.timing()
    reps = 5
    for _ in range(reps):
        for t in rt.plan_submit(plan, inps):
            rt.fetch(t)
    tm = rt.timing()
    # every rollout here queues behind its iteration's noise stage, so its
    # events span the kernel alone (the overhead of an idle-stream launch is
    # reported, not taken off)
    ev_ovh_ns = rt.timing_overhead_ns(64)
    rt.close()
    roll_ns_total = tm["rollout_ns"] * tm["launches"][1]
    flop = work * FLOP_PER_ROLLOUT_STEP * reps
    achieved = flop / (roll_ns_total * 1e-9) / 1e12 if roll_ns_total > 0 else 0.0
    line = {
        "metric": METRIC, "value": work * args.steps / elapsed, "unit": "rollout-steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "c3: 64 uneven controllers (N log-uniform 1024..16384, H 20..60, "
                               "MPPI/elite mix) in one graph-replayed fused tick",
                   "rollout_steps_per_tick": work, "tune": tune},
        "latency_ms": {"p50": pct(lat, 50), "p99": pct(lat, 99)},
        "roofline": {"kernel": "k_rollout (tuned form)", "bound": "alu", "achieved": achieved,
                     "peak": PEAK_FP32_VALU_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_VALU_TFLOPS,
                     "peak_published_packed": PEAK_FP32_PUBLISHED_TFLOPS,
                     "frac_of_published": achieved / PEAK_FP32_PUBLISHED_TFLOPS,
                     "traffic": stored_traffic("k_rollout", "c3"),
                     "duration_us": roll_ns_total / max(1, tm["launches"][1]) * 1e-3,
                     "event_interval_us": tm["rollout_ns"] * 1e-3,
                     "event_overhead_us": ev_ovh_ns * 1e-3, "event_overhead_taken_us": 0.0},
    }
    print(json.dumps(line), flush=True)


def main_copy(args):
    """Copies a 1 GiB device buffer `steps` times: 1 GiB read + 1 GiB written
    per copy kernel, the known-size reference for FETCH_SIZE / WRITE_SIZE."""
    import torch
    n = 1 << 30
    a = torch.empty(n, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b.copy_(a)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print(json.dumps({"workload": "copy", "bytes_per_copy": n, "copies": args.steps,
                      "GBps_read_plus_write": 2 * n * args.steps / dt / 1e9}), flush=True)


def study_episode(rt, binding, workloads, cfg, seed):
    """One push episode of the disturbance study on the host plant: returns
    the tick of the fall (None if the robot stays up), the executed frequency
    per tick and the submit-to-visible latency per tick [ms]."""
    cid = rt.init_controller(cfg)
    x0 = workloads.initial_state(np.random.default_rng(seed))
    plant = binding.Plant(cfg, x0, workloads.feet_under_hips(x0), phase=0)
    loop = binding.ClosedLoop(rt, cid, plant, v_ref=workloads.STUDY_VREF, z_ref=workloads.HEIGHT)
    fell, freq, lat = None, [], []
    for t in range(workloads.STUDY_TICKS):
        w = workloads.study_wrench(t)
        a = loop.step(w[:3], w[3:])
        freq.append(a.freq_hz)
        lat.append((a.t_done_ns - a.t_submit_ns) * 1e-6)
        x = loop.plant.st.x
        if not (abs(x[3]) < 0.8 and abs(x[4]) < 0.8 and 0.2 < x[2] < 0.6):  # NaN fails too
            fell = t
            break
    rt.destroy_controller(cid)
    return fell, freq, lat


def main_study(args):
    """Closed-loop disturbance study (the shape of the paper's Fig. 4 test):
    seeded episodes of a 40 N lateral push for 3 s, for the best-sample and
    MPPI controllers with gait adaptation (frequency set, at two weights of
    the frequency regulariser) and without it (fixed f_n).  Reports the
    episodes survived and, with adaptation, the mean executed frequency
    before, during and after the push over the surviving episodes."""
    from paper_2403_11383_amd import binding, workloads
    import torch
    rt = binding.Runtime(arena_bytes=int(args.arena_gb * (1 << 30)))
    p0, p1, _ = workloads.STUDY_PUSH
    settings = []
    for method in ("naive", "mppi"):
        settings += [(method, True, 1.0), (method, True, 300.0), (method, False, 1.0)]
    out, lat_all = [], []
    t0 = time.perf_counter()
    for method, adapt, rho in settings:
        cfg = workloads.study_config(method, adapt=adapt, rho=rho)
        falls, fpre, fpush, fpost = [], [], [], []
        for ep in range(args.episodes):
            fell, freq, lat = study_episode(rt, binding, workloads, cfg, seed=1 + ep)
            falls.append(fell)
            lat_all += lat
            if fell is None:
                f = np.asarray(freq)
                fpre.append(f[:p0].mean())
                fpush.append(f[p0:p1].mean())
                fpost.append(f[p1 + 10:].mean())
        rec = {"method": method, "gait_adaptation": adapt, "rho": rho,
               "survived": sum(f is None for f in falls), "episodes": len(falls),
               "fall_ticks": [f for f in falls if f is not None]}
        if adapt and fpre:
            rec["freq_hz_before_during_after"] = [round(float(np.mean(v)), 3)
                                                  for v in (fpre, fpush, fpost)]
        out.append(rec)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    rt.close()
    def rate(adapt):
        rs = [r for r in out if r["gait_adaptation"] == adapt]
        return sum(r["survived"] for r in rs) / max(1, sum(r["episodes"] for r in rs))
    print(json.dumps({
        "metric": "closed-loop push survival with gait adaptation",
        "value": rate(True), "without_gait_adaptation": rate(False),
        "unit": "fraction of episodes", "higher_is_better": True, "n_gpus": 1,
        "data": "synthetic",
        "config": {"workload": "study: 40 N lateral push for 3 s from 2 s, 0.1 m/s lateral "
                               "command, 8 s episodes, N=10240, H=25, host SRBD plant",
                   "episodes_per_setting": args.episodes},
        "settings": out,
        "tick_latency_ms": {"p50": pct(lat_all, 50), "p99": pct(lat_all, 99)},
        "wall_s": round(elapsed, 2)}), flush=True)


def saturated_run(binding, workloads, duration, mode, arena_bytes, robots=256):
    """The C4 fleet with every robot's next tick submitted as soon as its
    previous one completes (no arrival gaps): the most ticks per second each
    mode sustains, and their submit-to-done latency."""
    import ctypes as C
    import torch
    fleet = workloads.c4_fleet(robots=robots)
    rt = binding.Runtime(arena_bytes=arena_bytes, mode=mode, two_streams=(mode == "serving"))
    ids = [rt.init_controller(c) for c in fleet]
    rng = np.random.default_rng(6)
    inputs = [binding.make_input(workloads.tick_input(workloads.initial_state(rng))) for _ in fleet]
    L = binding.lib()
    tk = C.c_uint64()
    act = binding.Action()
    torch.cuda.synchronize()
    pending = {}
    lat, done_work = [], 0
    t_start = time.perf_counter_ns()
    t_end = t_start + int(duration * 1e9)
    idle = list(range(robots))
    while time.perf_counter_ns() < t_end or pending:
        if time.perf_counter_ns() < t_end:
            still = []
            for r in idle:
                rc = L.sbs_submit_tick(rt._h, ids[r], C.byref(inputs[r]), C.byref(tk))
                if rc == binding.ENOMEM:
                    still.append(r)
                    continue
                binding._check(rc)
                pending[tk.value] = r
            idle = still
        for t in list(pending):
            rc = L.sbs_fetch_action(rt._h, t, C.byref(act), 0)
            if rc == binding.OK:
                r = pending.pop(t)
                lat.append((act.t_done_ns - act.t_submit_ns) * 1e-6)
                done_work += fleet[r]["N"] * fleet[r]["H"]
                idle.append(r)
            elif rc != binding.EAGAIN:
                binding._check(rc)
    elapsed = (time.perf_counter_ns() - t_start) * 1e-9
    stats = rt.stats()
    rt.close()
    return {"ticks": len(lat), "elapsed_s": elapsed, "ticks_per_s": len(lat) / elapsed,
            "rollout_steps_per_s": done_work / elapsed, "p50_ms": pct(lat, 50),
            "p99_ms": pct(lat, 99), "batches": stats["batches"]}


def main_c4(args):
    from paper_2403_11383_amd import binding, workloads
    arena = int(args.arena_gb * (1 << 30))
    serve = serving_run(binding, workloads, args.duration, "serving", arena)
    plain = serving_run(binding, workloads, args.duration, "direct", arena)
    sat_serve = saturated_run(binding, workloads, 3.0, "serving", arena)
    sat_plain = saturated_run(binding, workloads, 3.0, "direct", arena)
    line = {
        "metric": METRIC, "value": serve["rollout_steps_per_s"], "unit": "rollout-steps/s",
        "n_gpus": 1, "steps": serve["ticks"], "warmup": 0,
        "ms_per_step": serve["elapsed_s"] / max(1, serve["ticks"]) * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "c4: 256 robots, Poisson 50 Hz each, N in {2048,4096,8192}, "
                               "H in {25,50}, continuous batching vs plain single MPPI",
                   "duration_s": args.duration, "arena_gb": args.arena_gb},
        "latency_ms": {"p50": serve["p50_ms"], "p99": serve["p99_ms"]},
        "serving": serve, "plain_single_mppi": plain,
        "saturated": {"serving": sat_serve, "plain_single_mppi": sat_plain},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
