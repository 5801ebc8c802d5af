"""Benchmark of one GPU: the serving workload (256 simulated robots, each
issuing control ticks at 50 Hz with Poisson jitter; N in {2048, 4096, 8192}
samples and H in {25, 50} steps per robot; MPPI with per-sample gait
frequency ~U[1.0, 2.5] Hz, GRF noise 25 N, lambda = 1, Q = I, R = 1e-4 I,
friction cone mu = 0.5; FP32 rollouts) through continuous batching, against
the plain single-controller MPPI (each tick its own launch sequence on one
stream) on the same GPU.  One JSON line is printed.

value: rollout-steps per second (N x H per tick, summed over completed
ticks) that continuous batching sustains with every robot's next tick
submitted as soon as its previous one completes (saturated), inputs already
resident.  Beside it: the same for the plain single-controller form
(vs_baseline = the ratio), and the p50/p99 tick latency from arrival of both
forms on the 50 Hz Poisson stream.  A step is 0.15 s of the saturated stream
(and 0.5 s of each 50 Hz arrival stream).

The roofline object rates the rollout kernel of the saturated serving run:
algorithmic FP32 FLOP of its timed launches (FLOP_PER_ROLLOUT_STEP x the
rollout-steps each launch covered) over their device time from HIP events
carried by the launches' own dispatches on the runtime's streams.  An
untimed serving pass records served ticks of the robots whose index is a
multiple of 100 (about 1 % of the ticks) with the controller state each
started from; the cpu_baseline leg reruns them on the FP64 oracle on the
host cores (timed: cpu_baseline) and compares the actions (shadow_oracle).

Other workloads (--workload): c1 closed-loop MPPI (N = 10240, H = 50), c2
closed-loop elite sampler (N = 16384, H = 50, 3 iterations), c3 64 uneven
controllers in one graph-replayed tick, study (push episodes with and
without gait adaptation), copy (HBM byte-counter reference).
"""
from __future__ import annotations

import argparse
import contextlib
import gc
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
# A rollout that also draws its noise does the FP32 arithmetic of the 12
# Gaussians of each step too: 50 FLOP per Box-Muller pair (the logarithm
# 24: f = m - 1, f^2, the degree-7 polynomial P and the two FMAs around it
# 20, the exponent terms 4; radius 2; the turn's sine and cosine polynomials
# 21; the two products 2; the fold's halving 1), 6 pairs per step; Philox's
# integer work is not counted.
FLOP_PER_GAUSS_PAIR = 50
FLOP_PER_NOISE_ROW = 6 * FLOP_PER_GAUSS_PAIR
FLOP_PER_ROLLOUT_STEP_WITH_NOISE = FLOP_PER_ROLLOUT_STEP + FLOP_PER_NOISE_ROW
# a stance-pair rollout that draws only its stance diagonal's noise evaluates
# three of the six pairs per step
FLOP_PER_ROLLOUT_STEP_WITH_STANCE_NOISE = FLOP_PER_ROLLOUT_STEP + 3 * FLOP_PER_GAUSS_PAIR
# MI355X FP32 vector peak as published (it counts packed FMAs: 256 CUs x 4
# SIMDs x 16 lanes x 2 FLOP x 2 packed x 2.4 GHz) and the non-packed peak the
# kernels can reach (they are built with packed FP32 off).
PEAK_FP32_PUBLISHED_TFLOPS = 157.3
PEAK_FP32_VALU_TFLOPS = 78.6


def pct(a, p):
    return float(np.percentile(np.asarray(a, np.float64), p))


@contextlib.contextmanager
def gc_paused():
    """Python's cyclic garbage collector paused over a timed region (after one
    full collection): a full pass over torch's object graph takes tens of
    milliseconds and would otherwise land inside the timing at random."""
    gc.collect()
    was = gc.isenabled()
    gc.disable()
    try:
        yield
    finally:
        if was:
            gc.enable()


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("sbs_kernels.hip", "sbs_device.h"):
        with open(os.path.join(ROOT, "paper_2403_11383_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_traffic(kernel: str, workload: str, rollout_steps_per_launch=None):
    """HBM bytes per launch from committed rocprofv3 counter summaries, only
    while the kernel source is the one the counters were taken on.  Entries
    of workloads whose launches vary in size (the serving fleet) hold bytes
    per rollout-step, scaled here by the launches' average rollout-steps."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        doc = json.load(open(path))
        ent = doc.get(f"{kernel}/{workload}")
        if ent and ent.get("kernel_source_hash") == kernel_source_hash():
            if "bytes_per_rollout_step" in ent:
                if rollout_steps_per_launch is None:
                    return None
                return ent["bytes_per_rollout_step"] * rollout_steps_per_launch
            return ent.get("bytes_per_launch")
    except Exception:
        return None
    return None


def closed_loop(rt, binding, workloads, cfg, ticks, warmup, push_from=30, push=40.0,
                prefetch=True, v_ref=(0.3, 0.0, 0.0), episode=100):
    """Receding-horizon episodes of `episode` ticks (the workload's 100): each
    starts the plant from the seeded initial state (the controller keeps its
    warm start and tick counter); the push acts from tick `push_from` of each
    episode.  An episode also ends when the robot falls (workloads.fallen:
    roll or pitch beyond 0.8 rad, CoM height outside (0.2, 0.6) m, or a
    non-finite state).  The first `warmup` ticks are untimed."""
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
    with gc_paused():
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
            if workloads.fallen(x):
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
    with gc_paused():
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="c4: 0.15 s of the saturated stream and 0.5 s of each 50 Hz stream "
                         "per step (default 20); c1/c2/c3: timed ticks (default 1000; c1/c2 in "
                         "episodes of 100 ticks from the seeded start)")
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--timing", type=int, default=1,
                    help="HIP events: 0 none, 1 the rollout kernel's own dispatch events on "
                         "one tick in 16, 2 event commands around every stage of every tick")
    ap.add_argument("--streams", type=int, default=1, choices=[1, 2],
                    help="c4: streams the serving scheduler alternates batches on")
    ap.add_argument("--shadow-seconds", type=float, default=6.0,
                    help="c4: arrival-stream length of the pass that records the served ticks "
                         "the oracle reruns (cpu_baseline and shadow_oracle)")
    ap.add_argument("--workload", default="c4", choices=["c1", "c2", "c3", "c4", "copy", "study"],
                    help="c4 serving vs plain single MPPI (default); c1 closed-loop single "
                         "MPPI; c2 closed-loop elite "
                         "sampler (N=16384, H=50, 3 iterations); c3 batched uneven "
                         "controllers; copy: "
                         "a plain 1 GiB device copy, the reference for HBM byte counters; "
                         "study: closed-loop push episodes with and without gait adaptation")
    ap.add_argument("--rollout-noise", type=int, default=2, choices=[0, 1, 2],
                    help="c4: sbs_set_rollout_noise mode (0 noise launch, 1 rows in the rollout, "
                         "2 stance legs only where the form allows)")
    ap.add_argument("--depth", type=int, default=2,
                    help="c4: serving batches in flight per stream (sbs_set_serving_depth)")
    ap.add_argument("--phase", default="all", choices=["all", "saturated"],
                    help="c4: 'saturated' runs only the saturated serving stream, with HIP "
                         "events on every rollout launch and no warm-up, and prints each "
                         "rollout form's launches, rollout-steps and average duration over "
                         "the whole process (for kernel traces and HBM byte counters)")
    ap.add_argument("--episodes", type=int, default=20, help="study: seeded episodes per setting")
    ap.add_argument("--duration", type=float, default=10.0, help="c4 stream length [s]")
    ap.add_argument("--arena-gb", type=float, default=4.0)
    ap.add_argument("--no-prefetch", action="store_true",
                    help="c1: generate each tick's noise inside the tick")
    ap.add_argument("--knots", type=int, default=0,
                    help="c1: GRF spline through this many knots (0: one GRF vector per step)")
    args = ap.parse_args()
    if args.steps is None:
        args.steps = 20 if args.workload == "c4" else 1000
    if args.warmup is None:
        args.warmup = 5 if args.workload == "c4" else 10
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
        "roofline": roofline_obj(
            "k_rollout_quad" if N <= 32768 else "k_rollout<float>", flop, t_roll * 1e9, 1,
            launches_per_tick=R, traffic=stored_traffic("k_rollout", workload_key),
            flop_per_launch=flop, duration_us=t_roll * 1e6,
            # four lanes per sample: waves in flight against the chip's 1024
            # SIMDs (one wave per SIMD leaves the step-to-step dependency
            # chain exposed)
            waves=(N * 4 + 63) // 64 if N <= 32768 else (N + 63) // 64, simds=1024,
            event_interval_us=timing["rollout_ns"] * 1e-3, event_overhead_us=ev_ovh_ns * 1e-3,
            event_overhead_taken_us=ev_taken_ns * 1e-3),
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
    for f in range(N_FORMS):
        rt.timing_rollout(f)
    reps = 5
    for _ in range(reps):
        for t in rt.plan_submit(plan, inps):
            rt.fetch(t)
    rt.timing()
    forms = [rt.timing_rollout(f) for f in range(N_FORMS)]
    # the events of a rollout queued behind other work span the kernel alone
    # (the overhead of an idle-stream launch is reported, not taken off)
    ev_ovh_ns = rt.timing_overhead_ns(64)
    rt.close()
    # dominant rollout form by device time, rated with its own FLOP count
    f = max(range(N_FORMS), key=lambda i: forms[i]["avg_ns"] * forms[i]["launches"])
    fo = forms[f]
    flop = fo["steps"] * FORM_FLOP_PER_STEP[f]
    line = {
        "metric": METRIC, "value": work * args.steps / elapsed, "unit": "rollout-steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "c3: 64 uneven controllers (N log-uniform 1024..16384, H 20..60, "
                               "MPPI/elite mix) in one graph-replayed fused tick",
                   "rollout_steps_per_tick": work, "tune": tune},
        "latency_ms": {"p50": pct(lat, 50), "p99": pct(lat, 99)},
        "roofline": roofline_obj(
            FORM_NAMES[f], flop, fo["avg_ns"], fo["launches"],
            flop_per_rollout_step=FORM_FLOP_PER_STEP[f],
            traffic=(stored_traffic(FORM_TRAFFIC_KEY[f], "c3", fo["steps"] / max(1, fo["launches"]))
                     if FORM_TRAFFIC_KEY[f] else None),
            timed_launches=fo["launches"], duration_us=fo["avg_ns"] * 1e-3,
            rollout_steps_per_launch=fo["steps"] / max(1, fo["launches"]),
            event_overhead_us=ev_ovh_ns * 1e-3, event_overhead_taken_us=0.0,
            other_forms={FORM_NAMES[i]: {"timed_launches": forms[i]["launches"],
                                         "duration_us": forms[i]["avg_ns"] * 1e-3,
                                         "rollout_steps_per_launch":
                                             forms[i]["steps"] / max(1, forms[i]["launches"])}
                         for i in range(N_FORMS) if i != f and forms[i]["launches"]}),
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
        if workloads.fallen(x):
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


# ---------------------------------------------------------------------------
# C4: serving 256 robots
# ---------------------------------------------------------------------------
STEP_S_ARRIVALS = 0.5    # one step: 0.5 s of each 50 Hz arrival stream
STEP_S_SATURATED = 0.15  # and 0.15 s of the saturated stream
SHADOW_EVERY = 100       # robots 0, 100, 200 are shadowed by the oracle


def roofline_obj(kernel, flop, dur_ns, launches, **extra):
    """The roofline object of an ALU-bound rollout: algorithmic FLOP over
    device time, against the published FP32 vector peak and (beside it) the
    non-packed peak the kernels can reach."""
    achieved = flop / (dur_ns * launches * 1e-9) / 1e12 if dur_ns > 0 and launches else 0.0
    out = {"kernel": kernel, "bound": "alu", "achieved": achieved,
           "peak": PEAK_FP32_PUBLISHED_TFLOPS, "unit": "TFLOP/s",
           "frac": achieved / PEAK_FP32_PUBLISHED_TFLOPS,
           "peak_nonpacked": PEAK_FP32_VALU_TFLOPS,
           "frac_nonpacked": achieved / PEAK_FP32_VALU_TFLOPS,
           "flop_per_rollout_step": FLOP_PER_ROLLOUT_STEP}
    out.update(extra)  # may restate flop_per_rollout_step for the form
    return out


def fleet_inputs(binding, workloads, fleet, seed):
    rng = np.random.default_rng(seed)
    return [binding.make_input(workloads.tick_input(workloads.initial_state(rng))) for _ in fleet]


def serving_run(binding, workloads, duration, mode, arena_bytes, robots=256, streams=2,
                depth=1, noise=2):
    """The C4 arrival stream: Poisson arrivals (50 Hz per robot) of control
    ticks; serving mode batches whatever is admitted, direct mode runs every
    tick as its own launch sequence ("plain single MPPI").  A robot's tick
    waits for its previous one (the warm start), inside the runtime.
    Latency is measured from the scheduled arrival to completion."""
    import ctypes as C
    import torch
    fleet = workloads.c4_fleet(robots=robots)
    arrivals = workloads.c4_arrivals(robots=robots, duration_s=duration)
    rt = binding.Runtime(arena_bytes=arena_bytes, mode=mode,
                         two_streams=(mode == "serving" and streams > 1))
    if mode == "serving":
        rt.set_serving_depth(depth)
    rt.set_rollout_noise(noise)
    ids = [rt.init_controller(c) for c in fleet]
    inputs = fleet_inputs(binding, workloads, fleet, 5)
    events = sorted((t, r) for r, ts in enumerate(arrivals) for t in ts)
    L = binding.lib()
    pending = {}
    lat, done_work = [], 0
    tk = C.c_uint64()
    # completed ticks come back in bulk (sbs_fetch_ready): one call per sweep
    rtk = (C.c_uint64 * 1024)()
    racts = (binding.Action * 1024)()
    nready = C.c_int32()
    torch.cuda.synchronize()
    with gc_paused():
        t_start = time.perf_counter_ns()
        i = 0
        while i < len(events) or pending:
            now = (time.perf_counter_ns() - t_start) * 1e-9
            while i < len(events) and events[i][0] <= now:
                t_arr, r = events[i]
                rc = L.sbs_submit_tick(rt._h, ids[r], C.byref(inputs[r]), C.byref(tk))
                if rc == binding.ENOMEM and mode == "direct":  # retire finished ticks first
                    break
                binding._check(rc)
                pending[tk.value] = (t_arr, r)
                i += 1
            if not pending:
                continue
            # wait for completions at most until the next arrival is due
            wait_us = 0
            if i < len(events):
                wait_us = max(0, min(100, int((events[i][0] - now) * 1e6)))
            binding._check(L.sbs_fetch_ready(rt._h, len(rtk), rtk, racts, C.byref(nready), wait_us))
            for i_ in range(nready.value):
                t_arr, r = pending.pop(rtk[i_])
                lat.append((racts[i_].t_done_ns - t_start) * 1e-6 - t_arr * 1e3)
                c = fleet[r]
                done_work += c["N"] * c["H"]
        elapsed = (time.perf_counter_ns() - t_start) * 1e-9
    stats = rt.stats()
    rt.close()
    return {"ticks": len(lat), "elapsed_s": elapsed, "ticks_per_s": len(lat) / elapsed,
            "rollout_steps_per_s": done_work / elapsed,
            "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99), "max_ms": float(np.max(lat)),
            "batches": stats["batches"], "admit_waits": stats["admit_waits"]}


def saturated_run(binding, workloads, duration, mode, arena_bytes, robots=256, timing=0,
                  warmup_ticks=0, streams=2, depth=1, noise=2):
    """The C4 fleet with every robot's next tick submitted as soon as its
    previous one completes (no arrival gaps): the most ticks per second each
    form sustains, and their submit-to-done latency.  The serving client
    works in bulk, as a fleet gateway would: every completed tick that one
    sbs_fetch_ready call returns is resubmitted in one sbs_submit_batch call
    (the scheduler still admits and batches them itself).  Plain single MPPI
    (direct mode) submits tick by tick, each its own launch sequence.  With
    timing, the rollout launches carry HIP events (one launch in 16; mode 3
    every launch) and the per-form rollout timings of the timed region are
    returned."""
    import ctypes as C
    import torch
    fleet = workloads.c4_fleet(robots=robots)
    rt = binding.Runtime(arena_bytes=arena_bytes, mode=mode,
                         two_streams=(mode == "serving" and streams > 1))
    if mode == "serving":
        rt.set_serving_depth(depth)
    rt.set_rollout_noise(noise)
    ids = [rt.init_controller(c) for c in fleet]
    inputs = fleet_inputs(binding, workloads, fleet, 6)
    L = binding.lib()
    tk = C.c_uint64()
    rtk = (C.c_uint64 * 1024)()
    racts = (binding.Action * 1024)()
    acts = np.ctypeslib.as_array(racts)
    nready = C.c_int32()
    ids_np = np.asarray(ids, np.int32)
    work_np = np.asarray([c["N"] * c["H"] for c in fleet], np.int64)
    id2robot = np.full(int(ids_np.max()) + 1, -1, np.int64)
    id2robot[ids_np] = np.arange(robots)
    # every robot's input once, contiguous; a bulk submission gathers its rows
    tin = binding.TickInput
    all_in = (tin * robots)(*inputs)
    all_np = np.frombuffer(all_in, np.uint8).reshape(robots, C.sizeof(tin))
    sub_in = (tin * robots)()
    sub_np = np.frombuffer(sub_in, np.uint8).reshape(robots, C.sizeof(tin))
    sub_ids = np.zeros(robots, np.int32)
    sub_tk = np.zeros(robots, np.uint64)
    # untimed warm-up: every robot's first ticks
    for _ in range(warmup_ticks):
        tks = [rt.submit_tick(cid, workloads.tick_input(workloads.initial_state(
            np.random.default_rng(6)))) for cid in ids]
        for t in tks:
            rt.fetch(t)
    torch.cuda.synchronize()
    if timing:
        rt.set_timing(timing)
        rt.timing()
        for f in range(N_FORMS):
            rt.timing_rollout(f)
    lat, done_work, n_pending = [], 0, 0
    with gc_paused():
        t_start = time.perf_counter_ns()
        t_end = t_start + int(duration * 1e9)
        idle = np.arange(robots)
        while time.perf_counter_ns() < t_end or n_pending:
            if len(idle) and time.perf_counter_ns() < t_end:
                if mode == "serving":
                    n = len(idle)
                    sub_np[:n] = all_np[idle]
                    sub_ids[:n] = ids_np[idle]
                    binding._check(L.sbs_submit_batch(
                        rt._h, n, sub_ids.ctypes.data_as(C.POINTER(C.c_int32)), sub_in,
                        sub_tk.ctypes.data_as(C.POINTER(C.c_uint64))))
                    n_pending += n
                    idle = idle[:0]
                else:
                    still = []
                    for r in idle:
                        rc = L.sbs_submit_tick(rt._h, ids[r], C.byref(all_in[r]), C.byref(tk))
                        if rc == binding.ENOMEM:  # retire finished ticks first
                            still.append(r)
                            continue
                        binding._check(rc)
                        n_pending += 1
                    idle = np.asarray(still, np.int64)
            binding._check(L.sbs_fetch_ready(rt._h, len(rtk), rtk, racts, C.byref(nready), 0))
            n = nready.value
            if n:
                a = acts[:n]
                rob = id2robot[a["controller"]]
                lat.append((a["t_done_ns"] - a["t_submit_ns"]) * 1e-6)
                done_work += int(work_np[rob].sum())
                idle = np.concatenate([idle, rob])
                n_pending -= n
        torch.cuda.synchronize()
        elapsed = (time.perf_counter_ns() - t_start) * 1e-9
    lat = np.concatenate(lat) if lat else np.zeros(1)
    stats = rt.stats()
    out = {"ticks": int(len(lat)), "elapsed_s": elapsed, "ticks_per_s": len(lat) / elapsed,
           "rollout_steps_per_s": done_work / elapsed, "p50_ms": pct(lat, 50),
           "p99_ms": pct(lat, 99), "batches": stats["batches"]}
    if timing:
        out["rollout_forms"] = [rt.timing_rollout(f) for f in range(N_FORMS)]
        out["event_overhead_ns"] = rt.timing_overhead_ns(64)
    rt.close()
    return out


def shadow_pass(binding, workloads, arena_bytes, seconds, robots=256, every=SHADOW_EVERY):
    """Records served ticks for the shadow oracle (untimed, GPU side only).
    The fleet runs a Poisson stream through the serving runtime; for the
    shadowed robots (index a multiple of `every`, about 1 % of the ticks) the
    bench exports the controller's state before each tick, waits for the
    tick in the mix and takes its FP32 costs and action."""
    fleet = workloads.c4_fleet(robots=robots)
    arrivals = workloads.c4_arrivals(robots=robots, duration_s=seconds, seed=9)
    rt = binding.Runtime(arena_bytes=arena_bytes, mode="serving", two_streams=True)
    ids = [rt.init_controller(c) for c in fleet]
    rng = np.random.default_rng(5)
    raw = [workloads.tick_input(workloads.initial_state(rng)) for _ in fleet]
    shadowed = set(range(0, robots, every))
    for r in shadowed:
        rt.set_debug(ids[r], True)
    events = sorted((t, r) for r, ts in enumerate(arrivals) for t in ts)
    recs, pending, total = [], [], 0
    t0 = time.perf_counter()
    for t_arr, r in events:
        while time.perf_counter() - t0 < t_arr:
            pass
        if r in shadowed:
            mu, mf, tick = rt.export_state(ids[r])  # its previous tick is done
            a = rt.fetch(rt.submit_tick(ids[r], raw[r]))
            J, _, _ = rt.debug_costs(ids[r])
            recs.append({"cfg": fleet[r], "inp": raw[r], "mu": mu, "mf": mf, "tick": tick,
                         "grf": a["grf"], "J": J})
        else:
            pending.append(rt.submit_tick(ids[r], raw[r]))
        total += 1
    for t in pending:
        rt.fetch(t)
    rt.close()
    return recs, total


def cpu_baseline_c4(workloads, recs, total_ticks):
    """The FP64 oracle on the host cores, on the served ticks that the shadow
    pass recorded: each reruns from the controller's exported state and
    input, timed on all cores (and a few on one core).  The same outputs are
    the shadow check: the GPU's action against the oracle's (FP32 rollouts
    and costs vs FP64), and against the oracle's update of the GPU's own
    costs (selection parity)."""
    import oracle
    oracle.build()
    cores = len(os.sched_getaffinity(0))
    mg2 = 0.5 * workloads.MASS * workloads.GRAVITY
    err_own, err_upd, steps = [], [], 0
    t0 = time.perf_counter()
    refs = []
    for rc in recs:
        refs.append(oracle.tick(rc["cfg"], rc["mu"], rc["mf"], rc["tick"], rc["inp"],
                                nthreads=cores))
        steps += rc["cfg"]["N"] * rc["cfg"]["H"]
    dt = time.perf_counter() - t0
    over = []
    for rc, ref in zip(recs, refs):
        upd = oracle.tick(rc["cfg"], rc["mu"], rc["mf"], rc["tick"], rc["inp"],
                          costs_override=rc["J"], nthreads=cores)
        scale = max(np.abs(ref["grf"]).max(), mg2)
        err_own.append(float(np.abs(rc["grf"] - ref["grf"]).max() / scale))
        err_upd.append(float(np.abs(rc["grf"] - upd["grf"]).max() / scale))
        if err_own[-1] > 1e-4:
            # first-order effect of the measured FP32-vs-FP64 cost differences
            # on the MPPI mean's first step: sum_k w_k |theta_k - mean|
            # |dJ_k - sum_i w_i dJ_i| / lambda (the weights of the oracle's
            # costs; FP32 rollouts of ill-conditioned samples move their costs)
            c, J = rc["cfg"], ref["costs"][-1]
            w, *_ = oracle.mppi_weights(J, c["lambda"])
            with np.errstate(invalid="ignore"):
                dJ = np.abs(np.asarray(rc["J"][-1], np.float64) - J)
            dJ = np.where(np.isfinite(dJ), dJ, 0.0)
            live = np.flatnonzero(w > 0)
            z = np.array([oracle.noise_step(c["seed"], rc["tick"], 0, int(k), 0) for k in live],
                         np.float64).reshape(len(live), 12)
            th = np.asarray(rc["mu"][0])[None] + c["sigma_grf"] * z
            dev = np.abs(th - ref["mean"][0][None])
            spread = np.abs(dJ[live] - (w * dJ).sum())
            bound = float((w[live][:, None] * dev * spread[:, None]).sum(0).max() / c["lambda"])
            # the conditioning of the samples the two sides weigh most: the
            # relative change of the FP64 cost under a 1e-7 relative change
            # of the decision variable, per unit (FP32 rounds at ~6e-8)
            rng = np.random.default_rng(12345)
            amp = {}
            for name, k in (("gpu_best", int(np.argmin(rc["J"][-1]))),
                            ("oracle_best", int(np.argmin(J)))):
                zk = np.array([oracle.noise_step(c["seed"], rc["tick"], 0, k, j)
                               for j in range(c["H"])], np.float64)
                thk = np.asarray(rc["mu"]) + c["sigma_grf"] * zk
                qk = int(ref["q_samples"][-1][k])
                j0 = oracle.rollout(c, rc["inp"], thk, qk)
                j1 = oracle.rollout(c, rc["inp"], thk * (1.0 + 1e-7 * rng.normal(size=thk.shape)), qk)
                amp[name] = float(abs(j1 - j0) / (1e-7 * max(abs(j0), 1.0)))
            over.append({"err_rel": err_own[-1], "first_order_rel": bound / scale,
                         "max_cost_diff_rel_of_weighted": float(
                             (dJ[live] / np.maximum(np.abs(J[live]), 1.0)).max()),
                         "weighted_samples": int(len(live)), "N": c["N"], "H": c["H"],
                         "same_best_sample": bool(np.argmin(rc["J"][-1]) == np.argmin(J)),
                         "cost_amplification": amp})
    n1, steps1, t1 = 0, 0, time.perf_counter()
    while n1 < len(recs) and (time.perf_counter() - t1 < 3.0 or n1 < 2):
        rc = recs[n1]
        oracle.tick(rc["cfg"], rc["mu"], rc["mf"], rc["tick"], rc["inp"], nthreads=1)
        steps1 += rc["cfg"]["N"] * rc["cfg"]["H"]
        n1 += 1
    dt1 = time.perf_counter() - t1
    base = {"value": steps / dt, "unit": "rollout-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"{len(recs)} served C4 ticks of robots 0, 100, 200 rerun from their "
                      f"exported states ({steps} rollout-steps), {dt:.1f} s wall",
            "ticks_per_s": len(recs) / dt,
            "single_core": {"value": steps1 / dt1,
                            "sample": f"the first {n1} of those ticks on one thread, "
                                      f"{dt1:.1f} s wall"}}
    e = np.asarray(err_own)
    shadow = {"ticks": len(recs), "of_ticks": total_ticks,
              "within_tolerance_fraction": float((e <= 1e-4).mean()),
              "median_action_err_rel": float(np.median(e)), "p99_action_err_rel": pct(e, 99),
              "max_action_err_rel": float(e.max()), "max_update_err_rel": max(err_upd),
              "tolerance_rel": 1e-4,
              "over_tolerance": sorted(over, key=lambda o: -o["err_rel"])[:5],
              "scale": "max(|grf|, m g / 2) of the oracle's action",
              "what": "action_err: the GPU's action vs the FP64 oracle's tick from the same "
                      "controller state and input; update_err: vs the oracle's update of the "
                      "GPU's own FP32 costs"}
    return base, shadow


def progress(msg):
    """A line per finished phase on stderr (the JSON line stays alone on stdout)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


# Rollout forms of sbs_timing_rollout: name, algorithmic FLOP per rollout-step,
# and the key of their stored HBM byte counts at C4
FORM_NAMES = ["k_rollout<float> (one lane per sample)", "k_rollout_quad (four lanes per sample)",
              "k_rollout<double>", "k_rollout<float> drawing its noise (one lane per sample)",
              "k_rollout<float> drawing its stance diagonal's noise (one lane per sample)"]
FORM_FLOP_PER_STEP = [FLOP_PER_ROLLOUT_STEP, FLOP_PER_ROLLOUT_STEP, FLOP_PER_ROLLOUT_STEP,
                      FLOP_PER_ROLLOUT_STEP_WITH_NOISE, FLOP_PER_ROLLOUT_STEP_WITH_STANCE_NOISE]
FORM_TRAFFIC_KEY = [None, None, None, "k_rollout", "k_rollout_stance_noise"]
N_FORMS = len(FORM_NAMES)


def main_c4_saturated(args, binding, workloads, arena):
    """Only the saturated serving stream, every rollout launch timed from the
    runtime's first one: a profiler's per-dispatch figures for the rollout
    kernels of this process cover exactly the launches counted here."""
    sat = saturated_run(binding, workloads, args.steps * STEP_S_SATURATED, "serving", arena,
                        timing=3, streams=args.streams, depth=args.depth,
                        noise=args.rollout_noise)
    names = ["fp32_one_lane", "fp32_quad", "fp64", "fp32_one_lane_noise",
             "fp32_one_lane_stance_noise"]
    forms = {names[i]: {"launches": f["launches"], "rollout_steps": f["steps"],
                        "avg_us": f["avg_ns"] * 1e-3}
             for i, f in enumerate(sat.pop("rollout_forms")) if f["launches"]}
    print(json.dumps({"workload": "c4 saturated serving only", "steps": args.steps,
                      "serving_streams": args.streams, "serving_depth": args.depth,
                      "rollout_noise": args.rollout_noise,
                      "rollout_forms": forms,
                      "saturated": sat}), flush=True)


def main_c4(args):
    from paper_2403_11383_amd import binding, workloads
    arena = int(args.arena_gb * (1 << 30))
    K = args.steps
    if args.phase == "saturated":
        return main_c4_saturated(args, binding, workloads, arena)
    # warm-up: code objects, first launches, the pinned pools
    progress("warm-up")
    _ = saturated_run(binding, workloads, 0.05 * max(1, args.warmup), "serving", arena,
                      warmup_ticks=1)
    progress("50 Hz stream, continuous batching")
    serve = serving_run(binding, workloads, K * STEP_S_ARRIVALS, "serving", arena,
                        streams=args.streams, depth=args.depth, noise=args.rollout_noise)
    progress(f"done: {serve['ticks']} ticks; 50 Hz stream, plain single MPPI")
    plain = serving_run(binding, workloads, K * STEP_S_ARRIVALS, "direct", arena)
    progress(f"done: {plain['ticks']} ticks; saturated, continuous batching")
    sat = saturated_run(binding, workloads, K * STEP_S_SATURATED, "serving", arena,
                        timing=args.timing, streams=args.streams, depth=args.depth,
                        noise=args.rollout_noise)
    progress(f"done: {sat['ticks']} ticks; saturated, plain single MPPI")
    sat_plain = saturated_run(binding, workloads, K * STEP_S_SATURATED, "direct", arena)
    progress(f"done: {sat_plain['ticks']} ticks")
    roof = None
    if args.timing and "rollout_forms" in sat:
        forms = sat["rollout_forms"]
        names = FORM_NAMES
        per_step = FORM_FLOP_PER_STEP
        f = max(range(N_FORMS), key=lambda i: forms[i]["avg_ns"] * forms[i]["launches"])
        fo = forms[f]
        flop = fo["steps"] * per_step[f]
        roof = roofline_obj(
            names[f], flop, fo["avg_ns"], fo["launches"], flop_per_rollout_step=per_step[f],
            traffic=(stored_traffic(FORM_TRAFFIC_KEY[f], "c4", fo["steps"] / max(1, fo["launches"]))
                     if FORM_TRAFFIC_KEY[f] else None),
            timed_launches=fo["launches"], duration_us=fo["avg_ns"] * 1e-3,
            rollout_steps_per_launch=fo["steps"] / max(1, fo["launches"]),
            flop_per_launch=flop / max(1, fo["launches"]),
            event_overhead_us=sat["event_overhead_ns"] * 1e-3, event_overhead_taken_us=0.0,
            other_forms={names[i]: {"timed_launches": forms[i]["launches"],
                                    "duration_us": forms[i]["avg_ns"] * 1e-3,
                                    "rollout_steps_per_launch":
                                        forms[i]["steps"] / max(1, forms[i]["launches"])}
                         for i in range(N_FORMS) if i != f and forms[i]["launches"]})
        del sat["rollout_forms"]
    c = workloads.config("c4")
    line = {
        "metric": METRIC, "value": sat["rollout_steps_per_s"], "unit": "rollout-steps/s",
        "n_gpus": 1, "steps": K, "warmup": args.warmup,
        "ms_per_step": sat["elapsed_s"] / K * 1e3,
        "higher_is_better": True, "scaling": "weak",
        "vs_baseline": sat["rollout_steps_per_s"] / sat_plain["rollout_steps_per_s"],
        "vs_baseline_is": "continuous batching / plain single-controller MPPI, saturated "
                          "rollout-steps/s on the same GPU (the paper prints no number)",
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "c4: 256 simulated robots, Poisson 50 Hz ticks each, N in "
                               "{2048,4096,8192}, H in {25,50}, MPPI with gait frequency "
                               f"~U[1.0,2.5] Hz per sample, GRF noise {c['sigma_grf']:g} N, "
                               f"lambda {c['lambda']:g}, Q = I, R = 1e-4 I, friction cone "
                               f"mu {c['mu_fric']:g}, dt {c['dt']:g} s, fixed seeded state "
                               "per robot, continuous batching vs plain single MPPI",
                   "robots": 256, "stream_s_50hz": K * STEP_S_ARRIVALS,
                   "stream_s_saturated": K * STEP_S_SATURATED, "arena_gb": args.arena_gb,
                   "serving_streams": args.streams, "serving_depth": args.depth,
                   "rollout_noise": args.rollout_noise},
        "latency_ms": {"p50": serve["p50_ms"], "p99": serve["p99_ms"],
                       "what": "arrival to completion, 50 Hz Poisson stream, continuous batching"},
        "vs_plain": {"throughput_saturated_x": sat["rollout_steps_per_s"] /
                     sat_plain["rollout_steps_per_s"],
                     "p99_50hz_x": plain["p99_ms"] / serve["p99_ms"],
                     "p99_saturated_x": sat_plain["p99_ms"] / sat["p99_ms"]},
        "serving_50hz": serve, "plain_single_mppi_50hz": plain,
        "saturated": {"serving": sat, "plain_single_mppi": sat_plain},
    }
    if roof is not None:
        line["roofline"] = roof
    if not args.no_cpu_baseline:
        progress("shadow pass")
        recs, total = shadow_pass(binding, workloads, arena, args.shadow_seconds)
        progress(f"done: {len(recs)} shadowed ticks; oracle on the host cores")
        line["cpu_baseline"], line["shadow_oracle"] = cpu_baseline_c4(workloads, recs, total)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
