"""Benchmark of one GPU: closed-loop receding-horizon MPPI with per-sample gait
frequency (N = 10240 samples, H = 50 steps, dt = 0.02 s, GRF noise 25 N,
friction cone mu = 0.5, 40 N lateral push from tick 30), FP32 rollouts.

A step is one control tick: noise, rollouts, selection and mean update on
the GPU (through the C ABI), then one step of the host plant with the
returned action.  The value is rollout-steps per second (N x H x iterations
per tick) over the timed ticks, with the inputs already resident.  One JSON
line is printed; see the design doc for the roofline and baseline definitions.
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
# Algorithmic FP32 work of one rollout step (policy, friction clip, stage cost,
# attitude, footholds, SRBD derivative and Euler update), counted with
# add/sub/mul = 1, fma = 2, each transcendental (sin, cos, sqrt, rcp, rsqrt) = 1.
FLOP_PER_ROLLOUT_STEP = 384
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


def closed_loop(rt, binding, workloads, cfg, ticks, warmup, push_from=30, push=40.0):
    cid = rt.init_controller(cfg)
    rng = np.random.default_rng(cfg["seed"])
    x0 = workloads.initial_state(rng)
    plant = binding.Plant(cfg, x0, workloads.feet_under_hips(x0), phase=0)
    loop = binding.ClosedLoop(rt, cid, plant, v_ref=(0.3, 0.0, 0.0), z_ref=workloads.HEIGHT)
    lat, acts = [], []
    t_start = None
    import torch
    no_push, push_f = (0.0, 0.0, 0.0), (0.0, push, 0.0)
    for t in range(warmup + ticks):
        if t == warmup:
            torch.cuda.synchronize()
            rt.timing()  # reset the stage-timing accumulators
            t_start = time.perf_counter()
        a = loop.step(push_f if t >= push_from else no_push)
        if t >= warmup:
            # submit-to-visible latency as recorded by the runtime
            lat.append((a.t_done_ns - a.t_submit_ns) * 1e-6)
            acts.append((a.flags, a.freq_hz))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    timing = rt.timing()
    rt.destroy_controller(cid)
    return elapsed, lat, acts, timing, plant


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
    mu = np.tile([0.0, 0.0, 0.5 * cfg["mass"] * cfg["gravity"]] * 4, (cfg["H"], 1))
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
    return {"value": steps / dt, "unit": "rollout-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"{n} full ticks (N={cfg['N']}, H={cfg['H']}) from the closed loop's "
                      f"initial state, {dt:.1f} s wall"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--timing", type=int, default=1,
                    help="HIP events: 0 none, 1 around the rollout stage, 2 around every stage")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    from paper_2403_11383_amd import binding, workloads
    import torch
    cfg = workloads.config("c1")
    rt = binding.Runtime(arena_bytes=4 << 30)
    rt.set_timing(args.timing)
    elapsed, lat, acts, timing, plant = closed_loop(rt, binding, workloads, cfg, args.steps,
                                                    args.warmup)
    rt.close()
    N, H, R = cfg["N"], cfg["H"], cfg["iterations"]
    steps_total = N * H * R * args.steps
    value = steps_total / elapsed
    t_roll = timing["rollout_ns"] * 1e-9
    achieved = N * H * FLOP_PER_ROLLOUT_STEP / t_roll / 1e12 if t_roll > 0 else 0.0
    line = {
        "metric": METRIC, "value": value, "unit": "rollout-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "c1: closed-loop MPPI, gait frequency ~U[1.0,2.5] Hz per sample, "
                               "N=10240, H=50, dt=0.02 s, 40 N lateral push from tick 30",
                   "N": N, "H": H, "iterations": R, "ticks": args.steps},
        "latency_ms": {"p50": pct(lat, 50), "p99": pct(lat, 99), "max": float(np.max(lat))},
        "stage_us": {k: timing[k] * 1e-3 for k in ("noise_ns", "rollout_ns", "select_ns",
                                                   "update_ns") if timing[k] > 0},
        "roofline": {"kernel": "k_rollout<float>", "bound": "alu", "achieved": achieved,
                     "peak": PEAK_FP32_VALU_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_VALU_TFLOPS,
                     "peak_published_packed": PEAK_FP32_PUBLISHED_TFLOPS,
                     "frac_of_published": achieved / PEAK_FP32_PUBLISHED_TFLOPS,
                     "traffic": stored_traffic("k_rollout", "c1"),
                     "flop_per_launch": N * H * FLOP_PER_ROLLOUT_STEP},
        "closed_loop": {"final_x": [round(float(v), 4) for v in plant.x],
                        "nonfinite_ticks": int(sum(f & 1 for f, _ in acts)),
                        "freq_hz_last": acts[-1][1]},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(cfg, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
