"""Serving runtime (continuous batching with memory admission) on the GPU:
results are the ones the controller gives alone, per-robot tick order is
kept, and a small arena forces admission waits without changing results."""
import numpy as np
import pytest

from paper_2403_11383_amd import workloads

pytestmark = pytest.mark.gpu


def fleet(n=12):
    rng = np.random.default_rng(21)
    cfgs, inps = [], []
    for r in range(n):
        N = int(rng.choice([512, 1024, 2048]))
        H = int(rng.choice([10, 25]))
        method = ["mppi", "elite", "naive"][r % 3]
        cfgs.append(workloads.config("c4", N=N, H=H, seed=500 + r, method=method,
                                     iterations=2 if method != "mppi" else 1))
        inps.append(workloads.tick_input(workloads.initial_state(rng)))
    return cfgs, inps


def run(mode, cfgs, inps, ticks=3, arena=1 << 30, lanes=1):
    from paper_2403_11383_amd import binding
    rt = binding.Runtime(arena_bytes=arena, mode=mode, two_streams=(mode == "serving"))
    rt.set_rollout_lanes(lanes)
    ids = [rt.init_controller(c) for c in cfgs]
    tks = []
    for t in range(ticks):  # every robot submits `ticks` ticks back to back
        for cid, inp in zip(ids, inps):
            tks.append(rt.submit_tick(cid, inp))
    out = [rt.fetch(t, timeout_us=30_000_000) for t in tks]
    stats = rt.stats()
    rt.close()
    return out, stats


def same(a, b):
    np.testing.assert_array_equal(a["grf"], b["grf"])
    assert a["best_cost"] == b["best_cost"] and a["q"] == b["q"]
    assert a["tick"] == b["tick"] and a["controller"] == b["controller"]


def test_serving_equals_direct():
    cfgs, inps = fleet()
    direct, _ = run("direct", cfgs, inps)
    served, st = run("serving", cfgs, inps)
    assert all(r is not None for r in served)
    for a, b in zip(direct, served):
        same(a, b)
    assert st["ticks"] == len(served)
    assert st["batches"] < len(served)  # ticks were fused


def test_serving_tick_order_per_robot():
    cfgs, inps = fleet(6)
    served, _ = run("serving", cfgs, inps, ticks=4)
    for r in range(6):
        ticks = [served[t * 6 + r]["tick"] for t in range(4)]
        assert ticks == [0, 1, 2, 3]


def test_serving_memory_admission():
    cfgs, inps = fleet()
    direct, _ = run("direct", cfgs, inps, ticks=2)
    # an arena that holds the persistent state and the workspaces of only a
    # few of the twelve controllers at once (the largest, N=2048 H=25, takes
    # about 2.5 MB; the fleet together about 12 MB)
    small = 6 << 20
    served, st = run("serving", cfgs, inps, ticks=2, arena=small)
    for a, b in zip(direct, served):
        same(a, b)
    assert st["admit_waits"] > 0


def test_serving_auto_lanes_within_tolerance():
    """With the automatic lane policy a tick may run in a small batch (four
    lanes per sample) or a large one (one lane): the results agree within
    FP32 rounding."""
    cfgs, inps = fleet()
    a, _ = run("direct", cfgs, inps, ticks=1, lanes=1)
    b, _ = run("serving", cfgs, inps, ticks=1, lanes=4)
    mg2 = 0.5 * workloads.MASS * workloads.GRAVITY
    for x, y in zip(a, b):
        assert abs(x["best_cost"] - y["best_cost"]) <= 1e-4 * abs(x["best_cost"]) + 1e-3
        if np.abs(x["grf"] - y["grf"]).max() > 1e-4 * mg2:
            # only a near-tie of the two best samples may flip the choice
            pytest.skip("near-tie between best samples")


def test_fetch_many_equals_one_by_one():
    """sbs_fetch_actions returns, in ticket order, the actions that
    sbs_fetch_action returns one ticket at a time (serving mode, so the
    tickets complete out of submission order inside the runtime)."""
    from paper_2403_11383_amd import binding
    cfgs, inps = fleet(8)
    one, _ = run("serving", cfgs, inps, ticks=2)
    rt = binding.Runtime(arena_bytes=1 << 30, mode="serving", two_streams=True)
    rt.set_rollout_lanes(1)
    ids = [rt.init_controller(c) for c in cfgs]
    tks = []
    for t in range(2):
        for cid, inp in zip(ids, inps):
            tks.append(rt.submit_tick(cid, inp))
    arr = (binding.C.c_uint64 * len(tks))(*tks)
    acts = (binding.Action * len(tks))()
    rt.fetch_many(arr, acts, timeout_us=30_000_000)
    rt.close()
    for a, b in zip(one, acts):
        same(a, binding.action_dict(b))
