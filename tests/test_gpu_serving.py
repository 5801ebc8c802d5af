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


def run(mode, cfgs, inps, ticks=3, arena=1 << 30, lanes=1, debug=False):
    from paper_2403_11383_amd import binding
    rt = binding.Runtime(arena_bytes=arena, mode=mode, two_streams=(mode == "serving"))
    rt.set_rollout_lanes(lanes)
    ids = [rt.init_controller(c) for c in cfgs]
    if debug:
        for cid in ids:
            rt.set_debug(cid, True)
    tks = []
    for t in range(ticks):  # every robot submits `ticks` ticks back to back
        for cid, inp in zip(ids, inps):
            tks.append(rt.submit_tick(cid, inp))
    out = [rt.fetch(t, timeout_us=30_000_000) for t in tks]
    if debug:  # costs and phase increments of each controller's last tick
        for i, cid in enumerate(ids):
            J, q, mean = rt.debug_fetch(cid)
            out[(ticks - 1) * len(ids) + i].update(J=J, q_samples=q, mean=mean)
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
    lanes per sample) or a large one (one lane), whose FP32 costs differ in
    rounding only.  For every controller: the phase increments are equal,
    the two forms' costs agree within the FP32 cost tolerance on every
    sample that can influence the update, and each form's action is the
    oracle's update of that form's own costs (selection parity).  The
    actions of the two forms are then compared directly except where the
    choice is a near-tie: a best-sample or elite controller whose deciding
    costs lie within twice the tolerance of each other may pick either
    sample, and both picks were just shown correct."""
    import oracle
    from parity_util import check_costs_fp32, cost_tol, hover, mppi_action_bound
    oracle.build()
    cfgs, inps = fleet()
    a, _ = run("direct", cfgs, inps, ticks=1, lanes=1, debug=True)
    b, _ = run("serving", cfgs, inps, ticks=1, lanes=4, debug=True)
    mg2 = 0.5 * workloads.MASS * workloads.GRAVITY
    ties = 0
    for cfg, inp, x, y in zip(cfgs, inps, a, b):
        np.testing.assert_array_equal(x["q_samples"], y["q_samples"])
        R = cfg["iterations"]
        ke = None if cfg["method"] == "mppi" else \
            (1 if cfg["method"] == "naive" else oracle.elite_count(cfg["N"], cfg["elite_frac"]))
        # the first iteration samples around the same mean in both forms
        check_costs_fp32(y["J"][0], x["J"][0], cfg["lambda"], elite_ke=ke)
        for out in (x, y):
            ref = oracle.tick(cfg, hover(cfg), cfg["mu_f0"], 0, inp, costs_override=out["J"],
                              nthreads=8)
            scale = max(np.abs(ref["grf"]).max(), mg2)
            assert np.abs(out["grf"] - ref["grf"]).max() <= 1e-4 * scale
            # FP32 weights on the GPU, FP64 in the oracle: the frequency within
            # the action tolerance, its phase increment within one count
            assert abs(out["freq_hz"] - ref["freq_hz"]) <= 1e-4 * ref["freq_hz"]
            assert abs(out["q"] - int(ref["q"])) <= 1
        d = np.abs(x["grf"] - y["grf"]).max()
        if cfg["method"] == "mppi":
            # a weighted mean moves with the costs: bounded by the measured
            # cost differences propagated through the weights
            with np.errstate(invalid="ignore"):
                dJ = np.abs(np.asarray(x["J"][0], np.float64) - np.asarray(y["J"][0], np.float64))
            bound = mppi_action_bound(cfg, x["J"][0], dJ, x["mean"][0])
            assert d <= max(1e-4 * mg2, 2.0 * bound), (d, bound)
            continue
        if d <= 1e-4 * mg2:
            continue
        # only a choice between near-tied samples may differ
        near = False
        for r in range(R):
            Js = np.sort(np.asarray(x["J"][r], np.float64))
            near |= bool(abs(Js[ke] - Js[ke - 1]) <= 2.0 * cost_tol(Js[ke - 1]))
        assert near, cfg
        ties += 1
    assert ties <= len(cfgs) // 3


def test_serving_rejects_a_workspace_that_never_fits():
    """A controller whose step workspace exceeds what the arena can lend
    beside the persistent state is refused at submission (SBS_ENOMEM)
    instead of waiting forever; the other controllers keep being served."""
    from paper_2403_11383_amd import binding
    rt = binding.Runtime(arena_bytes=8 << 20, mode="serving", two_streams=True)
    big = rt.init_controller(workloads.config("c4", N=65536, H=50, seed=9))  # ~160 MB of noise
    small = rt.init_controller(workloads.config("c4", N=512, H=10, seed=10))
    inp = workloads.tick_input(workloads.initial_state(np.random.default_rng(3)))
    with pytest.raises(binding.SBSError) as e:
        rt.submit_tick(big, inp)
    assert e.value.code == binding.ENOMEM
    for t in range(3):
        act = rt.fetch(rt.submit_tick(small, inp), timeout_us=30_000_000)
        assert act["tick"] == t
    rt.close()


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


def test_shadow_oracle_on_served_ticks():
    """Served ticks checked against the FP64 oracle, as the benchmark's
    shadow check does: a 16-robot slice of the serving fleet runs a Poisson
    stream in serving mode; for four robots each tick's controller state is
    exported before the tick, and after it the oracle reruns the tick from
    that state.  Per tick: the costs agree within the FP32 cost tolerance on
    every influential sample (or, where the FP64 cost is ill-conditioned,
    within what its conditioning allows FP32), the action is the oracle's update of the GPU's
    own costs within 1e-4 of max(|u|, m g / 2), and against the oracle's own
    costs it is within that bar or the bound the cost tolerance propagates
    through the MPPI weights."""
    import bench
    import oracle
    from paper_2403_11383_amd import binding
    from parity_util import check_costs_fp32, cost_tol, ill_conditioned, mppi_action_bound
    oracle.build()
    recs, total = bench.shadow_pass(binding, workloads, 1 << 30, 0.4, robots=16, every=4)
    print("shadowed ticks", len(recs), "of", total, flush=True)
    assert len(recs) >= 40
    mg2 = 0.5 * workloads.MASS * workloads.GRAVITY
    worst = 0.0
    for rc in recs:
        cfg = rc["cfg"]
        ref = oracle.tick(cfg, rc["mu"], rc["mf"], rc["tick"], rc["inp"], nthreads=8)
        upd = oracle.tick(cfg, rc["mu"], rc["mf"], rc["tick"], rc["inp"], costs_override=rc["J"],
                          nthreads=8)
        scale = max(np.abs(ref["grf"]).max(), mg2)
        Jg, Jr = np.asarray(rc["J"][0], np.float64), ref["costs"][0]
        ill = ill_conditioned(cfg, rc["inp"], rc["mu"], rc["tick"], ref["q_samples"][0], Jg, Jr,
                              cfg["lambda"])
        check_costs_fp32(Jg, Jr, cfg["lambda"], well=~ill)
        assert np.abs(rc["grf"] - upd["grf"]).max() <= 1e-4 * scale
        # the ill-conditioned samples move the weights by their own errors
        with np.errstate(invalid="ignore"):
            eps = np.where(ill, np.abs(Jg - Jr), cost_tol(Jr))
        bound = mppi_action_bound(cfg, Jr, eps, ref["mean"][0], tick=rc["tick"],
                                  mu_row0=rc["mu"][0])
        err = np.abs(rc["grf"] - ref["grf"]).max()
        assert err <= max(1e-4 * scale, bound), (err, bound, scale)
        worst = max(worst, err / scale)
    print("worst action error against the oracle (relative)", worst, flush=True)


def test_fetch_ready_returns_every_tick_once():
    """sbs_fetch_ready hands back completed ticks in bulk: over repeated
    calls every submitted ticket comes back exactly once, with the action
    that fetching it alone gives (serving mode, three ticks per robot)."""
    import time
    from paper_2403_11383_amd import binding
    cfgs, inps = fleet(8)
    one, _ = run("serving", cfgs, inps, ticks=3)
    rt = binding.Runtime(arena_bytes=1 << 30, mode="serving", two_streams=True)
    rt.set_rollout_lanes(1)
    ids = [rt.init_controller(c) for c in cfgs]
    tks = []
    for t in range(3):
        for cid, inp in zip(ids, inps):
            tks.append(rt.submit_tick(cid, inp))
    got = {}
    t0 = time.time()
    while len(got) < len(tks) and time.time() - t0 < 30:
        for tk, a in rt.fetch_ready(5):  # fewer than the ticks: several calls
            assert tk not in got
            got[tk] = a
    rt.close()
    assert sorted(got) == sorted(tks)
    for tk, a in zip(tks, one):
        same(got[tk], a)
