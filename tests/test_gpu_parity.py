"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs.

Bars:
* integers (sampled phase increments, contact flags, elite membership):
  bit-exact; the FP32 noise z: bit-exact.
* FP64 controllers: costs within 1e-10 relative, means and actions within
  1e-10 of max(|u|, m g / 2).
* FP32 controllers: per-sample costs within EPS_J (see cost_tol), actions
  within 1e-4 of max(|u|, m g / 2) when the oracle is fed the GPU's own costs
  (selection then identical), and against the oracle's own costs within the
  bound propagated from EPS_J through the MPPI weights.
"""
import numpy as np
import pytest

import oracle
from paper_2403_11383_amd import workloads
from parity_util import MG2, check_costs_fp32, check_fp64, cost_tol, hover, run_pair

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rt():
    from paper_2403_11383_amd import binding
    r = binding.Runtime(arena_bytes=2 << 30)
    yield r
    r.close()


@pytest.fixture(scope="module", autouse=True)
def _oracle_built():
    oracle.build()


# ---------------------------------------------------------------------------
# noise
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("mode", ["uniform", "gaussian", "fixed", "set"])
def test_noise_bit_exact(rt, mode):
    cfg = workloads.config("c1", N=333, H=7, freq_mode=mode, sigma_f=0.4, seed=0xDEADBEEF12345,
                           f_set=(1.4, 2.0, 2.4))
    cid = rt.init_controller(cfg)
    for tick, r in ((0, 0), (5, 0), (123456, 2)):
        z, q = rt.debug_noise(cid, tick, r)
        zr = oracle.noise_block(cfg["seed"], tick, r, 333, 7)
        assert np.array_equal(z.view(np.uint32), zr.view(np.uint32)), (tick, r)
        qr = np.array([oracle.freq_q(cfg, 1.4, 0.4, tick, r, k) for k in range(333)], np.uint32)
        assert np.array_equal(q, qr), (tick, r)
    rt.destroy_controller(cid)


def test_noise_bit_exact_many_draws(rt):
    """4000 samples x 40 steps x 12 = 1.92M Gaussians: every FP32 bit of
    every one equal to the oracle's."""
    cfg = workloads.config("c1", N=4000, H=40, seed=77)
    cid = rt.init_controller(cfg)
    z, q = rt.debug_noise(cid, 9, 1)
    zr = oracle.noise_block(77, 9, 1, 4000, 40)
    np.testing.assert_array_equal(z.view(np.uint32), zr.view(np.uint32))
    assert abs(float(z.mean())) < 5 / np.sqrt(z.size)
    assert abs(float(z.var()) - 1.0) < 5 * np.sqrt(2.0 / z.size)
    rt.destroy_controller(cid)


# ---------------------------------------------------------------------------
# FP64 controllers: tight parity
# ---------------------------------------------------------------------------
def test_c0_fp64_plain_mppi(rt):
    cfg = workloads.config("c0")
    out, ref = run_pair(rt, cfg, workloads.c0_input())
    check_fp64(out, ref, cfg)
    assert out["act"]["best_cost"] == pytest.approx(ref["best_cost"], rel=1e-10)


@pytest.mark.parametrize("N,H", [(1, 1), (63, 3), (65, 9), (1025, 4), (3000, 17)])
def test_fp64_ragged_sizes(rt, N, H):
    cfg = workloads.config("c1", N=N, H=H, precision="fp64", seed=N * 7 + H)
    inp = workloads.tick_input(workloads.initial_state(np.random.default_rng(N)), phase_robot=N * 99991)
    out, ref = run_pair(rt, cfg, inp, tick=N)
    check_fp64(out, ref, cfg)


@pytest.mark.parametrize("method", ["elite", "naive"])
def test_fp64_elite_and_naive(rt, method):
    cfg = workloads.config("c2", N=2500, H=12, precision="fp64", method=method, iterations=3,
                           seed=21)
    inp = workloads.tick_input(workloads.initial_state(np.random.default_rng(3)), v_ref=(0.2, 0, 0))
    out, ref = run_pair(rt, cfg, inp, tick=4)
    check_fp64(out, ref, cfg)


def test_fp64_duty_edges_and_pace(rt):
    for duty, offs in ((0.0, workloads.TROT_OFFSETS), (1.0, workloads.TROT_OFFSETS),
                       (0.5, workloads.PACE_OFFSETS), (0.7, (0, 1 << 30, 1 << 31, 3 << 30))):
        cfg = workloads.config("c1", N=200, H=10, precision="fp64", duty=duty,
                               phase_offset=list(offs), seed=5)
        inp = workloads.tick_input(workloads.initial_state(np.random.default_rng(4)))
        out, ref = run_pair(rt, cfg, inp)
        check_fp64(out, ref, cfg)


@pytest.mark.parametrize("method", ["naive", "mppi"])
def test_fp64_frequency_set_and_pace(rt, method):
    """The paper's discrete frequency set (nominal, 2.0, 2.4 Hz) with the
    best-sample update and a pacing gait."""
    cfg = workloads.config("c2", N=1200, H=14, precision="fp64", method=method, iterations=2,
                           freq_mode="set", f_set=(1.4, 2.0, 2.4),
                           phase_offset=list(workloads.PACE_OFFSETS), seed=31)
    inp = workloads.tick_input(workloads.initial_state(np.random.default_rng(31)),
                               phase_robot=1 << 30)
    out, ref = run_pair(rt, cfg, inp, tick=6)
    check_fp64(out, ref, cfg)
    qs = {oracle.q_of_freq(f, cfg["dt"]) for f in (1.4, 2.0, 2.4)}
    assert set(np.unique(out["q"])) <= qs


def test_nonfinite_costs_keep_mean(rt):
    cfg = workloads.config("c1", N=128, H=5, precision="fp64")
    x0 = workloads.initial_state(np.random.default_rng(1))
    x0[6] = 1e200  # every cost overflows to +inf
    inp = workloads.tick_input(x0)
    out, ref = run_pair(rt, cfg, inp)
    assert ref["flags"] == 1 and out["act"]["flags"] == 1
    check_fp64(out, ref, cfg)


def test_fp32_mppi_lambda_beyond_fp32_reciprocal(rt):
    """lambda = 1e-45: its reciprocal overflows FP32.  The update is the
    argmin limit of Alg. 4 (the best sample alone), as the FP64 oracle's
    update of the same costs gives it, with no NaN from 0 * inf."""
    cfg = workloads.config("c1", N=500, H=10, seed=5, **{"lambda": 1e-45})
    inp = workloads.tick_input(workloads.initial_state(np.random.default_rng(5)))
    out, _ = run_pair(rt, cfg, inp)
    assert out["act"]["flags"] == 0 and np.all(np.isfinite(out["act"]["grf"]))
    assert out["act"]["n_active"] == 1
    ref = oracle.tick(cfg, hover(cfg), 1.4, 0, inp, costs_override=out["J"], nthreads=8)
    scale = max(np.abs(ref["grf"]).max(), MG2)
    assert np.abs(out["act"]["grf"] - ref["grf"]).max() <= 1e-4 * scale
    assert np.abs(out["mean"] - ref["mean"]).max() <= 1e-4 * max(np.abs(ref["mean"]).max(), MG2)


def test_nonfinite_state_rejected(rt):
    from paper_2403_11383_amd import binding
    cfg = workloads.config("c1", N=64, H=5)
    cid = rt.init_controller(cfg)
    x0 = workloads.initial_state(np.random.default_rng(1))
    x0[2] = float("nan")
    with pytest.raises(binding.SBSError) as e:
        rt.submit_tick(cid, workloads.tick_input(x0))
    assert e.value.code == binding.EINVAL
    rt.destroy_controller(cid)


# ---------------------------------------------------------------------------
# FP32 controllers
# ---------------------------------------------------------------------------
def mppi_propagated_bound(ref, cfg, epsJ):
    """|d mean| <= sum_k w_k |theta_k - mean| |dJ_k - sum_i w_i dJ_i| / lambda
    with |dJ_k| <= epsJ_k; evaluated with the oracle's weights and samples."""
    J = ref["costs"][-1]
    w, *_ = oracle.mppi_weights(J, cfg["lambda"])
    H = cfg["H"]
    z = oracle.noise_block(cfg["seed"], 0, 0, cfg["N"], 1)[:, 0, :].astype(np.float64)
    th0 = hover(cfg)[0][None] + cfg["sigma_grf"] * z   # first step only
    dev = np.abs(th0 - ref["mean"][0][None])
    spread = epsJ + (w * epsJ).sum()
    return float((w[:, None] * dev * spread[:, None]).sum(0).max() / cfg["lambda"])


@pytest.fixture(params=[1, 4], ids=["lanes1", "lanes4"])
def lanes(request, rt):
    rt.set_rollout_lanes(request.param)
    yield request.param
    rt.set_rollout_lanes(0)


def test_fp32_mppi_small(rt, lanes):
    cfg = workloads.config("c1", N=777, H=20, seed=11)
    inp = workloads.tick_input(workloads.initial_state(np.random.default_rng(11)))
    out, ref = run_pair(rt, cfg, inp)
    np.testing.assert_array_equal(out["q"], ref["q_samples"])
    Jr = ref["costs"]
    check_costs_fp32(out["J"][0], Jr[0], cfg["lambda"])
    scale = max(np.abs(ref["grf"]).max(), MG2)
    # selection parity: the oracle's update on the GPU's own costs
    ref2 = oracle.tick(cfg, hover(cfg), 1.4, 0, inp, costs_override=out["J"], nthreads=8)
    assert np.abs(out["act"]["grf"] - ref2["grf"]).max() <= 1e-4 * scale
    assert np.abs(out["mean"] - ref2["mean"]).max() <= 1e-4 * max(np.abs(ref2["mean"]).max(), MG2)
    # against the oracle's own costs: within the propagated bound
    bound = mppi_propagated_bound(ref, cfg, cost_tol(Jr[-1]))
    assert np.abs(out["act"]["grf"] - ref["grf"]).max() <= max(1e-4 * scale, bound)
    np.testing.assert_array_equal(out["act"]["contact"], ref["contact"])


@pytest.mark.parametrize("H", [1, 2, 3])
def test_fp32_short_horizons(rt, lanes, H):
    # the rollouts load the next step's noise one step ahead; at the last
    # step (the first, for H = 1) they read their own row again
    cfg = workloads.config("c1", N=333, H=H, seed=40 + H)
    inp = workloads.tick_input(workloads.initial_state(np.random.default_rng(40 + H)))
    out, ref = run_pair(rt, cfg, inp)
    np.testing.assert_array_equal(out["q"], ref["q_samples"])
    check_costs_fp32(out["J"][0], ref["costs"][0], cfg["lambda"])
    # no rollout tumbles within three steps: every cost agrees, and a wrong
    # noise row would move it far beyond FP32 rounding
    np.testing.assert_allclose(out["J"][0], ref["costs"][0], rtol=1e-4)


def test_fp32_elite_selection(rt, lanes):
    cfg = workloads.config("c2", N=3000, H=16, seed=12)
    inp = workloads.tick_input(workloads.initial_state(np.random.default_rng(12)), v_ref=(-0.3, 0, 0))
    out, ref = run_pair(rt, cfg, inp)
    # iteration 0 samples from the same mean: costs comparable sample by sample
    check_costs_fp32(out["J"][0], ref["costs"][0], elite_ke=oracle.elite_count(3000, 0.1))
    np.testing.assert_array_equal(out["q"][0], ref["q_samples"][0])
    ref2 = oracle.tick(cfg, hover(cfg), 1.4, 0, inp, costs_override=out["J"], nthreads=8)
    scale = max(np.abs(ref2["mean"]).max(), MG2)
    assert np.abs(out["mean"] - ref2["mean"]).max() <= 1e-4 * scale
    assert np.abs(out["act"]["grf"] - ref2["grf"]).max() <= 1e-4 * scale
    assert abs(out["act"]["freq_hz"] - ref2["freq_hz"]) <= 1e-6


# ---------------------------------------------------------------------------
# runtime properties
# ---------------------------------------------------------------------------
def test_determinism_and_resume(rt):
    cfg = workloads.config("c1", N=1500, H=15, seed=99)
    inp = workloads.tick_input(workloads.initial_state(np.random.default_rng(5)))
    a = rt.init_controller(cfg)
    b = rt.init_controller(cfg)
    ra = [rt.tick(a, inp) for _ in range(3)]
    mu, mf, tk = rt.get_state(a)
    rb = [rt.tick(b, inp) for _ in range(3)]
    for x, y in zip(ra, rb):
        np.testing.assert_array_equal(x["grf"], y["grf"])
        assert x["q"] == y["q"] and x["best_cost"] == y["best_cost"]
    # export after 3 ticks, import into a fresh controller, continue
    c = rt.init_controller(cfg)
    rt.set_state(c, mu, mf, tk)
    x = rt.tick(a, inp)
    y = rt.tick(c, inp)
    np.testing.assert_array_equal(x["grf"], y["grf"])
    assert x["tick"] == y["tick"] == 3
    for cid in (a, b, c):
        rt.destroy_controller(cid)


def test_batch_equals_alone(rt):
    cfgs = [workloads.config("c1", N=n, H=h, seed=s, method=m, iterations=it)
            for n, h, s, m, it in ((700, 12, 1, "mppi", 1), (2100, 30, 2, "elite", 3),
                                   (64, 5, 3, "naive", 2), (5000, 21, 4, "mppi", 1))]
    cfgs.append(workloads.config("c0", N=300, H=8, seed=5))  # an FP64 one in the mix
    rng = np.random.default_rng(8)
    inps = [workloads.tick_input(workloads.initial_state(rng)) for _ in cfgs]
    alone = []
    for c, i in zip(cfgs, inps):
        cid = rt.init_controller(c)
        alone.append(rt.tick(cid, i))
        rt.destroy_controller(cid)
    ids = [rt.init_controller(c) for c in cfgs]
    tks = rt.submit_batch(ids, inps)
    mixed = [rt.fetch(t) for t in tks]
    for a, m in zip(alone, mixed):
        np.testing.assert_array_equal(a["grf"], m["grf"])
        assert a["q"] == m["q"] and a["best_cost"] == m["best_cost"]
    for cid in ids:
        rt.destroy_controller(cid)


def test_chunked_update_equals_one_row_per_workgroup(rt):
    """A batch of 192 controllers at H = 60, 80 elite or best-sample ones per
    precision (4800 mean rows per launch), gives each elite / best-sample
    update workgroup two rows; a controller alone gets one.  Each row is
    reduced as a one-row workgroup reduces it, so every action and mean is
    bit-identical (MPPI, elite and best sample, FP32 and FP64)."""
    rng = np.random.default_rng(41)
    cfgs, inps = [], []
    for i in range(192):
        method = ["elite", "naive", "elite", "naive", "elite", "mppi"][(i // 2) % 6]
        cfgs.append(workloads.config("c4", N=int(rng.choice([256, 400, 600])), H=60,
                                     method=method, iterations=1 if method == "mppi" else 2,
                                     precision="fp64" if i % 2 else "fp32", seed=700 + i))
        inps.append(workloads.tick_input(workloads.initial_state(rng)))
    rt.set_rollout_lanes(1)  # the same rollout form alone and in the batch
    try:
        alone = []
        for c, inp in zip(cfgs, inps):
            cid = rt.init_controller(c)
            alone.append((rt.tick(cid, inp), rt.get_state(cid)[0]))
            rt.destroy_controller(cid)
        ids = [rt.init_controller(c) for c in cfgs]
        batch = [rt.fetch(t) for t in rt.submit_batch(ids, inps)]
        for cid, (a, mu), b in zip(ids, alone, batch):
            np.testing.assert_array_equal(a["grf"], b["grf"])
            assert a["q"] == b["q"] and a["best_cost"] == b["best_cost"]
            np.testing.assert_array_equal(mu, rt.get_state(cid)[0])
            rt.destroy_controller(cid)
    finally:
        rt.set_rollout_lanes(0)


@pytest.mark.parametrize("use_graph", [False, True])
def test_plan_replay_matches_direct(rt, use_graph):
    cfgs = [workloads.config("c1", N=n, H=h, seed=s) for n, h, s in ((900, 10, 1), (2000, 25, 2))]
    cfgs.append(workloads.config("c2", N=1200, H=8, seed=3))
    rng = np.random.default_rng(9)
    inps = [workloads.tick_input(workloads.initial_state(rng)) for _ in cfgs]
    direct_ids = [rt.init_controller(c) for c in cfgs]
    plan_ids = [rt.init_controller(c) for c in cfgs]
    plan = rt.plan_create(plan_ids, use_graph=use_graph)
    for t in range(3):
        d = [rt.fetch(x) for x in rt.submit_batch(direct_ids, inps)]
        p = [rt.fetch(x) for x in rt.plan_submit(plan, inps)]
        for a, b in zip(d, p):
            np.testing.assert_array_equal(a["grf"], b["grf"])
            assert a["q"] == b["q"] and a["tick"] == b["tick"] == t
    rt.plan_destroy(plan)
    for cid in direct_ids + plan_ids:
        rt.destroy_controller(cid)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_stance_pair_form_equals_four_leg_form(rt, precision):
    """For the diagonal trot at duty 1/2 the one-lane rollout forms only the
    stance pair's forces; the four-leg form forms every leg and masks the
    swing pair to zero.  The swing legs add exact zeros, so every cost of
    the two forms is the same number (MPPI and elite controllers, per-step
    and spline GRFs)."""
    cfgs = [workloads.config("c1", N=3000, H=50, seed=61, precision=precision),
            workloads.config("c2", N=2500, H=30, seed=62, precision=precision),
            workloads.config("c1", N=1500, H=40, knots=8, seed=63, precision=precision)]
    rt.set_rollout_lanes(1)
    rt.set_rollout_noise(1)  # both forms store every noise row
    try:
        for cfg in cfgs:
            inp = workloads.tick_input(workloads.initial_state(np.random.default_rng(cfg["seed"])))
            res = {}
            for pairs in (True, False):
                rt.set_rollout_pairs(pairs)
                cid = rt.init_controller(cfg)
                rt.set_debug(cid, True)
                act = rt.tick(cid, inp)
                res[pairs] = (act, rt.debug_fetch(cid))
                rt.destroy_controller(cid)
            (a1, (J1, q1, m1)), (a0, (J0, q0, m0)) = res[True], res[False]
            np.testing.assert_array_equal(q1, q0)
            diff = np.flatnonzero(J1.view(np.uint64) != J0.view(np.uint64))
            print(cfg["method"], precision, "costs differing in any bit:", diff.size, flush=True)
            np.testing.assert_array_equal(J1, J0)
            np.testing.assert_array_equal(a1["grf"], a0["grf"])
            np.testing.assert_array_equal(m1, m0)
    finally:
        rt.set_rollout_pairs(True)
        rt.set_rollout_noise(2)
        rt.set_rollout_lanes(0)


def test_noise_made_in_rollout_equals_noise_launch(rt):
    """One-lane FP32 rollouts that make their noise rows themselves and store
    them (sbs_set_rollout_noise 1) compute exactly what the separate noise
    launch (0) gives: every cost, sampled increment, action and updated mean
    is bit-equal, over two consecutive ticks (the second warm-started).
    Cases: MPPI with few and with all samples weighed (lambda 1e9), an elite
    controller with three iterations whose update reads the stored rows, a
    four-leg gait and a batch of them all."""
    cfgs = [workloads.config("c1", N=3000, H=50, seed=81),
            workloads.config("c2", N=2500, H=30, seed=82),
            workloads.config("c1", N=1200, H=20, seed=83, duty=0.6),  # four-leg form
            workloads.config("c4", N=2600, H=12, seed=85, **{"lambda": 1e9})]
    rng = np.random.default_rng(84)
    inps = [workloads.tick_input(workloads.initial_state(rng)) for _ in cfgs]
    rt.set_rollout_lanes(1)
    try:
        res = {}
        for mode in (0, 1):
            rt.set_rollout_noise(mode)
            ids = [rt.init_controller(c) for c in cfgs]
            for cid in ids:
                rt.set_debug(cid, True)
            out = []
            for _ in range(2):
                acts = [rt.fetch(t) for t in rt.submit_batch(ids, inps)]
                out.append([(a, rt.debug_fetch(cid), rt.get_state(cid)[0])
                            for a, cid in zip(acts, ids)])
            res[mode] = out
            for cid in ids:
                rt.destroy_controller(cid)
        for tick in range(2):
            for c, ((a1, (J1, q1, m1), mu1), (a0, (J0, q0, m0), mu0)) in enumerate(
                    zip(res[1][tick], res[0][tick])):
                where = str((tick, c))
                np.testing.assert_array_equal(q1, q0, err_msg=where)
                np.testing.assert_array_equal(J1, J0, err_msg=where)
                np.testing.assert_array_equal(a1["grf"], a0["grf"], err_msg=where)
                np.testing.assert_array_equal(m1, m0, err_msg=where)
                np.testing.assert_array_equal(mu1, mu0, err_msg=where)
    finally:
        rt.set_rollout_noise(2)
        rt.set_rollout_lanes(0)


def test_stance_noise_rollouts_against_oracle(rt):
    """MPPI controllers in the stance-pair form whose rollouts draw only the
    stance legs' Gaussians and store no noise (sbs_set_rollout_noise 2), the
    update drawing the rows of the samples it weighs.  This form is compiled apart
    from the others, so its costs agree with theirs within FP32 rounding,
    not bit for bit.  Against the FP64 oracle from the state each controller
    holds before each of three consecutive ticks: every sampled increment
    is equal, the influential costs meet the FP32 bars, and the update
    reproduces the oracle's update of the GPU's own costs (selection parity)
    -- with few weighed samples (the list) and with all of them weighed
    (lambda 1e9: the update draws every row).  A four-leg controller in the
    same batch keeps the stored-row form."""
    cfgs = [workloads.config("c1", N=3000, H=50, seed=81),
            workloads.config("c4", N=2600, H=12, seed=85, **{"lambda": 1e9}),
            workloads.config("c4", N=2048, H=25, seed=86),
            workloads.config("c1", N=1200, H=20, seed=83, duty=0.6)]
    rng = np.random.default_rng(84)
    inps = [workloads.tick_input(workloads.initial_state(rng)) for _ in cfgs]
    rt.set_rollout_lanes(1)
    rt.set_rollout_noise(2)
    ids = [rt.init_controller(c) for c in cfgs]
    try:
        for cid in ids:
            rt.set_debug(cid, True)
        for tick in range(3):
            before = [rt.get_state(cid) for cid in ids]
            acts = [rt.fetch(t) for t in rt.submit_batch(ids, inps)]
            for c, (cfg, inp, cid, a, (mu, mf, tk)) in enumerate(zip(cfgs, inps, ids, acts, before)):
                J, q, mean = rt.debug_fetch(cid)
                own = oracle.tick(cfg, mu, mf, tk, inp, nthreads=8)
                np.testing.assert_array_equal(q, own["q_samples"], err_msg=str((tick, c)))
                check_costs_fp32(J[0], own["costs"][0], cfg["lambda"])
                sel = oracle.tick(cfg, mu, mf, tk, inp, costs_override=J, nthreads=8)
                scale = max(np.abs(sel["mean"]).max(), MG2)
                assert np.abs(mean - sel["mean"]).max() <= 1e-4 * scale, (tick, c)
                assert np.abs(a["grf"] - sel["grf"]).max() <= 1e-4 * scale, (tick, c)
        assert acts[1]["n_active"] > 2048 and acts[2]["n_active"] <= 32
    finally:
        for cid in ids:
            rt.destroy_controller(cid)
        rt.set_rollout_noise(2)
        rt.set_rollout_lanes(0)


def test_fp32_lane_forms_agree(rt):
    """The one-lane and four-lane rollouts agree on every cost within FP32
    rounding of the same arithmetic in a different order."""
    cfg = workloads.config("c1", N=3000, H=50, seed=31)
    inp = workloads.tick_input(workloads.initial_state(np.random.default_rng(31)))
    res = {}
    for lanes in (1, 4):
        rt.set_rollout_lanes(lanes)
        cid = rt.init_controller(cfg)
        rt.set_debug(cid, True)
        rt.tick(cid, inp)
        res[lanes] = rt.debug_fetch(cid)
        rt.destroy_controller(cid)
    rt.set_rollout_lanes(0)
    np.testing.assert_array_equal(res[1][1], res[4][1])  # same sampled increments
    J1, J4 = res[1][0][0], res[4][0][0]
    ref = oracle.tick(cfg, hover(cfg), 1.4, 0, inp, nthreads=8)["costs"][0]
    check_costs_fp32(J1, ref, cfg["lambda"])
    check_costs_fp32(J4, ref, cfg["lambda"])


def test_plan_forms_and_autotune(rt):
    """Every rollout form of a plan gives bit-identical results within one
    lane form and one noise form (workgroup size and unroll do not change
    any sample's arithmetic; the noise rows are stored, sbs_set_rollout_noise
    1); the autotuner restores the controllers' state and leaves a working
    plan."""
    cfgs = [workloads.config("c1", N=n, H=h, seed=s, method=m, iterations=it)
            for n, h, s, m, it in ((1500, 22, 1, "mppi", 1), (3000, 40, 2, "elite", 3),
                                   (700, 31, 3, "mppi", 1))]
    rng = np.random.default_rng(12)
    inps = [workloads.tick_input(workloads.initial_state(rng)) for _ in cfgs]
    ids = [rt.init_controller(c) for c in cfgs]
    rt.set_rollout_noise(1)
    plan = rt.plan_create(ids, use_graph=True)
    rt.set_rollout_noise(2)
    state0 = [rt.get_state(c) for c in ids]

    def run(form):
        rt.plan_set_tune(plan, *form)
        for c, (mu, mf, tk) in zip(ids, state0):
            rt.set_state(c, mu, mf, tk)
        return [rt.fetch(t) for t in rt.plan_submit(plan, inps)]

    for lanes, forms in ((1, [(64, 1), (128, 1), (256, 1), (64, 2), (128, 2)]),
                         (4, [(64, 1), (128, 1), (256, 1)])):
        ref = run((lanes, *forms[0]))
        for f in forms[1:]:
            out = run((lanes, *f))
            for a, b in zip(ref, out):
                np.testing.assert_array_equal(a["grf"], b["grf"])
                assert a["best_cost"] == b["best_cost"] and a["q"] == b["q"]
    for c, (mu, mf, tk) in zip(ids, state0):
        rt.set_state(c, mu, mf, tk)
    best = rt.plan_autotune(plan, inps, reps=2)
    assert best["lanes"] in (1, 4) and best["tick_us"] > 0
    after = [rt.get_state(c) for c in ids]
    for (mu0, mf0, t0), (mu1, mf1, t1) in zip(state0, after):
        np.testing.assert_array_equal(mu0, mu1)
        assert mf0 == mf1 and t0 == t1
    res = [rt.fetch(t) for t in rt.plan_submit(plan, inps)]
    assert all(np.isfinite(r["grf"]).all() for r in res)
    rt.plan_destroy(plan)
    for c in ids:
        rt.destroy_controller(c)


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_noise_prefetch_is_transparent(name):
    """Producing the next tick's noise ahead of time on the second stream
    changes no result, including after a state import."""
    from paper_2403_11383_amd import binding
    cfg = workloads.config(name, N=3000, H=20, seed=41)
    inp = workloads.tick_input(workloads.initial_state(np.random.default_rng(41)))
    rt = binding.Runtime(arena_bytes=1 << 30, two_streams=True)
    a = rt.init_controller(cfg)
    b = rt.init_controller(cfg)
    rt.set_prefetch(b, True)
    for t in range(4):
        x, y = rt.tick(a, inp), rt.tick(b, inp)
        np.testing.assert_array_equal(x["grf"], y["grf"])
        assert x["best_cost"] == y["best_cost"] and x["q"] == y["q"] and x["tick"] == y["tick"]
    mu, mf, tk = rt.get_state(a)
    rt.set_state(b, mu, mf, tk + 7)  # the prefetched tick no longer matches
    rt.set_state(a, mu, mf, tk + 7)
    for t in range(2):
        x, y = rt.tick(a, inp), rt.tick(b, inp)
        np.testing.assert_array_equal(x["grf"], y["grf"])
        assert x["best_cost"] == y["best_cost"]
    rt.close()


def test_timing_overhead_probe(rt):
    """sbs_timing_overhead: the interval that an empty dispatch's own events
    span is positive and a few microseconds at most."""
    v = rt.timing_overhead_ns(16)
    print("event overhead ns", v, flush=True)
    assert 0.0 < v < 50_000.0
