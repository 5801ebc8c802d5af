"""Pins of the GRF spline parametrisation (Sec. IV-B) in the oracle.

The spline is pinned to scipy's cubic Hermite interpolant with numpy's
finite-difference slopes (an independent implementation of the same
definition), to its interpolation of the knots, and to exactness on linear
data; the tick is pinned by composing the pinned parts: rollouts of spline
samples equal rollouts of the per-step forces the spline gives, the MPPI and
elite updates act on the knots, and the warm start re-samples the spline one
step later.
"""
import numpy as np
import pytest
from scipy.interpolate import CubicHermiteSpline

from paper_2403_11383_amd import workloads


def scfg(P=5, H=12, **over):
    return workloads.config("c1", N=16, H=H, knots=P, **over)


def knot_times(cfg):
    P, H, dt = cfg["knots"], cfg["H"], cfg["dt"]
    return np.linspace(0.0, (H - 1) * dt, P)


@pytest.mark.parametrize("P,H", [(2, 2), (2, 9), (3, 7), (5, 12), (8, 50), (12, 12)])
def test_spline_matches_scipy_hermite(orc, P, H):
    cfg = scfg(P, H)
    rng = np.random.default_rng(P * 100 + H)
    th = rng.normal(size=(P, 12)) * 30.0
    t = knot_times(cfg)
    np.testing.assert_allclose([orc.knot_time(cfg, p) for p in range(P)], t, rtol=1e-15, atol=1e-15)
    ref = CubicHermiteSpline(t, th, np.gradient(th, t, axis=0, edge_order=1), axis=0)
    for j in range(H):
        tj = j * cfg["dt"]
        np.testing.assert_allclose(orc.spline_eval(cfg, th, tj), ref(tj), rtol=1e-12, atol=1e-10)


def test_spline_interpolates_knots_and_clamps(orc):
    cfg = scfg(6, 20)
    th = np.random.default_rng(1).normal(size=(6, 12))
    t = knot_times(cfg)
    for p in range(6):
        np.testing.assert_allclose(orc.spline_eval(cfg, th, t[p]), th[p], rtol=1e-14, atol=1e-14)
    np.testing.assert_array_equal(orc.spline_eval(cfg, th, -1.0), orc.spline_eval(cfg, th, 0.0))
    np.testing.assert_array_equal(orc.spline_eval(cfg, th, 1e3), orc.spline_eval(cfg, th, t[-1]))


def test_spline_exact_on_linear_data(orc):
    cfg = scfg(7, 31)
    t = knot_times(cfg)
    a, b = np.arange(12.0), np.linspace(-5, 5, 12)
    th = a[None] + t[:, None] * b[None]
    for j in range(31):
        tj = j * cfg["dt"]
        np.testing.assert_allclose(orc.spline_eval(cfg, th, tj), a + tj * b, rtol=1e-12, atol=1e-12)


def test_rollout_of_knots_is_rollout_of_spline_forces(orc):
    cfg = scfg(5, 15)
    per_step = dict(cfg, knots=0)
    rng = np.random.default_rng(3)
    th = np.tile([0.0, 0.0, 0.5 * cfg["mass"] * cfg["gravity"]] * 4, (5, 1)) + rng.normal(size=(5, 12)) * 15
    u = np.array([orc.spline_eval(cfg, th, j * cfg["dt"]) for j in range(15)])
    inp = workloads.tick_input(workloads.initial_state(rng), phase_robot=12345)
    q = orc.q_of_freq(1.7, cfg["dt"])
    assert orc.rollout(cfg, inp, th, q) == orc.rollout(per_step, inp, u, q)


def hover(cfg, rows):
    return np.tile([0.0, 0.0, 0.5 * cfg["mass"] * cfg["gravity"]] * 4, (rows, 1))


def test_spline_tick_mppi_limit_and_warm_start(orc):
    """lambda -> infinity: the new knots are the sample mean of the knot
    samples; the warm start re-samples that spline one step later, hover at
    the last knot.  (The weights differ from uniform by about (J - beta) /
    lambda, costs here span ~1e4: lambda = 1e16 keeps that below 1e-11.)"""
    cfg = scfg(4, 10, **{"lambda": 1e16})
    mu = hover(cfg, 4) + np.random.default_rng(4).normal(size=(4, 12)) * 10
    inp = workloads.tick_input(workloads.initial_state(np.random.default_rng(5)))
    out = orc.tick(cfg, mu, 1.4, 3, inp)
    z = np.array([[orc.noise_step(cfg["seed"], 3, 0, k, p) for p in range(4)]
                  for k in range(cfg["N"])], np.float64)
    th = mu[None] + cfg["sigma_grf"] * z
    np.testing.assert_allclose(out["mean"], th.mean(0), rtol=1e-9, atol=1e-9)
    assert out["mean"].shape == (4, 12)
    t = knot_times(cfg)
    ref = CubicHermiteSpline(t, out["mean"], np.gradient(out["mean"], t, axis=0), axis=0)
    np.testing.assert_allclose(out["mu_next"][:3], ref(t[:3] + cfg["dt"]), rtol=1e-11, atol=1e-9)
    np.testing.assert_array_equal(out["mu_next"][3], hover(cfg, 1)[0])
    # the action is the first knot (the spline's value at t = 0), clipped and masked
    d, _ = orc.contact(cfg, inp["phase_robot"], out["q"], 0)
    for i in range(4):
        ref_f = orc.friction_clip(out["mean"][0, 3 * i:3 * i + 3], cfg["mu_fric"]) * d[i]
        np.testing.assert_array_equal(out["grf"][3 * i:3 * i + 3], ref_f)


def test_spline_tick_costs_are_rollouts_of_knot_samples(orc):
    cfg = scfg(3, 8)
    mu = hover(cfg, 3)
    rng = np.random.default_rng(6)
    inp = workloads.tick_input(workloads.initial_state(rng), phase_robot=777)
    out = orc.tick(cfg, mu, 1.4, 9, inp)
    for k in (0, 5, 15):
        z = np.array([orc.noise_step(cfg["seed"], 9, 0, k, p) for p in range(3)], np.float64)
        q = orc.freq_q(cfg, 1.4, 0.0, 9, 0, k)
        assert out["q_samples"][0, k] == q
        assert out["costs"][0, k] == orc.rollout(cfg, inp, mu + cfg["sigma_grf"] * z, q)


def test_spline_elite_moments_on_knots(orc):
    cfg = workloads.config("c2", N=20, H=9, knots=4, elite_frac=0.25, iterations=1)
    mu = hover(cfg, 4)
    inp = workloads.tick_input(workloads.initial_state(np.random.default_rng(7)))
    out = orc.tick(cfg, mu, 1.4, 2, inp)
    z = np.array([[orc.noise_step(cfg["seed"], 2, 0, k, p) for p in range(4)]
                  for k in range(20)], np.float64)
    th = mu[None] + cfg["sigma_grf"] * z
    e = np.lexsort((np.arange(20), out["costs"][0]))[:5]
    np.testing.assert_allclose(out["mean"], th[e].mean(0), rtol=1e-12, atol=1e-10)


@pytest.mark.parametrize("P", [1, 13, -2])
def test_spline_rejects_bad_knot_counts(orc, P):
    cfg = workloads.config("c1", N=4, H=12, knots=P)
    with pytest.raises(ValueError):
        orc.tick(cfg, np.zeros((orc.rows(cfg), 12)), 1.4, 0, workloads.tick_input(workloads.initial_state(np.random.default_rng(0))))
