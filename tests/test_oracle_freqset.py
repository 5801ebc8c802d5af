"""Pins of the discrete gait-frequency set (Sec. V: the stepping frequency
takes one of a few values, e.g. the nominal one, 2.0 and 2.4 Hz, drawn
uniformly) in the oracle: draws are set members, each with probability 1/n,
independent across samples, iterations and ticks; with one member the draw
is that member; the best-sample update returns the best sample's member."""
import numpy as np
import pytest
from scipy import stats

from paper_2403_11383_amd import workloads

FSET = (1.4, 2.0, 2.4)


def cfg_set(**over):
    base = dict(N=64, H=8, freq_mode="set", f_set=FSET, method="naive", iterations=2, rho=1.0)
    base.update(over)
    return workloads.config("c2", **base)


def test_draws_are_members_and_uniform(orc):
    cfg = cfg_set()
    qs = {orc.q_of_freq(f, cfg["dt"]): i for i, f in enumerate(FSET)}
    counts = np.zeros(3)
    for k in range(6000):
        q = orc.freq_q(cfg, 1.4, 0.4, 17, 0, k)
        assert q in qs
        counts[qs[q]] += 1
    assert stats.chisquare(counts).pvalue > 1e-3


def test_draws_independent_of_iteration_and_tick(orc):
    cfg = cfg_set()
    a = np.array([orc.freq_q(cfg, 1.4, 0.4, 5, 0, k) for k in range(3000)])
    b = np.array([orc.freq_q(cfg, 1.4, 0.4, 5, 1, k) for k in range(3000)])
    c = np.array([orc.freq_q(cfg, 1.4, 0.4, 6, 0, k) for k in range(3000)])
    for x, y in ((a, b), (a, c)):
        table = np.zeros((3, 3))
        vals = sorted(set(a))
        for u, v in zip(x, y):
            table[vals.index(u), vals.index(v)] += 1
        assert stats.chi2_contingency(table).pvalue > 1e-3


def test_single_member_set(orc):
    cfg = cfg_set(f_set=(2.2,))
    q = orc.q_of_freq(2.2, cfg["dt"])
    assert all(orc.freq_q(cfg, 1.4, 0.4, 1, 0, k) == q for k in range(200))


def test_naive_tick_returns_best_members_frequency(orc):
    cfg = cfg_set(phase_offset=list(workloads.PACE_OFFSETS))
    mu = np.tile([0.0, 0.0, 0.5 * cfg["mass"] * cfg["gravity"]] * 4, (cfg["H"], 1))
    inp = workloads.tick_input(workloads.initial_state(np.random.default_rng(3)))
    out = orc.tick(cfg, mu, 1.4, 4, inp)
    b = int(np.argmin(out["costs"][-1]))
    f_best = out["q_samples"][-1, b] / (cfg["dt"] * 2**32)
    assert out["mu_f_next"] == f_best
    # the executed frequency is the member quantised to an integer increment
    assert min(abs(f_best - f) for f in FSET) <= 0.5 / (cfg["dt"] * 2**32)
    assert out["q"] == orc.q_of_freq(f_best, cfg["dt"])


@pytest.mark.parametrize("fs", [(), (1.0, 1.5, 2.0, 2.5, 3.0)])
def test_set_size_validated(orc, fs):
    cfg = cfg_set(f_set=fs)
    mu = np.zeros((cfg["H"], 12))
    with pytest.raises(ValueError):
        orc.tick(cfg, mu, 1.4, 0, workloads.tick_input(workloads.initial_state(np.random.default_rng(0))))
