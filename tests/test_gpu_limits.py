"""Parity at the configuration limits the runtime accepts: the largest sample
count (N = 2^22), sample counts above 16384 where each select thread owns more
than the 16 costs it keeps in registers, and the longest horizon (H = 256).

Small cases compare every output with the FP64 oracle; at N = 2^22 the costs
of a strided subset (and the last sample) are re-rolled by the oracle one by
one, every phase increment is checked, and the update is checked by selection
parity (the oracle's update fed the GPU's own costs)."""
import numpy as np
import pytest

import oracle
from paper_2403_11383_amd import workloads
from parity_util import MG2, check_fp64, cost_tol, hover, run_pair

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _oracle_built():
    oracle.build()


@pytest.fixture(scope="module")
def rt():
    from paper_2403_11383_amd import binding
    r = binding.Runtime(arena_bytes=3 << 30)
    yield r
    r.close()


@pytest.mark.parametrize("method", ["mppi", "elite"])
def test_max_samples(rt, method):
    N, H = 1 << 22, 2
    cfg = workloads.config("c1", N=N, H=H, method=method, iterations=1, seed=22)
    inp = workloads.tick_input(workloads.initial_state(np.random.default_rng(5)))
    print("N", N, "H", H, method, flush=True)
    cid = rt.init_controller(cfg)
    rt.set_debug(cid, True)
    act = rt.tick(cid, inp)
    J, q, mean = rt.debug_fetch(cid)
    rt.destroy_controller(cid)
    ks = np.unique(np.concatenate([np.arange(0, N, 65537), [N - 1, int(np.argmin(J[0]))]]))
    for k in ks:
        assert q[0][k] == oracle.freq_q(cfg, cfg["mu_f0"], 0.0, 0, 0, int(k))
    mu = hover(cfg)
    for k in ks:
        z = np.array([oracle.noise_step(cfg["seed"], 0, 0, int(k), j) for j in range(H)])
        jr = oracle.rollout(cfg, inp, mu + cfg["sigma_grf"] * z, int(q[0][k]))
        assert abs(J[0][k] - jr) <= cost_tol(jr), (k, J[0][k], jr)
    ref = oracle.tick(cfg, mu, cfg["mu_f0"], 0, inp, costs_override=J, nthreads=8)
    np.testing.assert_array_equal(q, ref["q_samples"])
    scale = max(np.abs(ref["mean"]).max(), MG2)
    assert np.abs(mean - ref["mean"]).max() <= 1e-4 * scale
    assert np.abs(act["grf"] - ref["grf"]).max() <= 1e-4 * scale
    assert act["q"] == ref["q"]


@pytest.mark.parametrize("N", [16385, 20000, 70001])
def test_elite_select_beyond_register_slice(rt, N):
    """Above 16384 samples each select thread owns ceil(N / 1024) costs and
    reads all but the first 16 from memory on every pass: FP64, so the elite
    set, the mean and the action must match the oracle's exactly (to FP64
    rounding), also for a ragged N."""
    cfg = workloads.config("c0", N=N, H=4, method="elite", iterations=2, elite_frac=0.1, seed=N)
    inp = workloads.c0_input()
    print("N", N, flush=True)
    out, ref = run_pair(rt, cfg, inp)
    check_fp64(out, ref, cfg)


def test_max_horizon(rt):
    """H = 256 steps (5.12 s at dt = 0.02), FP64 MPPI: costs compared on the
    samples that can carry weight (most of so long a horizon tumbles)."""
    cfg = workloads.config("c0", N=200, H=256, seed=256)
    inp = workloads.c0_input()
    print("H", cfg["H"], flush=True)
    out, ref = run_pair(rt, cfg, inp)
    check_fp64(out, ref, cfg, influential_only=True)
