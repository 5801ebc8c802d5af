"""Tick-by-tick parity inside a closed loop: an FP64 controller drives the
host plant for 40 ticks (noise produced ahead on the second stream, a 40 N
lateral push from tick 10), and before every tick the oracle is handed the
state the GPU controller holds (its warm-started mean, frequency mean and
tick counter) and the plant's state, footholds and gait phase.  Its action
must match the GPU's to FP64 rounding: this pins the warm-start shift, the
tick counter of the noise, the phase hand-off to the plant and the footholds
across many consecutive ticks, not just one."""
import numpy as np
import pytest

import oracle
from paper_2403_11383_amd import workloads
from parity_util import MG2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _oracle_built():
    oracle.build()


@pytest.mark.parametrize("method", ["mppi", "naive"])
def test_fp64_closed_loop_tick_by_tick(method):
    from paper_2403_11383_amd import binding
    # the disturbance study's weights keep the robot upright, so every tick's
    # costs stay well-conditioned
    cfg = workloads.config("c0", N=256, H=12, method=method, freq_mode="uniform",
                           friction_on=True, mu_fric=0.5, sigma_grf=10.0, seed=41,
                           **{"lambda": 30.0})
    cfg["Q"] = list(workloads.STUDY_Q)
    rt = binding.Runtime(arena_bytes=256 << 20, two_streams=True)
    cid = rt.init_controller(cfg)
    rt.set_prefetch(cid, True)
    x0 = workloads.initial_state(np.random.default_rng(41))
    plant = binding.Plant(cfg, x0, workloads.feet_under_hips(x0), phase=0)
    v_ref = (0.3, 0.0, 0.0)
    loop = binding.ClosedLoop(rt, cid, plant, v_ref=v_ref, z_ref=workloads.HEIGHT)
    for t in range(40):
        mu, mf, tick = rt.get_state(cid)
        x = plant.x
        inp = workloads.tick_input(x, v_ref=v_ref, p_ref0=(x[0], x[1], workloads.HEIGHT),
                                   phase_robot=plant.phase, foot_pos=plant.foot_pos)
        ref = oracle.tick(cfg, mu, mf, tick, inp, nthreads=4)
        a = loop.step((0.0, 40.0 if t >= 10 else 0.0, 0.0))
        scale = max(np.abs(ref["grf"]).max(), MG2)
        grf = np.array(a.grf[:])
        print("tick", t, "max |grf - oracle|", np.abs(grf - ref["grf"]).max(), flush=True)
        assert np.abs(grf - ref["grf"]).max() <= 1e-9 * scale, t
        assert a.q == ref["q"] and list(a.contact[:]) == [int(c) for c in ref["contact"]], t
        assert tick == t
    rt.close()
