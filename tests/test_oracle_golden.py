"""Regression pin: the oracle still produces the stored result for the plain
MPPI workload (written by tests/golden/make_c0_golden.py, which calls only
the oracle)."""
import json
import os

import numpy as np

from paper_2403_11383_amd import workloads

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c0_oracle.json")


def test_c0_oracle_matches_stored(orc):
    ref = json.load(open(GOLDEN))
    cfg = workloads.config("c0")
    inp = workloads.c0_input()
    assert inp["x0"] == ref["input"]["x0"]
    mu = np.tile([0.0, 0.0, 0.5 * cfg["mass"] * cfg["gravity"]] * 4, (cfg["H"], 1))
    out = orc.tick(cfg, mu, cfg["mu_f0"], 0, inp, nthreads=4)
    c = out["costs"][0]
    np.testing.assert_allclose(c[:8], ref["costs_first8"], rtol=1e-13)
    assert int(c.argmin()) == ref["cost_argmin"]
    np.testing.assert_allclose(c.sum(), ref["cost_sum"], rtol=1e-13)
    np.testing.assert_allclose(out["grf"], ref["grf"], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(out["mean"][0], ref["mean_step0"], rtol=1e-12, atol=1e-12)
    assert list(out["contact"]) == ref["contact"] and int(out["q"]) == ref["q"]
