"""Writes c0_oracle.json: the FP64 oracle's result for the plain MPPI
workload (N=256, H=25, fixed 1.4 Hz trot, seed 0).  Calls only oracle/.
It guards the oracle against unintended changes; a deliberate change to the
oracle's arithmetic regenerates it in the same commit and names the reason."""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2403_11383_amd import workloads  # noqa: E402


def main():
    oracle.build()
    cfg = workloads.config("c0")
    inp = workloads.c0_input()
    mu = np.tile([0.0, 0.0, 0.5 * cfg["mass"] * cfg["gravity"]] * 4, (cfg["H"], 1))
    out = oracle.tick(cfg, mu, cfg["mu_f0"], 0, inp)
    c = out["costs"][0]
    doc = {
        "workload": "c0", "tick": 0, "input": inp,
        "costs_first8": c[:8].tolist(), "cost_min": float(c.min()), "cost_argmin": int(c.argmin()),
        "cost_sum": float(c.sum()), "grf": out["grf"].tolist(),
        "contact": out["contact"].tolist(), "q": int(out["q"]),
        "mean_step0": out["mean"][0].tolist(), "mean_last": out["mean"][-1].tolist(),
    }
    with open(os.path.join(HERE, "c0_oracle.json"), "w") as f:
        json.dump(doc, f, indent=1)


if __name__ == "__main__":
    main()
