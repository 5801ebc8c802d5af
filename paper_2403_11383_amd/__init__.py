"""MI355X-native sample-based stochastic predictive controller for a quadruped.

The hot path (noise, rollouts, selection, mean/covariance update) is HIP for
gfx950 in ``csrc/`` behind the C ABI declared in ``include/sbs.h``.
``binding`` marshals arguments to that library; ``workloads`` holds the
seeded synthetic inputs.  Importing the package loads nothing.
"""
__all__ = ["binding", "workloads"]
