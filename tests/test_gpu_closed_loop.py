"""Closed-loop disturbance study on the GPU path (the shape of the paper's
gait-adaptation test, Sec. V-C, Fig. 4): with the frequency set, the
best-sample controller keeps the host SRBD plant upright through a 40 N
lateral push for 3 s in most seeded episodes and steps faster while the push
acts; at the fixed nominal frequency the robot falls.  The closed loop is
chaotic (a last-bit change in any kernel reshuffles which episodes survive),
so the checks are on counts over several seeded episodes."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

SEEDS = range(1, 7)


@pytest.fixture(scope="module")
def rt():
    from paper_2403_11383_amd import binding
    r = binding.Runtime(arena_bytes=1 << 30)
    yield r
    r.close()


def episodes(rt, adapt):
    from paper_2403_11383_amd import binding, workloads
    import bench
    cfg = workloads.study_config("naive", adapt=adapt, rho=1.0)
    out = []
    for seed in SEEDS:
        fell, freq, lat = bench.study_episode(rt, binding, workloads, cfg, seed=seed)
        print("adapt", adapt, "seed", seed, "fell", fell, flush=True)
        assert np.all(np.asarray(lat) > 0)
        out.append((fell, np.asarray(freq)))
    return out


def test_push_with_and_without_gait_adaptation(rt):
    from paper_2403_11383_amd import workloads
    p0, p1, _ = workloads.STUDY_PUSH
    with_ad = episodes(rt, True)
    without = episodes(rt, False)
    survivors = [f for fell, f in with_ad if fell is None]
    assert len(survivors) >= 2
    assert sum(fell is None for fell, _ in without) <= 1
    for f in survivors:
        assert set(np.round(f, 6)) <= set(np.round(workloads.STUDY_FSET, 6))
    # steps faster while the push acts than before it (mean over survivors)
    before = np.mean([f[:p0].mean() for f in survivors])
    during = np.mean([f[p0:p1].mean() for f in survivors])
    print("frequency before/during", before, during, flush=True)
    assert during > before
    # without adaptation every step runs at the nominal frequency
    for fell, f in without:
        np.testing.assert_allclose(f, workloads.STUDY_FSET[0], rtol=1e-9)
