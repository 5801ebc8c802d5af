"""Closed-loop disturbance study on the GPU path (the shape of the paper's
gait-adaptation test, Sec. V-C, Fig. 4): the best-sample controller with the
frequency set keeps the host SRBD plant upright through a 40 N lateral push
for 3 s and raises the step frequency while the push acts."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rt():
    from paper_2403_11383_amd import binding
    r = binding.Runtime(arena_bytes=1 << 30)
    yield r
    r.close()


def test_push_survived_with_gait_adaptation(rt):
    from paper_2403_11383_amd import binding, workloads
    import bench
    cfg = workloads.study_config("naive", adapt=True, rho=300.0)
    fell, freq, lat = bench.study_episode(rt, binding, workloads, cfg, seed=1)
    print("fell", fell, "ticks", len(freq), flush=True)
    assert fell is None
    f = np.asarray(freq)
    p0, p1, _ = workloads.STUDY_PUSH
    before, during, after = f[:p0].mean(), f[p0:p1].mean(), f[p1 + 10:].mean()
    print("frequency before/during/after", before, during, after, flush=True)
    assert set(np.round(f, 6)) <= set(np.round(workloads.STUDY_FSET, 6))
    assert during > before + 0.3 and during > after
    assert np.all(np.asarray(lat) > 0)
