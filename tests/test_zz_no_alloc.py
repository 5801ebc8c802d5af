"""sbs_submit_tick_noalloc (step workspace in the library's static device
scratch array) against sbs_submit_tick (workspace carved from the arena):
the same kernels on the same inputs, so every result is bit-identical.  Two
calls in a row, the second with a smaller controller, then a warm-started
second tick of the first, then a controller too large for the scratch."""
import numpy as np
import pytest

from paper_2403_11383_amd import workloads

pytestmark = pytest.mark.gpu


def _same(a, b):
    np.testing.assert_array_equal(a["grf"], b["grf"])
    assert a["q"] == b["q"] and a["best_cost"] == b["best_cost"] and a["flags"] == b["flags"]
    assert a["tick"] == b["tick"] and a["n_active"] == b["n_active"]
    np.testing.assert_array_equal(a["contact"], b["contact"])


def test_noalloc_tick_equals_arena_tick():
    from paper_2403_11383_amd import binding
    rt = binding.Runtime(arena_bytes=1 << 30)
    cfgs = [workloads.config("c1", N=10240, H=50, seed=71),                    # ~25 MB of noise
            workloads.config("c2", N=3000, H=20, iterations=2, seed=72)]       # smaller, elite
    rng = np.random.default_rng(73)
    inps = [workloads.tick_input(workloads.initial_state(rng)) for _ in cfgs]
    pairs = []
    for cfg in cfgs:
        a, b = rt.init_controller(cfg), rt.init_controller(cfg)
        rt.set_debug(a, True)
        rt.set_debug(b, True)
        pairs.append((a, b))
    for tick in range(2):  # the second round is a warm-started tick
        for (a, b), inp in zip(pairs, inps):
            got = rt.fetch(rt.submit_tick_noalloc(a, inp))
            want = rt.fetch(rt.submit_tick(b, inp))
            print("tick", tick, "controller", a, "grf", got["grf"][:3], flush=True)
            _same(got, want)
            ja, qa, ma = rt.debug_costs(a)
            jb, qb, mb = rt.debug_costs(b)
            np.testing.assert_array_equal(ja, jb)
            np.testing.assert_array_equal(qa, qb)
            np.testing.assert_array_equal(ma, mb)
            np.testing.assert_array_equal(rt.export_state(a)[0], rt.export_state(b)[0])
    # a workspace beyond the 64 MiB scratch is refused (N x H x 48 B of noise)
    big = rt.init_controller(workloads.config("c1", N=32768, H=60, seed=74))
    with pytest.raises(binding.SBSError) as e:
        rt.submit_tick_noalloc(big, inps[0])
    assert e.value.code == binding.EINVAL
    rt.close()


def test_noalloc_needs_direct_mode():
    from paper_2403_11383_amd import binding
    rt = binding.Runtime(arena_bytes=64 << 20, mode="serving", two_streams=True)
    cid = rt.init_controller(workloads.config("c4", N=512, H=10, seed=75))
    inp = workloads.tick_input(workloads.initial_state(np.random.default_rng(75)))
    with pytest.raises(binding.SBSError) as e:
        rt.submit_tick_noalloc(cid, inp)
    assert e.value.code == binding.EINVAL
    rt.close()
