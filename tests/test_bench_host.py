"""Host-side pieces of bench.py (no GPU): the one-GPU guard, the roofline
object's arithmetic, the FLOP accounting and the stored HBM-traffic lookup."""
import gc
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_rollout_flop_table_sums_to_the_constant():
    # policy, friction cone, attitude, footholds, stage cost, force and torque,
    # R^T tau, gyroscopic term, Euler-angle rates, accelerations, Euler update
    parts = [24, 36, 24, 3, 94, 72, 15, 12, 11, 10, 25]
    assert sum(parts) == bench.FLOP_PER_ROLLOUT_STEP == 326
    # one Box-Muller pair: logarithm 24, fold 1, radius 2, sine and cosine 21,
    # the two products 2
    assert bench.FLOP_PER_GAUSS_PAIR == 24 + 1 + 2 + 21 + 2
    assert bench.FLOP_PER_NOISE_ROW == 6 * bench.FLOP_PER_GAUSS_PAIR
    assert bench.FORM_FLOP_PER_STEP == [326, 326, 326, 326 + 300, 326 + 150]
    assert len(bench.FORM_NAMES) == len(bench.FORM_TRAFFIC_KEY) == bench.N_FORMS


def test_roofline_object_arithmetic():
    # 1e9 FLOP over 2 launches of 100 us average duration: 5 TFLOP/s
    r = bench.roofline_obj("k", 1e9, 100e3, 2, flop_per_rollout_step=476, traffic=None)
    assert r["achieved"] == pytest.approx(5.0)
    assert r["frac"] == pytest.approx(r["achieved"] / 157.3)
    assert r["frac_nonpacked"] == pytest.approx(r["achieved"] / 78.6)
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s" and r["peak"] == 157.3
    assert r["flop_per_rollout_step"] == 476
    assert bench.roofline_obj("k", 1e9, 0.0, 0)["achieved"] == 0.0


def test_stored_traffic_follows_the_kernel_source(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    h = bench.kernel_source_hash()
    doc = {"k/per_launch": {"bytes_per_launch": 123.0, "kernel_source_hash": h},
           "k/per_step": {"bytes_per_rollout_step": 0.5, "kernel_source_hash": h},
           "k/stale": {"bytes_per_launch": 1.0, "kernel_source_hash": "0" * 16}}
    (prof / "traffic.json").write_text(json.dumps(doc))
    real_join = os.path.join

    def join(a, *rest):
        if a == bench.ROOT and rest and rest[0] == "profiles":
            return real_join(str(tmp_path), *rest)
        return real_join(a, *rest)

    monkeypatch.setattr(bench.os.path, "join", join)
    assert bench.stored_traffic("k", "per_launch") == 123.0
    assert bench.stored_traffic("k", "per_step", 1000.0) == 500.0
    assert bench.stored_traffic("k", "per_step") is None   # no launch size to scale by
    assert bench.stored_traffic("k", "stale") is None      # counters of other source
    assert bench.stored_traffic("k", "absent") is None


def test_committed_traffic_entries_name_their_source():
    doc = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    for key, ent in doc.items():
        assert len(ent["kernel_source_hash"]) == 16, key
        assert ("bytes_per_launch" in ent) != ("bytes_per_rollout_step" in ent), key
        assert ent["fetch_cal_kib_per_kib"] == pytest.approx(2.0, rel=1e-3)
        assert ent["write_cal_kib_per_kib"] == pytest.approx(1.0, rel=1e-3)


def test_gc_paused_restores_the_collector():
    assert gc.isenabled()
    with bench.gc_paused():
        assert not gc.isenabled()
    assert gc.isenabled()
    with pytest.raises(RuntimeError):
        with bench.gc_paused():
            raise RuntimeError("inside")
    assert gc.isenabled()
