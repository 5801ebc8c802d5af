"""The gfx950 code object of the kernels: no kernel uses per-lane scratch
memory or spills vector registers (scalar registers may spill into vector
register lanes, which costs no memory traffic).  (A descriptor passed by value in the kernel
arguments is read in place; if a change lets the compiler copy it to scratch,
every lane of every workgroup writes ~1 KB before doing any work.)"""
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def metadata():
    from paper_2403_11383_amd import build
    src = os.path.join(ROOT, "paper_2403_11383_amd", "csrc", "sbs_kernels.hip")
    with tempfile.TemporaryDirectory() as td:
        out = os.path.join(td, "k.s")
        cmd = [os.environ.get("HIPCC", "/opt/rocm/bin/hipcc"), *build.HIP_FLAGS, "-I",
               os.path.join(ROOT, "include"), "-x", "hip", "--cuda-device-only", "-S", src,
               "-o", out]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-2000:]
        text = open(out).read()
    kernels = {}
    for block in text.split("  - .agpr_count")[1:]:
        name = re.search(r"\.name:\s+(\S+)", block).group(1)
        field = lambda f: int(re.search(r"\." + f + r":\s+(\d+)", block).group(1))
        kernels[name] = {f: field(f) for f in ("private_segment_fixed_size", "vgpr_spill_count",
                                               "sgpr_spill_count", "vgpr_count")}
        kernels[name]["args"] = [(int(o), int(z)) for o, z in
                                 re.findall(r"\.offset:\s+(\d+)\n\s+\.size:\s+(\d+)", block)][:2]
    return kernels


def test_every_stage_is_built(metadata):
    names = " ".join(metadata)
    for k in ("k_noise", "k_rollout", "k_rollout_quad", "k_select", "k_update", "k_update_mppi"):
        assert k in names, k


def test_no_scratch_and_no_vector_spills(metadata):
    bad = {n: m for n, m in metadata.items()
           if m["private_segment_fixed_size"] or m["vgpr_spill_count"]}
    assert not bad, bad


def test_inline_descriptor_offset(metadata):
    """Every kernel takes (LaunchTab, TickDesc) and reads the descriptor in
    place at the LaunchTab's size rounded up to 8 bytes."""
    for name, m in metadata.items():
        if "k_empty" in name:  # the argument-free event-overhead probe
            assert not m["args"], (name, m["args"])
            continue
        (o0, z0), (o1, z1) = m["args"]
        assert o0 == 0 and o1 == (z0 + 7) // 8 * 8, (name, m["args"])
