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
def compiled():
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
    return {"kernels": kernels, "text": text}


@pytest.fixture(scope="module")
def metadata(compiled):
    return compiled["kernels"]


def kernel_body(text, name_part):
    """Assembly lines of the first kernel whose symbol contains name_part (up
    to the function's end label: a kernel may end its waves in several
    places)."""
    lines = text.split("\n")
    for i, line in enumerate(lines):
        if re.match(r"^_Z\S*:", line) and name_part in line.split(":")[0]:
            body = []
            for l in lines[i:]:
                if l.startswith(".Lfunc_end"):
                    return body
                body.append(l)
    raise AssertionError(f"no kernel matching {name_part}")


def largest_loop(body):
    """Instructions of the kernel's largest loop (header label to its last
    back-edge)."""
    best = []
    for i, line in enumerate(body):
        m = re.match(r"^(\.LBB\d+_\d+):.*Loop Header", line)
        if not m:
            continue
        ends = [k for k in range(i + 1, len(body))
                if re.search(r"s_(cbranch_\w+|branch)\s+" + re.escape(m.group(1)) + r"$", body[k])]
        if ends and ends[-1] - i > len(best):
            best = body[i:ends[-1] + 1]
    return [l.split()[0] for l in best if re.match(r"^\s+[a-z]", l)]


def test_every_stage_is_built(metadata):
    names = " ".join(metadata)
    for k in ("k_noise", "k_rollout", "k_rollout_quad", "k_select", "k_update", "k_update_mppi"):
        assert k in names, k
    # both one-lane forms: four legs masked by contact, and the stance pair
    assert "k_rolloutIfLi256ELi1ELb0ELb0ELb0ELi0EE" in names
    assert "k_rolloutIfLi256ELi1ELb0ELb0ELb1ELi0EE" in names
    # and the stance-pair one-lane forms that make their own noise: every
    # row, and the stance legs' Gaussians only
    assert "k_rolloutIfLi256ELi1ELb0ELb0ELb1ELi1EE" in names
    assert "k_rolloutIfLi256ELi1ELb0ELb0ELb1ELi2EE" in names


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


def test_noise_row_loop(compiled):
    """The batched noise kernel's per-row loop: no divergent branch, no
    memory load (the descriptor fields stay in registers), and each Philox
    round's two three-word XORs as single three-input bit operations."""
    ins = largest_loop(kernel_body(compiled["text"], "k_noiseILb0E"))
    assert ins, "row loop not found"
    assert not [i for i in ins if i.startswith("s_cbranch_exec")], "divergent branch in the row loop"
    assert not [i for i in ins if i.startswith(("global_load", "s_load", "buffer_load"))]
    assert sum(i == "v_bitop3_b32" for i in ins) >= 50  # 3 calls x 10 rounds x 2, a few folded


@pytest.mark.parametrize("kernel,budget", [("k_rolloutIfLi256ELi1ELb0ELb0ELb0ELi0EE", 535),
                                           ("k_rolloutIfLi256ELi1ELb0ELb0ELb1ELi0EE", 410),
                                           ("k_rolloutIfLi256ELi1ELb0ELb0ELb1ELi1EE", 905),
                                           ("k_rolloutIfLi256ELi1ELb0ELb0ELb1ELi2EE", 670),
                                           ("k_rollout_quadILi256ELi1ELb1ELb0E", 250)])
def test_rollout_step_instruction_budget(compiled, kernel, budget):
    """Instructions in the step loop (scalar and memory ones included, both
    paths of the attitude sine and cosine counted: the reduced one taken
    when any lane of the wave has a large angle, and the polynomial alone):
    526 for the one-lane four-leg form, 403 for the one-lane stance-pair
    form, 895 for the stance-pair form that also makes the step's noise
    (three Philox calls, six Box-Muller pairs), 657 for the stance-pair form
    that makes only its stance diagonal's Gaussians (two Philox calls, three
    pairs) and 245 for the quad form when this was written; the budget catches a change that adds branches
    or moves to the step."""
    ins = largest_loop(kernel_body(compiled["text"], kernel))
    assert ins and len(ins) <= budget, (kernel, len(ins))
