"""The C-ABI library loads on the CPU host and exports every entry point that
include/sbs.h declares; the ctypes mirrors have the C layouts.  No compute
call is made here (no GPU)."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sbs.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sbs_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def built():
    from paper_2403_11383_amd import binding, build
    if not os.path.exists(binding.LIB_PATH):
        build.build()
    return binding


def test_every_declared_symbol_is_exported(built):
    L = C.CDLL(built.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 18
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(built.EXPORTED)
    # the boundary's three method calls and the checkpoint / debug taps
    for n in ("sbs_init_controller", "sbs_submit_tick", "sbs_fetch_action", "sbs_export_state",
              "sbs_import_state", "sbs_debug_costs", "sbs_debug_noise", "sbs_last_error"):
        assert n in names, n


def test_method_calls_cite_their_passage():
    """The declarations of the three calls the method needs cite the passage
    that defines them."""
    text = open(HEADER).read()
    for fn, cite in (("sbs_init_controller", "Sec. III-A"), ("sbs_submit_tick", "Alg. 5"),
                     ("sbs_fetch_action", "Fig. 2")):
        decl = text.index(f"int {fn}(")
        comment = text[text.rindex("/*", 0, decl):decl]
        assert cite in comment, (fn, cite)


def test_abi_version_and_error_string(built):
    L = built.lib()
    assert L.sbs_abi_version() == 4
    assert isinstance(L.sbs_last_error(), bytes)


def test_null_arguments_are_rejected_without_a_device(built):
    L = built.lib()
    h = C.c_void_p()
    assert L.sbs_runtime_create(None, 0, None, None, 0, C.byref(h)) == built.EINVAL
    assert b"arena" in L.sbs_last_error()
    assert L.sbs_runtime_destroy(None) == built.EINVAL
    assert L.sbs_fetch_action(None, 1, None, 0) == built.EINVAL
    assert L.sbs_closed_loop_step(None, 0, None, None, None, None, 0.35, 0.0, None) == built.EINVAL
    assert L.sbs_timing_overhead(None, 1, None) == built.EINVAL


def test_struct_layouts_match_c(built):
    src = r'''
#include <stdio.h>
#include <stddef.h>
#include "sbs.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu\n", sizeof(sbs_controller_cfg), sizeof(sbs_tick_input),
         sizeof(sbs_action), offsetof(sbs_controller_cfg, seed),
         offsetof(sbs_tick_input, phase_robot), offsetof(sbs_action, t_done_ns));
  return 0;
}
'''
    d = tempfile.mkdtemp()
    cpath, exe = os.path.join(d, "probe.c"), os.path.join(d, "probe")
    open(cpath, "w").write(src)
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), cpath, "-o", exe], check=True)
    vals = [int(v) for v in subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()]
    b = built
    assert vals == [C.sizeof(b.ControllerCfg), C.sizeof(b.TickInput), C.sizeof(b.Action),
                    b.ControllerCfg.seed.offset, b.TickInput.phase_robot.offset,
                    b.Action.t_done_ns.offset]
