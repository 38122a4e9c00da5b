"""C-ABI checks that need no GPU: the library loads, exports every function
include/plan.h declares, and rejects invalid arguments before touching the
device."""
import ctypes as C
import os
import re
import subprocess

import pytest

from paper_2603_20525_amd import inputs
from paper_2603_20525_amd import plan as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        src = open(os.path.join(ROOT, "include", h)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names |= set(re.findall(r"\b(plan_[a-z_]+)\s*\(", src))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(P.LIB_PATH):
        from paper_2603_20525_amd import build
        build.build()
    return P.lib()


def test_header_declares_the_binding_surface():
    assert _declared() == sorted(P.EXPORTS + P.SERVER_EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    for name in _declared():
        assert hasattr(lib, name), name
    # nothing of the oracle is linked into the product library
    out = os.popen(f"nm -D --defined-only {P.LIB_PATH}").read()
    assert "oracle_" not in out
    for name in _declared():
        assert re.search(rf"\bT {name}\b", out), name


def test_create_rejects_invalid_arguments_without_a_device(lib):
    v = P._struct(P.Vehicle, inputs.WORKLOAD_VEHICLE)
    c = P._struct(P.Cost, inputs.BASE_COST)
    i = P._struct(P.Integ, inputs.BASE_INTEG)
    h = C.c_void_p()
    assert lib.plan_create(None, C.byref(v), C.byref(c), C.byref(i), 8, 8, 8, 8, None) == P.PLAN_EINVAL
    assert lib.plan_create(C.byref(h), None, C.byref(c), C.byref(i), 8, 8, 8, 8, None) == P.PLAN_EINVAL
    assert "NULL" in P.plan_last_error(None)
    bad = P._struct(P.Vehicle, dict(inputs.WORKLOAD_VEHICLE, M=-1.0))
    assert lib.plan_create(C.byref(h), C.byref(bad), C.byref(c), C.byref(i), 8, 8, 8, 8, None) == P.PLAN_EINVAL
    assert "vehicle" in P.plan_last_error(None)
    nan = P._struct(P.Vehicle, dict(inputs.WORKLOAD_VEHICLE, Jzz=float("nan")))
    assert lib.plan_create(C.byref(h), C.byref(nan), C.byref(c), C.byref(i), 8, 8, 8, 8, None) == P.PLAN_EINVAL
    bi = P._struct(P.Integ, dict(inputs.BASE_INTEG, substeps=0))
    assert lib.plan_create(C.byref(h), C.byref(v), C.byref(c), C.byref(bi), 8, 8, 8, 8, None) == P.PLAN_EINVAL
    bi = P._struct(P.Integ, dict(inputs.BASE_INTEG, dt=0.0))
    assert lib.plan_create(C.byref(h), C.byref(v), C.byref(c), C.byref(bi), 8, 8, 8, 8, None) == P.PLAN_EINVAL
    for sizes in ((0, 8, 8, 8), (8, 0, 8, 8), (8, 8, 1, 8), (8, 8, 8, 1)):
        assert lib.plan_create(C.byref(h), C.byref(v), C.byref(c), C.byref(i), *sizes, None) == P.PLAN_EINVAL
    # terrain grids of 2^26 nodes or more (the byte offsets of their 64-byte
    # cells, one per node, would not fit in 32 bits) are refused before
    # anything touches a device, the limit itself (W*H = 2^26) included
    assert lib.plan_create(C.byref(h), C.byref(v), C.byref(c), C.byref(i), 8, 8, 1 << 14, 1 << 13,
                           None) == P.PLAN_EINVAL
    assert "2^26" in P.plan_last_error(None)
    assert lib.plan_create(C.byref(h), C.byref(v), C.byref(c), C.byref(i), 8, 8, 1 << 13,
                           1 << 13, None) == P.PLAN_EINVAL
    assert "2^26" in P.plan_last_error(None)
    assert not h.value


def test_calls_on_null_context_are_rejected(lib):
    s0 = (C.c_float * 13)()
    assert lib.plan_rollout(None, s0, None, 1, 1, None, None) == P.PLAN_EINVAL
    assert lib.plan_select(None, 0, 0.0, None, None, 1, 1, None, None, None) == P.PLAN_EINVAL
    assert lib.plan_set_terrain(None, None, 2, 2, 0.0, 0.0, 1.0, None) == P.PLAN_EINVAL
    assert lib.plan_set_launch(None, 4, 64) == P.PLAN_EINVAL
    assert lib.plan_set_order(None, P.PLAN_ORDER_ON) == P.PLAN_EINVAL
    o = C.c_int(7)
    assert lib.plan_get_order(None, C.byref(o)) == P.PLAN_EINVAL and o.value == 7
    assert lib.plan_set_stream(None, None) == P.PLAN_EINVAL
    assert lib.plan_set_cost(None, None) == P.PLAN_EINVAL
    assert lib.plan_enable_timing(None, 1) == P.PLAN_EINVAL
    sp = P.sample_spec(P.PLAN_SAMPLE_UNIFORM, 0, 0, (1.0, 0.0))
    assert lib.plan_sample_controls(None, C.byref(sp), 1, 1, None) == P.PLAN_EINVAL
    assert lib.plan_rollout_sampled(None, s0, C.byref(sp), 1, 1, None, None) == P.PLAN_EINVAL
    assert lib.plan_select_sampled(None, C.byref(sp), None, 1, 1, None, None,
                                   None) == P.PLAN_EINVAL
    lib.plan_destroy(None)


def test_server_create_and_submit_reject_invalid_arguments(lib):
    P._bind_server()
    v = P._struct(P.Vehicle, inputs.WORKLOAD_VEHICLE)
    h = C.c_void_p()
    cr = lib.plan_server_create
    assert cr(None, C.byref(v), 4, 8, 8, 8, 8, 1 << 20, 4, None) == P.PLAN_EINVAL
    assert cr(C.byref(h), C.byref(v), 0, 8, 8, 8, 8, 1 << 20, 4, None) == P.PLAN_EINVAL
    assert cr(C.byref(h), C.byref(v), 129, 8, 8, 8, 8, 1 << 20, 4, None) == P.PLAN_EINVAL
    assert cr(C.byref(h), C.byref(v), 4, 8, 8, 8, 8, 0, 4, None) == P.PLAN_EINVAL
    assert cr(C.byref(h), C.byref(v), 4, 8, 8, 8, 8, 1 << 20, 0, None) == P.PLAN_EINVAL
    bad = P._struct(P.Vehicle, dict(inputs.WORKLOAD_VEHICLE, M=0.0))
    assert cr(C.byref(h), C.byref(bad), 4, 8, 8, 8, 8, 1 << 20, 4, None) == P.PLAN_EINVAL
    assert cr(C.byref(h), C.byref(v), 4, 8, 8, 1 << 14, 1 << 13, 1 << 20, 4, None) == P.PLAN_EINVAL
    assert cr(C.byref(h), C.byref(v), 4, 8, 8, 1 << 13, 1 << 13, 1 << 20, 4,
              None) == P.PLAN_EINVAL
    assert not h.value
    rid = C.c_int(0)
    assert lib.plan_server_submit(None, None, C.byref(rid)) == P.PLAN_EINVAL
    assert lib.plan_server_step(None, None, None) == P.PLAN_EINVAL
    assert lib.plan_server_drain(None) == P.PLAN_EINVAL
    n = C.c_int(-1)
    assert lib.plan_server_completions(None, None, 0, C.byref(n)) == P.PLAN_EINVAL
    lib.plan_server_destroy(None)


def test_struct_layouts_match_the_header(tmp_path):
    """The ctypes mirrors have the sizes and offsets the C compiler gives the
    header's structs."""
    prog = tmp_path / "layout.c"
    prog.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "plan.h"\n#include "plan_serve.h"\n'
        "int main(void) {\n"
        '  printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(plan_sample_t),'
        " offsetof(plan_sample_t, seed), offsetof(plan_sample_t, stream),"
        " offsetof(plan_sample_t, scale), offsetof(plan_sample_t, nominal_dev),"
        " sizeof(plan_vehicle_t));\n"
        '  printf("%zu %zu %zu %zu %zu\\n", sizeof(plan_request_t),'
        " offsetof(plan_request_t, controls_dev), offsetof(plan_request_t, plan_dev),"
        " offsetof(plan_request_t, cost_dev), sizeof(plan_result_t));\n"
        "  return 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(prog), "-o",
                    str(exe)], check=True)
    a, b = subprocess.run([str(exe)], check=True, capture_output=True,
                          text=True).stdout.split("\n")[:2]
    a = [int(x) for x in a.split()]
    b = [int(x) for x in b.split()]
    assert a == [C.sizeof(P.Sample), P.Sample.seed.offset, P.Sample.stream.offset,
                 P.Sample.scale.offset, P.Sample.nominal_dev.offset, C.sizeof(P.Vehicle)]
    assert b == [C.sizeof(P.Request), P.Request.controls_dev.offset, P.Request.plan_dev.offset,
                 P.Request.cost_dev.offset, C.sizeof(P.Result)]


def test_package_has_no_oracle_or_cpu_fallback():
    pkg = os.path.join(ROOT, "paper_2603_20525_amd")
    for dp, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dp, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
                assert "liboracle" not in txt, f
