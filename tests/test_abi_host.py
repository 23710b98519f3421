"""Host-only checks of the C ABI: the library loads without a GPU, exports
every function include/vr.h declares, and its argument rules agree with
the oracle's on a table of valid and invalid calls (no device work)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle import vro
from paper_1805_08893_amd import vr
from paper_1805_08893_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "vr.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(vr_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    names = _declared_functions()
    assert set(names) == set(vr.EXPORTS), names
    L = C.CDLL(vr.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n


def test_oracle_is_separate_library():
    assert os.path.realpath(vro.LIB_PATH) != os.path.realpath(vr.LIB_PATH)
    L = C.CDLL(vro.LIB_PATH)
    assert not hasattr(L, "vr_process_draw")


def _cases():
    sp = W.make_shader(W.SHADER_PHONG, 1, num_lights=4)
    yield "ok_static", dict(n=300, strategy=vr.VR_STATIC_SORT, bt=64)
    yield "ok_dyn", dict(n=300, strategy=vr.VR_DYN_HASH, bt=341, nu=256)
    yield "ok_dyn_default", dict(n=300, strategy=vr.VR_DYN_PHASH, bt=100)
    yield "ok_empty", dict(n=0, strategy=vr.VR_DYN_SORT, bt=64)
    yield "not_triangles", dict(n=301, strategy=vr.VR_NAIVE, bt=1)
    yield "too_many", dict(n=3 * (1 << 30), strategy=vr.VR_NAIVE, bt=1)
    yield "bad_strategy", dict(n=300, strategy=9, bt=1)
    yield "ok_multi", dict(n=300, strategy=vr.VR_MULTI, bt=1)
    yield "multi_verts_cap", dict(n=300, strategy=vr.VR_MULTI, bt=1, verts_cap=99)        # V = 100
    yield "multi_verts_cap_ok", dict(n=300, strategy=vr.VR_MULTI, bt=1, verts_cap=100)    # below 3T
    yield "multi_units_cap_ok", dict(n=300, strategy=vr.VR_MULTI, bt=1, units_cap=1)
    yield "multi_local_idx", dict(n=300, strategy=vr.VR_MULTI, bt=1, local=True)
    yield "batch0", dict(n=300, strategy=vr.VR_STATIC_HASH, bt=0)
    yield "static_cap", dict(n=300, strategy=vr.VR_STATIC_HASH, bt=257)
    yield "ballot_cap_ok", dict(n=300, strategy=vr.VR_STATIC_BALLOT, bt=1024)
    yield "ballot_cap", dict(n=300, strategy=vr.VR_STATIC_BALLOT, bt=1025)
    yield "dyn_cap", dict(n=300, strategy=vr.VR_DYN_BALLOT, bt=4097)
    yield "dyn_cap_ok", dict(n=300, strategy=vr.VR_DYN_HASH, bt=4096, nu=4096)
    yield "nu2", dict(n=300, strategy=vr.VR_DYN_SORT, bt=64, nu=2)
    yield "nu4097", dict(n=300, strategy=vr.VR_DYN_SORT, bt=64, nu=4097)
    yield "slots_big", dict(n=300, strategy=vr.VR_DYN_HASH, bt=64, nu=64, slots=16384)
    yield "slots_big_ok", dict(n=300, strategy=vr.VR_DYN_HASH, bt=64, nu=64, slots=8192)
    yield "nu_ignored_static", dict(n=300, strategy=vr.VR_STATIC_SORT, bt=64, nu=2)
    yield "wg_bad", dict(n=300, strategy=vr.VR_DYN_SORT, bt=64, wg=100)
    yield "wg_ok", dict(n=300, strategy=vr.VR_DYN_SORT, bt=64, wg=192)
    yield "slots_not_pow2", dict(n=300, strategy=vr.VR_DYN_HASH, bt=64, slots=96)
    yield "slots_small", dict(n=300, strategy=vr.VR_DYN_HASH, bt=64, nu=64, slots=32)
    yield "slots_ok", dict(n=300, strategy=vr.VR_DYN_HASH, bt=64, nu=64, slots=64)
    yield "probes", dict(n=300, strategy=vr.VR_DYN_PHASH, bt=64, probes=65)
    yield "lights", dict(n=300, strategy=vr.VR_NAIVE, bt=1, lights=17)
    yield "verts_cap", dict(n=300, strategy=vr.VR_NAIVE, bt=1, verts_cap=299)
    yield "verts_cap_ok", dict(n=300, strategy=vr.VR_NAIVE, bt=1, verts_cap=300)
    yield "units_cap_static", dict(n=300, strategy=vr.VR_STATIC_SORT, bt=64, units_cap=1)
    yield "units_cap_static_ok", dict(n=300, strategy=vr.VR_STATIC_SORT, bt=64, units_cap=2)
    yield "units_cap_dyn", dict(n=300, strategy=vr.VR_DYN_SORT, bt=64, units_cap=99)


@pytest.mark.parametrize("name,case", list(_cases()))
def test_argument_rules_match_oracle(name, case):
    sp = W.make_shader(W.SHADER_PHONG, 1, num_lights=4)
    sp.num_lights = case.get("lights", 4)
    o_opts = vro.make_opts(case.get("nu", 0), case.get("wg", 0), case.get("slots", 0), case.get("probes", 0))
    g_opts = vr.make_opts(case.get("nu", 0), case.get("wg", 0), case.get("slots", 0), case.get("probes", 0))
    dummy = 0x1000
    vcap = case.get("verts_cap")
    ucap = case.get("units_cap")
    loc = dummy if case.get("local") else None
    o_out = vro.Outputs(None, None, dummy if vcap is not None else None, vcap or 0, loc,
                        dummy if ucap is not None else None, None, ucap or 0, None)
    g_out = vr.vr_outputs(None, None, dummy if vcap is not None else None, vcap or 0, loc,
                          dummy if ucap is not None else None, None, ucap or 0, None)
    o_sh = vro.make_shader(sp)
    st_o = vro.lib().vro_check_args(case["n"], 100, C.byref(o_sh), case["strategy"], case["bt"], C.byref(o_opts),
                                    C.byref(o_out), None)
    st_g = vr.vr_check_args(case["n"], 100, sp, case["strategy"], case["bt"], g_opts, g_out)
    assert st_o == st_g, (name, st_o, st_g)
    expect_ok = name.startswith("ok") or name.endswith("_ok") or name == "nu_ignored_static"
    assert (st_g == vr.VR_OK) == expect_ok, (name, st_g)


def test_null_context_is_an_argument_error():
    assert vr.lib().vr_sync(None, None) == vr.VR_ERR_ARG
    assert vr.lib().vr_set_stream(None, None) == vr.VR_ERR_ARG
    assert vr.lib().vr_math_selftest(None, 0, 0, 1, None, None) == vr.VR_ERR_ARG


def test_binding_limits_match_header():
    text = open(os.path.join(ROOT, "include", "vr.h")).read()
    defs = dict(re.findall(r"#define (VR_MAX_[A-Z_]+)\s+(\d+)", text))
    for name in ("VR_MAX_BATCH_STATIC", "VR_MAX_BATCH_BALLOT", "VR_MAX_BATCH_DYNAMIC", "VR_MAX_UNIQUE",
                 "VR_MAX_HASH_SLOTS"):
        assert getattr(vr, name) == int(defs[name]), name
