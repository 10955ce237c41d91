"""The C-ABI library loads on the host and exports every entry point include/visfly.h declares (no GPU calls)."""
import ctypes
import os
import re

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "visfly.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:vf_status|const char\*)\s+(vf_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("vf_scene_build", "vf_step", "vf_render", "vf_step_backward", "vf_render_backward",
                     "vf_create", "vf_destroy", "vf_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2407_14783_amd import capi
    lib = ctypes.CDLL(capi.LIB_PATH)
    names = _declared()
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, f"not exported: {missing}"
    assert sorted(capi.EXPORTED) == names


def test_struct_layouts_match_header():
    from paper_2407_14783_amd import capi
    assert ctypes.sizeof(capi.DynParams) == 128
    assert capi.VIEW_DTYPE.itemsize == 72 and capi.VIEW_DTYPE.fields["out_offset"][1] == 32
    assert capi.VIEW_DTYPE.fields["mount_q"][1] == 40 and capi.VIEW_DTYPE.fields["mount_t"][1] == 56
    assert capi.VIEW_DTYPE.fields["swarm"][1] == 68
    assert capi.NODE_DTYPE.itemsize == 128 and capi.TRI_DTYPE.itemsize == 48
    assert capi.NODE_DTYPE.fields["child"][1] == 96 and capi.NODE_DTYPE.fields["count"][1] == 112
    assert capi.NODE_DTYPE.fields["order"][1] == 116
    assert ctypes.sizeof(capi.SceneInfo) == 80 and capi.SceneInfo.builder.offset == 72
    assert capi.NODE8_DTYPE.itemsize == 256 and capi.NODE8_DTYPE.fields["child"][1] == 192
    assert capi.NODE8_DTYPE.fields["order"][1] == 224


def test_params_struct_roundtrip():
    from paper_2407_14783_amd import capi
    from workloads import default_params
    p = default_params()
    s = capi.params_struct(p)
    raw = np.frombuffer(bytes(s), dtype=np.float32)
    assert np.isclose(raw[0], p["dt"]) and np.isclose(s.f_max, p["f_max"]) and list(s.k_rate) == [20.0, 20.0, 10.0]


def test_option_setters_reject_a_null_context():
    """Every option setter answers a NULL context with VF_EINVAL and a message naming itself, on the host
    (no device call is made on that path)."""
    from paper_2407_14783_amd import capi
    lib = ctypes.CDLL(capi.LIB_PATH)
    lib.vf_last_error.restype = ctypes.c_char_p
    lib.vf_last_error.argtypes = [ctypes.c_void_p]
    for name in ("vf_set_spatial_order", "vf_set_cost_order", "vf_set_launch_mode", "vf_set_bvh_builder",
                 "vf_set_bvh_leaf_size", "vf_set_stats", "vf_set_timing"):
        fn = getattr(lib, name)
        fn.restype = ctypes.c_int32
        fn.argtypes = [ctypes.c_void_p, ctypes.c_int32]
        assert fn(None, 1) == -1, name            # VF_EINVAL
        assert name in lib.vf_last_error(None).decode(), name
