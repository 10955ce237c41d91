"""ctypes binding of include/visfly.h: the same entry points, argument marshalling only.

The shared library libvisfly_hip.so must have been built in-tree
(``python -m paper_2407_14783_amd.build``); importing this module without it
raises ImportError -- there is no fallback.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvisfly_hip.so")

VF_OK, VF_EINVAL, VF_ENOMEM, VF_ENOSCENE, VF_EHIP, VF_EBUSY, VF_EDEVICE = 0, -1, -2, -3, -4, -5, -6
VF_RK4, VF_EULER = 0, 1
VF_CTBR, VF_SRT, VF_PS, VF_LV = 0, 1, 2, 3
VF_LAUNCH_SPLIT, VF_LAUNCH_FUSED, VF_LAUNCH_AUTO = 0, 1, 2
VF_BVH_CLUSTER, VF_BVH_RADIX = 0, 1
VF_NOISE_NONE, VF_NOISE_NORMAL, VF_NOISE_SPECKLE, VF_NOISE_SALT_PEPPER, VF_NOISE_POISSON = 0, 1, 2, 3, 4
STATUS_NAMES = {0: "VF_OK", -1: "VF_EINVAL", -2: "VF_ENOMEM", -3: "VF_ENOSCENE", -4: "VF_EHIP", -5: "VF_EBUSY",
                -6: "VF_EDEVICE"}

# every symbol include/visfly.h declares
EXPORTED = ("vf_create", "vf_destroy", "vf_scene_build", "vf_scene_free", "vf_scene_info_get", "vf_scene_export",
            "vf_step", "vf_render", "vf_step_backward", "vf_render_backward", "vf_set_stats", "vf_stats_read",
            "vf_sync_check", "vf_mem_usage", "vf_last_error", "vf_set_launch_mode", "vf_set_bvh_builder", "vf_set_bvh_leaf_size", "vf_server_create",
            "vf_server_submit", "vf_server_poll", "vf_server_wait", "vf_server_stats_get", "vf_server_destroy",
            "vf_closest_point", "vf_sensor_noise", "vf_scene_set_labels", "vf_segmentation", "vf_imu", "vf_collision", "vf_set_swarms", "vf_set_spatial_order", "vf_set_cost_order", "vf_set_timing", "vf_timing_read",
            "vf_set_render_noise", "vf_server_inject_faults", "vf_step_noalloc")


class DynParams(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_float), ("n_sub", ctypes.c_int32), ("integrator", ctypes.c_int32),
                ("ctrl", ctypes.c_int32), ("mass", ctypes.c_float), ("arm", ctypes.c_float),
                ("J", ctypes.c_float * 3), ("tau_motor", ctypes.c_float), ("kappa_yaw", ctypes.c_float),
                ("f_max", ctypes.c_float), ("k_lin", ctypes.c_float * 3), ("c_quad", ctypes.c_float * 3),
                ("g", ctypes.c_float), ("k_rate", ctypes.c_float * 3), ("k_pos", ctypes.c_float * 3),
                ("k_vel", ctypes.c_float * 3), ("k_att", ctypes.c_float * 3), ("max_tilt", ctypes.c_float)]


class Noise(ctypes.Structure):
    _fields_ = [("depth_model", ctypes.c_int32), ("depth_sigma", ctypes.c_float), ("depth_p", ctypes.c_float),
                ("depth_scale", ctypes.c_float),
                ("rgb_model", ctypes.c_int32), ("rgb_sigma", ctypes.c_float), ("rgb_p", ctypes.c_float),
                ("rgb_scale", ctypes.c_float),
                ("seg_model", ctypes.c_int32), ("seg_sigma", ctypes.c_float), ("seg_p", ctypes.c_float),
                ("seg_scale", ctypes.c_float), ("seg_salt_label", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("seed", ctypes.c_uint64)]


class SceneInfo(ctypes.Structure):
    _fields_ = [("n_tris", ctypes.c_int64), ("n_nodes", ctypes.c_int64), ("n_leaves", ctypes.c_int64),
                ("bytes", ctypes.c_int64), ("depth", ctypes.c_int32), ("leaf_max", ctypes.c_int32),
                ("bounds_lo", ctypes.c_float * 3), ("bounds_hi", ctypes.c_float * 3), ("build_ms", ctypes.c_float),
                ("width", ctypes.c_int32), ("builder", ctypes.c_int32), ("reserved", ctypes.c_int32)]


VIEW_DTYPE = np.dtype([("scene_id", "<i4"), ("H", "<i4"), ("W", "<i4"), ("flags", "<i4"), ("hfov", "<f4"),
                       ("near_clip", "<f4"), ("far_clip", "<f4"), ("miss_depth", "<f4"), ("out_offset", "<i8"),
                       ("mount_q", "<f4", 4), ("mount_t", "<f4", 3), ("swarm", "<i4")])
NODE_DTYPE = np.dtype([("lo_x", "<f4", 4), ("hi_x", "<f4", 4), ("lo_y", "<f4", 4), ("hi_y", "<f4", 4),
                       ("lo_z", "<f4", 4), ("hi_z", "<f4", 4), ("child", "<i4", 4), ("count", "u1", 4),
                       ("order", "<u4", 3)])
NODE8_DTYPE = np.dtype([("lo_x", "<f4", 8), ("hi_x", "<f4", 8), ("lo_y", "<f4", 8), ("hi_y", "<f4", 8),
                        ("lo_z", "<f4", 8), ("hi_z", "<f4", 8), ("child", "<i4", 8), ("order", "<u4", 8)])
EMPTY_CHILD = -2 ** 31
TRI_DTYPE = np.dtype([("v0", "<f4", 3), ("id", "<i4"), ("e1", "<f4", 3), ("pad1", "<f4"), ("e2", "<f4", 3),
                      ("pad2", "<f4")])
assert VIEW_DTYPE.itemsize == 72 and NODE_DTYPE.itemsize == 128 and TRI_DTYPE.itemsize == 48
assert NODE8_DTYPE.itemsize == 256
assert ctypes.sizeof(DynParams) == 128 and ctypes.sizeof(Noise) == 64


class VfError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2407_14783_amd.build` (hipcc, gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, U64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
    sig = {
        "vf_create": ([ctypes.c_int, ctypes.c_size_t, ctypes.POINTER(P)], I32),
        "vf_destroy": ([P], I32),
        "vf_scene_build": ([P, P, I64, P, I64, P, P, ctypes.POINTER(I32)], I32),
        "vf_scene_free": ([P, I32], I32),
        "vf_scene_info_get": ([P, I32, ctypes.POINTER(SceneInfo)], I32),
        "vf_scene_export": ([P, I32, P, I64, P, I64], I32),
        "vf_step": ([P, ctypes.POINTER(DynParams), I64, P, P, I64, P, P, I32, I32, P, P, P, I64, P], I32),
        "vf_step_noalloc": ([P, ctypes.POINTER(DynParams), I64, P, P, I64, P, P, I32, I32, P, P, P, I64, P], I32),
        "vf_render": ([P, I64, P, P, I64, P, I32, I32, P, P, P, I64, P], I32),
        "vf_step_backward": ([P, ctypes.POINTER(DynParams), I64, P, P, P, P, P, P], I32),
        "vf_render_backward": ([P, I64, P, P, I32, I32, P, P, I64, P, P], I32),
        "vf_set_stats": ([P, I32], I32),
        "vf_set_launch_mode": ([P, I32], I32),
        "vf_set_bvh_builder": ([P, I32], I32),
        "vf_set_bvh_leaf_size": ([P, I32], I32),
        "vf_set_spatial_order": ([P, I32], I32),
        "vf_set_cost_order": ([P, I32], I32),
        "vf_set_timing": ([P, I32], I32),
        "vf_timing_read": ([P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(I64), I32], I32),
        "vf_closest_point": ([P, I64, P, P, I32, ctypes.c_float, P, P, P, P], I32),
        "vf_sensor_noise": ([P, I64, P, I32, I32, ctypes.POINTER(Noise), P, P, P, P, I64, P], I32),
        "vf_set_render_noise": ([P, ctypes.POINTER(Noise)], I32),
        "vf_scene_set_labels": ([P, I32, P], I32),
        "vf_set_swarms": ([P, I32, P, P, P, P], I32),
        "vf_collision": ([P, I64, P, P, I64, P, ctypes.c_float, ctypes.c_float, P, P, P, P], I32),
        "vf_segmentation": ([P, I64, P, I32, I32, P, P, I64, P], I32),
        "vf_imu": ([P, ctypes.POINTER(DynParams), I64, P, P, I64, ctypes.c_float, ctypes.c_float, U64, P, P, P], I32),
        "vf_stats_read": ([P, ctypes.POINTER(U64), I32], I32),
        "vf_sync_check": ([P, P], I32),
        "vf_mem_usage": ([P, ctypes.POINTER(I64), ctypes.POINTER(I64)], I32),
        "vf_last_error": ([P], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


lib = _load()


def last_error():
    return lib.vf_last_error(None).decode(errors="replace")


def check(status, what=""):
    if status != VF_OK:
        raise VfError(status, f"{what}: {last_error()}" if what else last_error())
    return status


def params_struct(p):
    """DynParams from a dict with the keys of workloads.default_params()."""
    s = DynParams()
    s.dt = p["dt"]
    s.n_sub = int(p["n_sub"])
    s.integrator = int(p["integrator"])
    s.ctrl = int(p["ctrl"])
    s.mass = p["mass"]
    s.arm = p["arm"]
    s.J[:] = list(p["J"])
    s.tau_motor = p["tau_motor"]
    s.kappa_yaw = p["kappa_yaw"]
    s.f_max = p["f_max"]
    s.k_lin[:] = list(p["k_lin"])
    s.c_quad[:] = list(p["c_quad"])
    s.g = p["g"]
    s.k_rate[:] = list(p["k_rate"])
    s.k_pos[:] = list(p["k_pos"])
    s.k_vel[:] = list(p["k_vel"])
    s.k_att[:] = list(p["k_att"])
    s.max_tilt = p["max_tilt"]
    return s
