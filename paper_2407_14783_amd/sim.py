"""Torch-facing wrapper over the C ABI.  Torch supplies device memory and streams only;
every step of the path runs in the library's HIP kernels."""
import ctypes

import numpy as np
import torch

from . import capi
from .capi import check, lib


def _ptr(t):
    """Device address of a contiguous device tensor, as an integer (every entry point declares its pointer
    arguments as void*, so ctypes passes it at full width)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return t.data_ptr()


def _check_views(views, n):
    """views must hold at least n vf_view records (72 bytes each)."""
    if views is not None and views.numel() * views.element_size() < capi.VIEW_DTYPE.itemsize * n:
        raise ValueError(f"views holds fewer than n = {n} entries of {capi.VIEW_DTYPE.itemsize} bytes")


def _check_rows(t, n, cols, name):
    if t is not None and (t.numel() < n * cols):
        raise ValueError(f"{name} holds fewer than {n} x {cols} values")


# The current stream's raw handle without building a torch Stream object (that costs a few microseconds per
# call, as much as a small step's whole launch); the public route where the raw getter is absent.
_raw_stream = getattr(torch._C, "_cuda_getCurrentRawStream", None)


def _stream(stream):
    if stream is not None:
        return stream.cuda_stream
    if _raw_stream is not None:
        return _raw_stream(torch.cuda.current_device())
    return torch.cuda.current_stream().cuda_stream


def make_views(n, scene_ids, hw, hfov=np.pi / 2, near=0.01, far=100.0, miss_depth=None, device="cuda",
               noise_keys=None, mount_q=None, mount_t=None, swarm=None):
    """Per-view array [n] on the device plus (out_pixels, offsets, max_h, max_w).

    scene_ids: int or [n]; hw: (H, W) or [n, 2]; outputs are packed view after view.
    noise_keys: per-view sensor-noise key ([n] ints; default the view index).
    mount_q / mount_t: camera orientation (w, x, y, z) and position in the body frame, [4] / [3] or
    [n, 4] / [n, 3]; default no rotation, no offset.
    swarm: per-view swarm index (int or [n]; -1 none) of the table given to Context.set_swarms.
    """
    scene_ids = np.broadcast_to(np.asarray(scene_ids, dtype=np.int64).reshape(-1), (n,))
    hw = np.broadcast_to(np.asarray(hw, dtype=np.int64).reshape(-1, 2), (n, 2))
    v = np.zeros(n, dtype=capi.VIEW_DTYPE)
    v["scene_id"] = scene_ids
    v["H"] = hw[:, 0]
    v["W"] = hw[:, 1]
    v["hfov"] = hfov
    v["near_clip"] = near
    v["far_clip"] = far
    v["miss_depth"] = far if miss_depth is None else miss_depth
    v["flags"] = np.arange(n) if noise_keys is None else np.broadcast_to(np.asarray(noise_keys), (n,))
    v["mount_q"] = (1.0, 0.0, 0.0, 0.0) if mount_q is None else np.broadcast_to(np.asarray(mount_q), (n, 4))
    v["mount_t"] = 0.0 if mount_t is None else np.broadcast_to(np.asarray(mount_t), (n, 3))
    v["swarm"] = 0 if swarm is None else np.broadcast_to(np.asarray(swarm), (n,)) + 1
    px = hw[:, 0] * hw[:, 1]
    offsets = np.concatenate([[0], np.cumsum(px)[:-1]]).astype(np.int64)
    v["out_offset"] = offsets
    dev = torch.from_numpy(v.view(np.uint8).copy()).to(device)
    return dev, int(px.sum()), offsets, int(hw[:, 0].max()), int(hw[:, 1].max())


class Context:
    """One library context on one GPU (scenes, scratch, counters)."""

    def __init__(self, device=0, budget_bytes=0):
        torch.cuda.init()
        self.device = device
        h = ctypes.c_void_p()
        check(lib.vf_create(device, budget_bytes, ctypes.byref(h)), "vf_create")
        self.h = h

    def close(self):
        if self.h:
            check(lib.vf_destroy(self.h), "vf_destroy")
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- scenes
    def build_scene(self, verts, tris, rgb=None, stream=None):
        v = torch.as_tensor(np.asarray(verts, dtype=np.float32)).cuda(self.device).contiguous()
        t = torch.as_tensor(np.asarray(tris, dtype=np.int32)).cuda(self.device).contiguous()
        c = None if rgb is None else torch.as_tensor(np.asarray(rgb, dtype=np.uint8)).cuda(self.device).contiguous()
        sid = ctypes.c_int32(-1)
        check(lib.vf_scene_build(self.h, _ptr(v), v.shape[0], _ptr(t), t.shape[0], _ptr(c), _stream(stream),
                                 ctypes.byref(sid)), "vf_scene_build")
        return sid.value

    def free_scene(self, sid):
        check(lib.vf_scene_free(self.h, sid), "vf_scene_free")

    def scene_info(self, sid):
        info = capi.SceneInfo()
        check(lib.vf_scene_info_get(self.h, sid, ctypes.byref(info)), "vf_scene_info_get")
        return {"n_tris": info.n_tris, "n_nodes": info.n_nodes, "bytes": info.bytes, "depth": info.depth,
                "leaf_max": info.leaf_max, "bounds_lo": list(info.bounds_lo), "bounds_hi": list(info.bounds_hi),
                "build_ms": info.build_ms, "width": info.width,
                "builder": "cluster" if info.builder == capi.VF_BVH_CLUSTER else "radix"}

    def export_scene(self, sid):
        info = self.scene_info(sid)
        nodes = np.zeros(info["n_nodes"], dtype=capi.NODE_DTYPE if info["width"] == 4 else capi.NODE8_DTYPE)
        tris = np.zeros(info["n_tris"], dtype=capi.TRI_DTYPE)
        check(lib.vf_scene_export(self.h, sid, nodes.ctypes.data_as(ctypes.c_void_p), nodes.nbytes,
                                  tris.ctypes.data_as(ctypes.c_void_p), tris.nbytes), "vf_scene_export")
        return nodes, tris

    # ---------------------------------------------------------------- step / render
    def step(self, params, state, action, views=None, env_idx=None, max_hw=(0, 0), depth=None, tri_id=None,
             rgb=None, out_pixels=0, stream=None):
        p = params if isinstance(params, capi.DynParams) else capi.params_struct(params)
        n = action.shape[0]
        _check_views(views, n)
        if env_idx is not None and env_idx.numel() < n:
            raise ValueError("env_idx holds fewer than n entries")
        if env_idx is None:
            _check_rows(state, n, 17, "state")
        check(lib.vf_step(self.h, ctypes.byref(p), n, _ptr(env_idx), _ptr(state), state.shape[0], _ptr(action),
                          _ptr(views), int(max_hw[0]), int(max_hw[1]), _ptr(depth), _ptr(tri_id), _ptr(rgb),
                          int(out_pixels), _stream(stream)), "vf_step")

    def step_noalloc(self, params, state, action, views=None, env_idx=None, max_hw=(0, 0), depth=None, tri_id=None,
                     rgb=None, out_pixels=0, stream=None):
        """vf_step_noalloc: step() with no device allocation (scratch in the library's per-GPU array)."""
        p = params if isinstance(params, capi.DynParams) else capi.params_struct(params)
        n = action.shape[0]
        _check_views(views, n)
        if env_idx is not None and env_idx.numel() < n:
            raise ValueError("env_idx holds fewer than n entries")
        if env_idx is None:
            _check_rows(state, n, 17, "state")
        check(lib.vf_step_noalloc(self.h, ctypes.byref(p), n, _ptr(env_idx), _ptr(state), state.shape[0],
                                  _ptr(action), _ptr(views), int(max_hw[0]), int(max_hw[1]), _ptr(depth),
                                  _ptr(tri_id), _ptr(rgb), int(out_pixels), _stream(stream)), "vf_step_noalloc")

    def render(self, state, views, n=None, env_idx=None, max_hw=(64, 64), depth=None, tri_id=None, rgb=None,
               out_pixels=0, stream=None):
        n = state.shape[0] if n is None else n
        _check_views(views, n)
        if env_idx is not None and env_idx.numel() < n:
            raise ValueError("env_idx holds fewer than n entries")
        if env_idx is None:
            _check_rows(state, n, 17, "state")
        check(lib.vf_render(self.h, n, _ptr(env_idx), _ptr(state), state.shape[0], _ptr(views), int(max_hw[0]),
                            int(max_hw[1]), _ptr(depth), _ptr(tri_id), _ptr(rgb), int(out_pixels),
                            _stream(stream)), "vf_render")

    def step_backward(self, params, state_in, action, grad_out, grad_in, grad_action, stream=None):
        n = state_in.shape[0]
        for t, c, nm in ((action, 4, "action"), (grad_out, 17, "grad_out"), (grad_in, 17, "grad_in"),
                         (grad_action, 4, "grad_action")):
            _check_rows(t, n, c, nm)
        p = params if isinstance(params, capi.DynParams) else capi.params_struct(params)
        check(lib.vf_step_backward(self.h, ctypes.byref(p), state_in.shape[0], _ptr(state_in), _ptr(action),
                                   _ptr(grad_out), _ptr(grad_in), _ptr(grad_action), _stream(stream)),
              "vf_step_backward")

    def render_backward(self, state, views, max_hw, tri_id, grad_depth, out_pixels, grad_state, stream=None):
        _check_views(views, state.shape[0])
        _check_rows(grad_state, state.shape[0], 17, "grad_state")
        check(lib.vf_render_backward(self.h, state.shape[0], _ptr(state), _ptr(views), int(max_hw[0]),
                                     int(max_hw[1]), _ptr(tri_id), _ptr(grad_depth), int(out_pixels),
                                     _ptr(grad_state), _stream(stream)), "vf_render_backward")

    def closest_point(self, points, scene_id, max_dist=1e30, closest=None, tri_id=None, stream=None):
        """Distance [n] from each point [n, 3] (device) to the nearest triangle of scene_id (an int or a
        device int32 tensor [n] of per-point scenes)."""
        n = points.shape[0]
        _check_rows(points, n, 3, "points")
        dist = torch.empty(n, dtype=torch.float32, device=points.device)
        ids_t = scene_id if torch.is_tensor(scene_id) else None
        sid0 = 0 if ids_t is not None else int(scene_id)
        check(lib.vf_closest_point(self.h, n, _ptr(points), _ptr(ids_t), sid0, float(max_dist), _ptr(dist),
                                   _ptr(closest), _ptr(tri_id), _stream(stream)), "vf_closest_point")
        return dist

    def collision(self, state, views, radius, n=None, env_idx=None, max_dist=1e30, rel=None, collided=None,
                  stream=None):
        """Nearest-obstacle distance [n] of each agent's position in its view's scene, with the offset to
        that point (rel [n, 3], optional) and the contact flag dist <= radius (collided [n] uint8, optional)."""
        n = state.shape[0] if n is None else n
        _check_views(views, n)
        if env_idx is not None and env_idx.numel() < n:
            raise ValueError("env_idx holds fewer than n entries")
        if env_idx is None:
            _check_rows(state, n, 17, "state")
        _check_rows(rel, n, 3, "rel")
        _check_rows(collided, n, 1, "collided")
        dist = torch.empty(n, dtype=torch.float32, device=state.device)
        check(lib.vf_collision(self.h, n, _ptr(env_idx), _ptr(state), state.shape[0], _ptr(views), float(radius),
                               float(max_dist), _ptr(dist), _ptr(rel), _ptr(collided), _stream(stream)),
              "vf_collision")
        return dist

    def set_swarms(self, groups, half_extent=(0.15, 0.15, 0.05), rgb=(255, 64, 0)):
        """Swarms as lists of state slots (agents that see each other); [] clears."""
        offs = np.zeros(len(groups) + 1, dtype=np.int32)
        offs[1:] = np.cumsum([len(g) for g in groups])
        slots = np.concatenate([np.asarray(g, dtype=np.int32) for g in groups]) if groups else np.zeros(0, np.int32)
        slots = np.ascontiguousarray(slots, dtype=np.int32)
        half = (ctypes.c_float * 3)(*half_extent)
        col = (ctypes.c_uint8 * 3)(*rgb)
        check(lib.vf_set_swarms(self.h, len(groups), offs.ctypes.data_as(ctypes.c_void_p),
                                slots.ctypes.data_as(ctypes.c_void_p), half, col), "vf_set_swarms")

    # ---------------------------------------------------------------- sensors
    @staticmethod
    def noise_config(depth_model=capi.VF_NOISE_NONE, depth_sigma=0.0, depth_p=0.0, depth_scale=1.0,
                     rgb_model=capi.VF_NOISE_NONE, rgb_sigma=0.0, rgb_p=0.0, rgb_scale=1.0,
                     seg_model=capi.VF_NOISE_NONE, seg_sigma=0.0, seg_p=0.0, seg_scale=1.0, seg_salt_label=0, seed=0):
        """A vf_noise record (Table II models of the three image sensors)."""
        return capi.Noise(int(depth_model), float(depth_sigma), float(depth_p), float(depth_scale), int(rgb_model),
                          float(rgb_sigma), float(rgb_p), float(rgb_scale), int(seg_model), float(seg_sigma),
                          float(seg_p), float(seg_scale), int(seg_salt_label), 0, int(seed) & 0xFFFFFFFFFFFFFFFF)

    def sensor_noise(self, views, n, max_hw, out_pixels, depth=None, rgb=None, tri_id=None, seg=None, stream=None,
                     **cfg):
        """Table II noise applied in place to rendered depth / planar rgb / labels (keys from views' flags);
        cfg takes the keyword arguments of noise_config()."""
        _check_views(views, n)
        for t, c, nm in ((depth, 1, "depth"), (rgb, 3, "rgb"), (tri_id, 1, "tri_id"), (seg, 1, "seg")):
            _check_rows(t, out_pixels, c, nm)
        rec = self.noise_config(**cfg)
        check(lib.vf_sensor_noise(self.h, n, _ptr(views), int(max_hw[0]), int(max_hw[1]), ctypes.byref(rec),
                                  _ptr(tri_id), _ptr(depth), _ptr(rgb), _ptr(seg), int(out_pixels), _stream(stream)),
              "vf_sensor_noise")

    def set_render_noise(self, **cfg):
        """Depth / colour noise applied by the render kernel's epilogue in later step / render calls (no
        arguments: off); cfg takes the keyword arguments of noise_config()."""
        if not cfg:
            check(lib.vf_set_render_noise(self.h, None), "vf_set_render_noise")
            return
        rec = self.noise_config(**cfg)
        check(lib.vf_set_render_noise(self.h, ctypes.byref(rec)), "vf_set_render_noise")

    def set_labels(self, sid, labels):
        """Per-triangle int32 semantic labels of a scene (None removes them)."""
        if labels is None:
            check(lib.vf_scene_set_labels(self.h, sid, None), "vf_scene_set_labels")
            return
        lab = torch.as_tensor(np.asarray(labels, dtype=np.int32)).cuda(self.device)
        if lab.numel() != self.scene_info(sid)["n_tris"]:
            raise ValueError("labels must hold one value per triangle")
        check(lib.vf_scene_set_labels(self.h, sid, _ptr(lab)), "vf_scene_set_labels")

    def segmentation(self, views, n, max_hw, tri_id, out_pixels, seg=None, stream=None):
        _check_views(views, n)
        _check_rows(tri_id, out_pixels, 1, "tri_id")
        if seg is None:
            seg = torch.empty(out_pixels, dtype=torch.int32, device=tri_id.device)
        _check_rows(seg, out_pixels, 1, "seg")
        check(lib.vf_segmentation(self.h, n, _ptr(views), int(max_hw[0]), int(max_hw[1]), _ptr(tri_id), _ptr(seg),
                                  int(out_pixels), _stream(stream)), "vf_segmentation")
        return seg

    def imu(self, params, state, n=None, env_idx=None, sigma_acc=0.0, sigma_gyro=0.0, seed=0, keys=None,
            out=None, stream=None):
        """[n, 6] accelerometer (specific force, body frame) and gyro readings at the given states."""
        p = params if isinstance(params, capi.DynParams) else capi.params_struct(params)
        n = state.shape[0] if n is None else n
        if env_idx is not None and env_idx.numel() < n:
            raise ValueError("env_idx holds fewer than n entries")
        if env_idx is None:
            _check_rows(state, n, 17, "state")
        if keys is not None and keys.numel() < n:
            raise ValueError("keys holds fewer than n entries")
        if out is None:
            out = torch.empty((n, 6), dtype=torch.float32, device=state.device)
        _check_rows(out, n, 6, "out")
        check(lib.vf_imu(self.h, ctypes.byref(p), n, _ptr(env_idx), _ptr(state), state.shape[0], float(sigma_acc),
                         float(sigma_gyro), int(seed) & 0xFFFFFFFFFFFFFFFF, _ptr(keys), _ptr(out), _stream(stream)),
              "vf_imu")
        return out

    # ---------------------------------------------------------------- diagnostics
    def sync_check(self, stream=None):
        check(lib.vf_sync_check(self.h, _stream(stream)), "vf_sync_check")

    def set_launch_mode(self, fused):
        """True: fused single launch; False: split; None: automatic by batch size (the default)."""
        mode = capi.VF_LAUNCH_AUTO if fused is None else (capi.VF_LAUNCH_FUSED if fused else capi.VF_LAUNCH_SPLIT)
        check(lib.vf_set_launch_mode(self.h, mode), "vf_set_launch_mode")

    def set_bvh_builder(self, builder):
        """Binary tree of later scene builds: "cluster" (locally-ordered clustering, the default) or "radix"
        (the Morton radix tree)."""
        code = {"cluster": capi.VF_BVH_CLUSTER, "radix": capi.VF_BVH_RADIX}[builder]
        check(lib.vf_set_bvh_builder(self.h, code), "vf_set_bvh_builder")

    def set_bvh_leaf_size(self, max_tris):
        """Largest number of triangles per BVH leaf (1..4) for later scene builds."""
        check(lib.vf_set_bvh_leaf_size(self.h, int(max_tris)), "vf_set_bvh_leaf_size")

    def set_spatial_order(self, on):
        """Sort split-launch batches by (scene, position) before rendering (default on)."""
        check(lib.vf_set_spatial_order(self.h, 1 if on else 0), "vf_set_spatial_order")

    def set_cost_order(self, on):
        """Start each XCD's longest packets first, by the work the previous launch of the same shape
        reported (default on)."""
        check(lib.vf_set_cost_order(self.h, 1 if on else 0), "vf_set_cost_order")

    def set_timing(self, on):
        """Record HIP events around every render-kernel launch (see timing_read)."""
        check(lib.vf_set_timing(self.h, 1 if on else 0), "vf_set_timing")

    def timing_read(self, reset=True):
        """(summed render-kernel milliseconds, launches) since the last reset."""
        ms, n = ctypes.c_double(), ctypes.c_int64()
        check(lib.vf_timing_read(self.h, ctypes.byref(ms), ctypes.byref(n), 1 if reset else 0), "vf_timing_read")
        return ms.value, n.value

    def set_stats(self, on):
        check(lib.vf_set_stats(self.h, 1 if on else 0), "vf_set_stats")

    def read_stats(self, reset=True):
        out = (ctypes.c_uint64 * 12)()
        check(lib.vf_stats_read(self.h, out, 1 if reset else 0), "vf_stats_read")
        keys = ("rays", "node_lane", "box_lane", "tri_lane", "node_wave", "tri_wave", "box_ops", "hits",
                "need_node", "need_box", "need_tri", "member_tests")
        return dict(zip(keys, list(out)))

    def mem_usage(self):
        u, b = ctypes.c_int64(), ctypes.c_int64()
        check(lib.vf_mem_usage(self.h, ctypes.byref(u), ctypes.byref(b)), "vf_mem_usage")
        return u.value, b.value
