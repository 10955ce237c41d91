"""FP64 pinhole camera and brute-force closest-hit render (Sec. III-B).

Readings of what the paper leaves open (it rasterises with Habitat-Sim and
gives no camera model):
  * The camera sits at the body origin: optical axis +x_B, image right -y_B,
    image up +z_B.  Pixel (row r from the top, column c from the left) of an
    H x W image with horizontal field of view hfov looks along
        d_B = (1, -u, v),  u = (2 (c + 1/2) / W - 1) tan(hfov/2),
                           v = (1 - 2 (r + 1/2) / H) tan(hfov/2) H / W,
    and d = R(q) d_B in the world frame.  Because the forward component of d_B
    is 1, the hit distance t along d is the planar (z-buffer) depth.
  * near = 0.01 m, far = 100 m; hits outside [near, far] are ignored; a miss
    gives depth = miss_depth, id = -1, colour (0, 0, 0).
  * Colour is the flat per-triangle uint8 RGB of the hit triangle.
The brute-force caster itself is ``brute.c`` (every ray against every triangle).
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "brute.c")
_LIB = os.path.join(_HERE, "liboracle_brute.so")
_lib = None


def build_library(force=False):
    """Compile brute.c with gcc (FP64, no contraction, OpenMP) into oracle/liboracle_brute.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
                               "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build_library()
        lib = ctypes.CDLL(_LIB)
        d, i64, i32 = ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32)
        lib.oracle_cast.argtypes = [ctypes.c_int64, d, d, ctypes.c_int64, d, d, d, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_int32, d, i64, d, d, d, i32, i32]
        lib.oracle_cast.restype = None
        lib.oracle_closest_point.argtypes = [ctypes.c_int64, d, ctypes.c_int64, d, d, d, d, d, i64]
        lib.oracle_closest_point.restype = None
        _lib = lib
    return _lib


def _p(a, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


def triangle_vertices(verts, tris):
    v = np.asarray(verts, dtype=np.float64)
    t = np.asarray(tris, dtype=np.int64)
    return (np.ascontiguousarray(v[t[:, 0]]), np.ascontiguousarray(v[t[:, 1]]), np.ascontiguousarray(v[t[:, 2]]))


def cast(orig, dirs, verts, tris, near=0.01, far=100.0, with_mask=True):
    """Brute-force closest hit of rays [R,3] (origins [R,3] or [3]) against all triangles.

    Returns a dict of per-ray arrays: t (inf on miss), id (-1 on miss) and, with
    with_mask, t2, edge_hit, near_miss, boundary, plus 'threads'.
    """
    dirs = np.ascontiguousarray(np.asarray(dirs, dtype=np.float64).reshape(-1, 3))
    n = dirs.shape[0]
    orig = np.ascontiguousarray(np.broadcast_to(np.asarray(orig, dtype=np.float64).reshape(-1, 3), (n, 3)))
    v0, v1, v2 = triangle_vertices(verts, tris)
    lib = _load()
    out = {k: np.empty(n) for k in ("t", "t2", "edge_hit", "near_miss")}
    out["id"] = np.empty(n, dtype=np.int64)
    out["boundary"] = np.zeros(n, dtype=np.int32)
    th = np.zeros(1, dtype=np.int32)
    d = ctypes.c_double
    lib.oracle_cast(n, _p(orig, d), _p(dirs, d), v0.shape[0], _p(v0, d), _p(v1, d), _p(v2, d), near, far,
                    1 if with_mask else 0, _p(out["t"], d), _p(out["id"], ctypes.c_int64), _p(out["t2"], d),
                    _p(out["edge_hit"], d), _p(out["near_miss"], d), _p(out["boundary"], ctypes.c_int32),
                    _p(th, ctypes.c_int32))
    out["threads"] = int(th[0])
    return out


def cast_boxes(orig, dirs, centers, quats, half, near=0.01, far=100.0):
    """Entry of each ray [R] into the nearest of K oriented boxes (the body boxes of other agents),
    by the slab method in each box's frame, FP64.

    A box is hit where the ray enters it at t in [near, far]; a ray starting inside a box does not
    see that box.  Equal entries go to the lower box index.  Returns t [R] (inf on a miss), k [R]
    (-1 on a miss) and two mask quantities: edge, the distance of the entry point to the border of
    the face it enters through, and gap, for a ray missing a box, (t_enter - t_exit) |d| minimised
    over the boxes (how far the slab intervals miss).
    """
    dirs = np.asarray(dirs, dtype=np.float64).reshape(-1, 3)
    r = dirs.shape[0]
    orig = np.broadcast_to(np.asarray(orig, dtype=np.float64).reshape(-1, 3), (r, 3))
    half = np.asarray(half, dtype=np.float64)
    t_best = np.full(r, np.inf)
    k_best = np.full(r, -1, dtype=np.int64)
    edge = np.full(r, np.inf)
    gap = np.full(r, np.inf)
    for k in range(np.asarray(centers).shape[0]):
        rot = quat_to_rot(np.asarray(quats[k], dtype=np.float64))
        o = (orig - np.asarray(centers[k], dtype=np.float64)) @ rot      # R^T (o - c), row-wise
        d = dirs @ rot
        with np.errstate(divide="ignore", invalid="ignore"):
            t1 = (-half - o) / d
            t2 = (half - o) / d
        lo = np.where(d == 0, np.where(np.abs(o) <= half, -np.inf, np.inf), np.minimum(t1, t2))
        hi = np.where(d == 0, np.where(np.abs(o) <= half, np.inf, -np.inf), np.maximum(t1, t2))
        t_in = lo.max(axis=1)
        t_out = hi.min(axis=1)
        hit = (t_in <= t_out) & (t_in >= near) & (t_in <= far)
        take = hit & (t_in < t_best)
        if take.any():
            axis = lo.argmax(axis=1)
            x = o + t_in[:, None] * d
            margin = half[None, :] - np.abs(x)
            margin[np.arange(r), axis] = np.inf
            edge = np.where(take, margin.min(axis=1), edge)
            t_best = np.where(take, t_in, t_best)
            k_best = np.where(take, k, k_best)
        miss = ~(t_in <= t_out) & np.isfinite(t_in) & np.isfinite(t_out)
        g = np.where(miss, (t_in - t_out) * np.linalg.norm(dirs, axis=1), np.inf)
        gap = np.minimum(gap, g)
    return {"t": t_best, "k": k_best, "edge": edge, "gap": gap}


def closest_points(points, verts, tris):
    """Nearest point on the mesh to each query point (exact point-triangle distance, brute force)."""
    pts = np.ascontiguousarray(np.asarray(points, dtype=np.float64).reshape(-1, 3))
    v0, v1, v2 = triangle_vertices(verts, tris)
    n = pts.shape[0]
    dist = np.empty(n)
    pt = np.empty((n, 3))
    ids = np.empty(n, dtype=np.int64)
    d = ctypes.c_double
    _load().oracle_closest_point(n, _p(pts, d), v0.shape[0], _p(v0, d), _p(v1, d), _p(v2, d), _p(dist, d),
                                 _p(pt, d), _p(ids, ctypes.c_int64))
    return dist, pt, ids


def quat_to_rot(q):
    """R_WB of a quaternion (w,x,y,z), normalised first."""
    q = np.asarray(q, dtype=np.float64)
    q = q / np.linalg.norm(q, axis=-1, keepdims=True)
    w, x, y, z = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1),
    ], -2)


def camera_dirs_body(h, w, hfov):
    """Body-frame ray directions [H,W,3] = (1, -u, v) with pixel centres at +1/2."""
    tan_half = np.tan(0.5 * hfov)
    c = np.arange(w, dtype=np.float64)
    r = np.arange(h, dtype=np.float64)
    u = (2.0 * (c + 0.5) / w - 1.0) * tan_half
    v = (1.0 - 2.0 * (r + 0.5) / h) * tan_half * h / w
    d = np.empty((h, w, 3))
    d[..., 0] = 1.0
    d[..., 1] = -u[None, :]
    d[..., 2] = v[:, None]
    return d


def camera_pose(state_row, mount=None):
    """The camera's own pose row for a camera mounted at (q_m, t_m) in the body frame: position
    p + R(q) t_m and orientation q (x) q_m, so that its rays are R(q) R(q_m) (1, -u, v).  A mount
    quaternion with zero vector part is no rotation."""
    s = np.array(state_row, dtype=np.float64)
    if mount is None:
        return s
    qm = np.asarray(mount[0], dtype=np.float64)
    tm = np.asarray(mount[1], dtype=np.float64)
    rot = quat_to_rot(s[3:7])
    out = s.copy()
    out[0:3] = s[0:3] + rot @ tm
    if np.any(qm[1:4] != 0):
        qb = s[3:7] / np.linalg.norm(s[3:7])
        qm = qm / np.linalg.norm(qm)
        w1, x1, y1, z1 = qb
        w2, x2, y2, z2 = qm
        out[3:7] = [w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                    w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2]
    return out


def camera_rays(state_row, h, w, hfov):
    """Origin [3] and world directions [H,W,3] of one agent's camera at its state row."""
    s = np.asarray(state_row, dtype=np.float64)
    rot = quat_to_rot(s[3:7])
    d = camera_dirs_body(h, w, hfov) @ rot.T
    return s[0:3].copy(), d


def frustum_keep(state_row, verts, tris, h, w, hfov, near, far, margin=1e-3):
    """Triangles that can meet a ray of this view: False only when all three vertices lie outside
    one bounding plane of the view's truncated pyramid, widened by `margin`.

    In camera coordinates X_B = R^T (X - o) a ray t (1, -u, v) reaches exactly the points with
    x_B = t in [near, far], -y_B / x_B = u and z_B / x_B = v; u and v range over the pixel centres.
    A triangle is convex, so if every vertex violates the same half-space no point of it is
    reachable.  The margin (relative, in u, v and t) keeps triangles that pass just outside the
    view, so the near-miss data of boundary rays is unchanged.
    """
    s = np.asarray(state_row, dtype=np.float64)
    rot = quat_to_rot(s[3:7])
    v = np.asarray(verts, dtype=np.float64)
    t = np.asarray(tris, dtype=np.int64)
    xb = (v - s[0:3]) @ rot            # rows: (x_B, y_B, z_B) = R^T (X - o)
    p = xb[t]                          # [T, 3 vertices, 3]
    x, y, z = p[..., 0], p[..., 1], p[..., 2]
    th = np.tan(0.5 * hfov)
    u_max = (1.0 - 1.0 / w) * th + margin
    v_max = (1.0 - 1.0 / h) * th * h / w + margin
    lo, hi = near * (1.0 - margin), far * (1.0 + margin)
    out = ((x < lo).all(1) | (x > hi).all(1)
           | (-y > u_max * x).all(1) | (-y < -u_max * x).all(1)
           | (z > v_max * x).all(1) | (z < -v_max * x).all(1))
    return ~out


def mask_from(out, eps_edge=1e-5, eps_tie=1e-5):
    """Pixels whose closest-hit id is not decided robustly (edges, near misses, ties, clip planes)."""
    t = out["t"]
    scale = np.maximum(1.0, np.where(np.isfinite(t), t, 1.0))
    both = np.isfinite(out["t2"]) & np.isfinite(t)
    gap = np.full(t.shape, np.inf)
    gap[both] = (out["t2"][both] - t[both]) / np.maximum(t[both], 1e-300)
    return ((out["edge_hit"] < eps_edge * scale) | (out["near_miss"] < eps_edge * scale) | (gap < eps_tie)
            | (out["boundary"] != 0))


def render_view(state_row, scene, h=64, w=64, hfov=np.pi / 2, near=0.01, far=100.0, miss_depth=None,
                eps_edge=1e-5, eps_tie=1e-5, with_mask=True, pixels=None, cull=True, mount=None, others=None):
    """Depth [H,W] (or [P] for a pixel subset), triangle id, planar RGB and the comparison mask.

    pixels: optional int array of flat pixel indices (row * W + col) to render only those.
    cull: pre-filter the triangles with frustum_keep() (exact: never changes a result).
    mount: optional camera mount (q_m (w,x,y,z), t_m) in the body frame, see camera_pose().
    others: optional swarm members seen by this camera, a dict with centers [K,3], quats [K,4],
      half [3] (body-box half sizes), rgb [3] and ids [K] (the id each member's pixels get; above
      every triangle index).  A member nearer than the mesh hides it; equal depths keep the mesh.
    """
    miss_depth = far if miss_depth is None else miss_depth
    state_row = camera_pose(state_row, mount)
    o, d = camera_rays(state_row, h, w, hfov)
    d = d.reshape(-1, 3)
    if pixels is not None:
        d = d[np.asarray(pixels)]
    tris_all = np.asarray(scene["tris"])
    keep = np.nonzero(frustum_keep(state_row, scene["verts"], tris_all, h, w, hfov, near, far))[0] if cull \
        else np.arange(tris_all.shape[0])
    out = cast(o, d, scene["verts"], tris_all[keep], near, far, with_mask=with_mask)
    if keep.size:
        out["id"] = np.where(out["id"] >= 0, keep[np.maximum(out["id"], 0)], -1)
    hit = out["id"] >= 0
    rgb = np.zeros((3, d.shape[0]), dtype=np.uint8)
    if "rgb" in scene and scene["rgb"] is not None:
        rgb[:, hit] = np.asarray(scene["rgb"])[out["id"][hit]].T
    swarm_mask = np.zeros(d.shape[0], dtype=bool)
    if others is not None and len(others["centers"]):
        b = cast_boxes(o, d, others["centers"], others["quats"], others["half"], near, far)
        mesh_t = np.where(hit, out["t"], np.inf)
        take = (b["k"] >= 0) & (b["t"] < mesh_t)
        out["t"] = np.where(take, b["t"], out["t"])
        out["id"] = np.where(take, np.asarray(others["ids"])[np.maximum(b["k"], 0)], out["id"])
        rgb[:, take] = np.asarray(others["rgb"], dtype=np.uint8)[:, None]
        hit = hit | take
        scale = np.maximum(1.0, np.where(np.isfinite(b["t"]), b["t"], 1.0))
        both = np.isfinite(b["t"]) & np.isfinite(mesh_t)
        close = np.zeros_like(both)
        close[both] = np.abs(b["t"][both] - mesh_t[both]) < eps_tie * np.maximum(mesh_t[both], 1e-300)
        swarm_mask = ((np.isfinite(b["t"]) & (b["edge"] < eps_edge * scale)) | (b["gap"] < eps_edge * scale) | close
                      | (np.isfinite(b["t"]) & ((np.abs(b["t"] - near) < 1e-6 * scale) |
                                                (np.abs(b["t"] - far) < 1e-6 * scale))))
    depth = np.where(hit, out["t"], miss_depth)
    res = {"depth": depth, "id": out["id"].astype(np.int64), "rgb": rgb, "threads": out["threads"]}
    if with_mask:
        res["mask"] = mask_from(out, eps_edge, eps_tie) | swarm_mask
        res["raw"] = out
    if pixels is None:
        res["depth"] = res["depth"].reshape(h, w)
        res["id"] = res["id"].reshape(h, w)
        res["rgb"] = res["rgb"].reshape(3, h, w)
        if with_mask:
            res["mask"] = res["mask"].reshape(h, w)
    return res
