"""Pins of the FP64 brute-force render oracle (Sec. III-B) against closed forms and exact arithmetic."""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import render as ren
from workloads import scenes
from workloads.agents import yaw_quat


def _state(pos, quat):
    s = np.zeros(17)
    s[0:3] = pos
    s[3:7] = quat
    return s


def _pitch_quat(angle):
    """Rotation about body/world +y by angle (positive pitches the nose down)."""
    return np.array([math.cos(angle / 2), 0.0, math.sin(angle / 2), 0.0])


def test_camera_pitched_down_over_floor_has_constant_planar_depth():
    """P1: image plane parallel to the floor -> every pixel's planar depth equals the height."""
    floor = scenes.floor_quad(half=100.0)
    for h in (0.5, 1.7, 3.25):
        st = _state([0.3, -0.2, h], _pitch_quat(math.pi / 2))
        r = ren.render_view(st, floor, 32, 48, math.radians(90))
        assert np.all(r["id"] >= 0)
        assert np.allclose(r["depth"], h, rtol=1e-13, atol=0)


def test_box_interior_matches_slab_exit_distance():
    """P2: inside an axis-aligned room the closest hit is the slab exit distance min_k (b_k - o_k)/d_k."""
    lo, hi = np.array([0.0, 0.0, 0.0]), np.array([10.0, 8.0, 4.0])
    room = scenes.box_interior(lo, hi, split=2)
    rng = np.random.default_rng(11)
    for _ in range(6):
        q = rng.normal(size=4)
        q /= np.linalg.norm(q)
        o = rng.uniform(lo + 0.5, hi - 0.5)
        st = _state(o, q)
        r = ren.render_view(st, room, 16, 16, math.radians(90))
        _, d = ren.camera_rays(st, 16, 16, math.radians(90))
        d = d.reshape(-1, 3)
        with np.errstate(divide="ignore"):
            exit_t = np.where(d > 0, (hi - o) / d, np.where(d < 0, (lo - o) / d, np.inf)).min(axis=1)
        assert np.all(r["id"].reshape(-1) >= 0)
        assert np.allclose(r["depth"].reshape(-1), exit_t, rtol=1e-12)
        # colour is the flat colour of the face that was hit
        face_rgb = np.asarray(room["rgb"])[r["id"].reshape(-1)].T
        assert np.array_equal(r["rgb"].reshape(3, -1), face_rgb)


def test_tilted_plane_depth_and_pixel_convention():
    """P3: plane n.(X - X0) = 0 seen from an identity pose: t = n.(X0 - o) / n.d for the pixel ray
    d = (1, -u_c, v_r), u_c = (2(c+1/2)/W - 1) tan(hfov/2), v_r = (1 - 2(r+1/2)/H) tan(hfov/2) H/W."""
    o = np.array([0.0, 0.0, 0.0])
    x0 = np.array([6.0, 0.0, 0.0])
    n = np.array([1.0, 0.35, -0.2])
    # a large parallelogram in that plane
    e_u = np.cross(n, [0, 0, 1.0]); e_u = 80 * e_u / np.linalg.norm(e_u)
    e_v = np.cross(n, e_u); e_v = 80 * e_v / np.linalg.norm(e_v)
    plane = scenes.plane_quad(x0 - 0.5 * e_u - 0.5 * e_v, e_u, e_v)
    h, w, hfov = 12, 20, math.radians(75)
    st = _state(o, [1, 0, 0, 0])
    r = ren.render_view(st, plane, h, w, hfov)
    # the plane is stored in float32 in the scene; use its stored vertices for the analytic plane
    # the float32 quad is two triangles whose planes differ by rounding: use the plane of the one hit
    v = np.asarray(plane["verts"], dtype=np.float64)
    tri = np.asarray(plane["tris"])
    th = math.tan(hfov / 2)
    for row in range(h):
        for col in range(w):
            u = (2 * (col + 0.5) / w - 1) * th
            vv = (1 - 2 * (row + 0.5) / h) * th * h / w
            d = np.array([1.0, -u, vv])
            a, b, c = v[tri[r["id"][row, col]]]
            nn = np.cross(b - a, c - a)
            t = nn @ (a - o) / (nn @ d)
            assert math.isclose(r["depth"][row, col], t, rel_tol=1e-11)


def test_image_orientation_left_right_up_down():
    """Image columns run from body +y (left) to -y (right); rows from +z (top) to -z (bottom)."""
    # a wall patch covering only the body-left half-space (y > 0) in front of the camera
    left = scenes.plane_quad([5.0, 0.0, -10.0], [0.0, 20.0, 0.0], [0.0, 0.0, 20.0])
    r = ren.render_view(_state([0, 0, 0], [1, 0, 0, 0]), left, 8, 8, math.radians(90))
    assert np.all(r["id"][:, :4] >= 0) and np.all(r["id"][:, 4:] < 0)
    up = scenes.plane_quad([5.0, -10.0, 0.0], [0.0, 20.0, 0.0], [0.0, 0.0, 20.0])
    r = ren.render_view(_state([0, 0, 0], [1, 0, 0, 0]), up, 8, 8, math.radians(90))
    assert np.all(r["id"][:4, :] >= 0) and np.all(r["id"][4:, :] < 0)
    # a yaw of +90 deg turns the optical axis onto world +y
    wall_y = scenes.plane_quad([-50.0, 7.0, -50.0], [100.0, 0.0, 0.0], [0.0, 0.0, 100.0])
    r = ren.render_view(_state([0, 0, 0], yaw_quat(math.pi / 2)), wall_y, 6, 6, math.radians(90))
    assert np.allclose(r["depth"], 7.0, rtol=1e-12)


def test_field_of_view_edges():
    """A slab of columns at |y/x| <= tan(hfov/2) fills the image edge to edge; one just outside is never seen."""
    hfov = math.radians(60)
    w = 16
    th = math.tan(hfov / 2)
    # vertical strip at x = 4 covering y in [4 th (1 - 1/w) - eps, ...] -> only the leftmost column sees it
    y_edge = 4 * th * (1 - 1 / w)
    strip = scenes.plane_quad([4.0, y_edge - 1e-6, -5.0], [0.0, 1.0, 0.0], [0.0, 0.0, 10.0])
    r = ren.render_view(_state([0, 0, 0], [1, 0, 0, 0]), strip, 4, w, hfov)
    assert np.all(r["id"][:, 0] >= 0) and np.all(r["id"][:, 1:] < 0)
    strip2 = scenes.plane_quad([4.0, y_edge + 1e-6, -5.0], [0.0, 1.0, 0.0], [0.0, 0.0, 10.0])
    r = ren.render_view(_state([0, 0, 0], [1, 0, 0, 0]), strip2, 4, w, hfov)
    assert np.all(r["id"] < 0)


def _ray_sphere(o, d, c, rad):
    oc = o - c
    a = d @ d
    b = 2 * oc @ d
    cc = oc @ oc - rad * rad
    disc = b * b - 4 * a * cc
    if disc < 0:
        return math.inf
    return (-b - math.sqrt(disc)) / (2 * a)


def test_icosphere_depth_between_inscribed_and_circumscribed_spheres():
    """P4: the mesh lies between its inscribed sphere (face planes) and the vertex sphere."""
    sph = scenes.icosphere(radius=2.0, subdiv=2, center=(8.0, 0.5, -0.3))
    v = np.asarray(sph["verts"], dtype=np.float64)
    t = np.asarray(sph["tris"])
    c = np.asarray(sph["center"])
    nrm = np.cross(v[t[:, 1]] - v[t[:, 0]], v[t[:, 2]] - v[t[:, 0]])
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    r_in = np.abs(np.einsum("ij,ij->i", v[t[:, 0]] - c, nrm)).min()
    r_out = np.linalg.norm(v - c, axis=1).max()
    st = _state([0, 0, 0], [1, 0, 0, 0])
    res = ren.render_view(st, sph, 24, 24, math.radians(40))
    o, d = ren.camera_rays(st, 24, 24, math.radians(40))
    d = d.reshape(-1, 3)
    depth = res["depth"].reshape(-1)
    ids = res["id"].reshape(-1)
    n_hit = 0
    for k in range(d.shape[0]):
        t_out, t_in = _ray_sphere(o, d[k], c, r_out), _ray_sphere(o, d[k], c, r_in)
        if math.isfinite(t_in):
            assert ids[k] >= 0
        if not math.isfinite(t_out):
            assert ids[k] < 0
        if ids[k] >= 0:
            n_hit += 1
            assert t_out - 1e-9 <= depth[k] <= (t_in if math.isfinite(t_in) else math.inf) + 1e-9
    assert n_hit > 100


def test_near_far_clip_and_miss_values():
    near_wall = scenes.plane_quad([0.005, -5, -5], [0, 10, 0], [0, 0, 10])      # at t = 0.005 < near
    far_wall = scenes.plane_quad([3.0, -5, -5], [0, 10, 0], [0, 0, 10], rgb=(1, 2, 3))
    both = {"verts": np.concatenate([near_wall["verts"], far_wall["verts"]]),
            "tris": np.concatenate([near_wall["tris"], far_wall["tris"] + 4]),
            "rgb": np.concatenate([near_wall["rgb"], far_wall["rgb"]])}
    r = ren.render_view(_state([0, 0, 0], [1, 0, 0, 0]), both, 4, 4, math.radians(60), near=0.01, far=100.0)
    assert np.allclose(r["depth"], 3.0) and np.all(r["id"] >= 2)
    assert np.all(r["rgb"][:, r["id"] >= 0] == np.array([[1], [2], [3]]))
    r = ren.render_view(_state([0, 0, 0], [1, 0, 0, 0]), both, 4, 4, math.radians(60), near=0.01, far=2.0,
                        miss_depth=-1.0)
    assert np.all(r["depth"] == -1.0) and np.all(r["id"] == -1) and np.all(r["rgb"] == 0)


def test_coplanar_duplicate_goes_to_lower_index_and_is_masked():
    wall = scenes.plane_quad([4.0, -5, -5], [0, 10, 0], [0, 0, 10])
    dup = {"verts": np.concatenate([wall["verts"], wall["verts"]]),
           "tris": np.concatenate([wall["tris"], wall["tris"] + 4]),
           "rgb": np.concatenate([wall["rgb"], wall["rgb"]])}
    r = ren.render_view(_state([0, 0, 0], [1, 0, 0, 0]), dup, 6, 6, math.radians(60))
    assert np.all(r["id"] < 2) and np.all(r["mask"])


def test_ray_parallel_to_triangle_misses():
    tri = {"verts": np.array([[1.0, 0.0, -1.0], [3.0, 0.0, -1.0], [2.0, 0.0, 1.0]], dtype=np.float32),
           "tris": np.array([[0, 1, 2]], dtype=np.int32)}
    out = ren.cast(np.zeros(3), np.array([[1.0, 0.0, 0.0]]), tri["verts"], tri["tris"])
    assert out["id"][0] == -1


# ---------------------------------------------------------------------------
# P10: exact rational arithmetic on tiny scenes
# ---------------------------------------------------------------------------

def _exact_hits(o, d, verts, tris, near, far):
    """All exact (t, index) hits of one ray, in Fraction arithmetic, by the same closed-triangle rule."""
    fo = [Fraction(x) for x in o]
    fd = [Fraction(x) for x in d]
    hits = []
    for k, (a, b, c) in enumerate(tris):
        v0 = [Fraction(float(x)) for x in verts[a]]
        v1 = [Fraction(float(x)) for x in verts[b]]
        v2 = [Fraction(float(x)) for x in verts[c]]
        e1 = [v1[i] - v0[i] for i in range(3)]
        e2 = [v2[i] - v0[i] for i in range(3)]
        # solve o + t d = v0 + u e1 + v e2 by Cramer's rule
        m = [[-fd[i], e1[i], e2[i]] for i in range(3)]
        rhs = [fo[i] - v0[i] for i in range(3)]

        def det3(mm):
            return (mm[0][0] * (mm[1][1] * mm[2][2] - mm[1][2] * mm[2][1])
                    - mm[0][1] * (mm[1][0] * mm[2][2] - mm[1][2] * mm[2][0])
                    + mm[0][2] * (mm[1][0] * mm[2][1] - mm[1][1] * mm[2][0]))
        dm = det3(m)
        if dm == 0:
            continue
        sol = []
        for j in range(3):
            mj = [row[:] for row in m]
            for i in range(3):
                mj[i][j] = rhs[i]
            sol.append(det3(mj) / dm)
        t, u, v = sol
        if u >= 0 and v >= 0 and u + v <= 1 and Fraction(near) <= t <= Fraction(far):
            hits.append((t, k))
    return hits


def _tiny_scene():
    q = Fraction(1, 4)
    pts = []
    tris = []
    # two triangles sharing an edge (a unit square split on its diagonal) at x = 2
    base = len(pts)
    pts += [(2, -1, -1), (2, 1, -1), (2, 1, 1), (2, -1, 1)]
    tris += [(base, base + 1, base + 2), (base, base + 2, base + 3)]
    # coplanar duplicate of the first triangle
    tris += [(base, base + 1, base + 2)]
    # a tilted triangle in front, partly overlapping, with quarter coordinates
    base = len(pts)
    pts += [(1 + q, -q, -q), (1 + 2 * q, 3 * q, -q), (1 + q, q, 3 * q)]
    tris += [(base, base + 1, base + 2)]
    # a T-junction: a triangle whose vertex lies on the shared diagonal, behind the wall plane
    base = len(pts)
    pts += [(3, 0, 0), (3, 2, 0), (3, 0, 2)]
    tris += [(base, base + 1, base + 2)]
    return np.array(pts, dtype=np.float64).astype(np.float32), np.array(tris, dtype=np.int32)


def test_exact_rational_tiny_scene_agrees_off_ties():
    verts, tris = _tiny_scene()
    o = np.array([0.0, 0.0, 0.0])
    rng = np.random.default_rng(3)
    dirs = [np.array([1.0, y, z]) for y, z in rng.uniform(-0.6, 0.6, size=(150, 2))]
    # rays aimed exactly at vertices, along the shared diagonal and at the tilted triangle's edges
    for target in [(2, 1, 1), (2, -1, -1), (2, 0.5, 0.5), (2, 0.25, 0.25), (1.25, 0.0, 0.0), (1.5, 0.75, -0.25),
                   (2, 1, -1), (2, 0, 0)]:
        dirs.append(np.array(target, dtype=np.float64) - o)
    dirs = np.stack(dirs)
    out = ren.cast(o, dirs, verts, tris)
    mask = ren.mask_from(out)
    n_checked = 0
    for k in range(dirs.shape[0]):
        hits = _exact_hits(o, dirs[k], verts, tris, 0.01, 100.0)
        if not hits:
            assert out["id"][k] == -1 or mask[k]
            continue
        t_min = min(h[0] for h in hits)
        tie_set = sorted(i for t, i in hits if t == t_min)
        # the FP64 depth equals the exact depth to rounding
        assert math.isclose(out["t"][k], float(t_min), rel_tol=1e-12)
        # the oracle's id is the lowest of the exact tie set whenever the pixel is not masked
        if not mask[k]:
            assert len(tie_set) == 1 and out["id"][k] == tie_set[0]
            n_checked += 1
        else:
            assert out["id"][k] in tie_set
        # exact ties are always masked
        if len(tie_set) > 1:
            assert mask[k]
    assert n_checked > 60


def test_mask_fraction_small_on_box_room():
    sc = scenes.box_room(seed=1)
    st = _state([5.0, 5.0, 2.0], yaw_quat(0.3))
    r = ren.render_view(st, sc, 64, 64, math.radians(90))
    assert r["mask"].mean() < 0.02
    assert np.all(r["id"] >= 0)


def test_frustum_prefilter_never_changes_a_result():
    """The oracle's view-frustum pre-filter is exact: culled and unculled renders agree bit for bit."""
    rng = np.random.default_rng(17)
    sc = scenes.forest(seed=3, n_trees=120)
    room = scenes.box_room(seed=1)
    for scene, lo, hi in ((sc, [-15, -15, 0.5], [15, 15, 6]), (room, [0.5, 0.5, 0.3], [9.5, 9.5, 3.7])):
        for _ in range(4):
            q = rng.normal(size=4)
            q /= np.linalg.norm(q)
            st = _state(rng.uniform(lo, hi), q)
            for hw, fov in (((24, 24), math.pi / 2), ((9, 20), 1.1)):
                a = ren.render_view(st, scene, hw[0], hw[1], fov, cull=True)
                b = ren.render_view(st, scene, hw[0], hw[1], fov, cull=False)
                assert np.array_equal(a["id"], b["id"]) and np.array_equal(a["depth"], b["depth"])
                assert np.array_equal(a["mask"], b["mask"])


def test_camera_mount_down_facing_with_offset():
    """A level, yawed body with a camera mounted pitched 90 deg down and offset by t_m: the camera
    sits at height z + t_m,z (a level body keeps body z vertical), so every planar depth is z + t_m,z;
    the offset's horizontal part moves the camera without changing any depth."""
    floor = scenes.floor_quad(half=100.0)
    for z, yaw, tm in ((1.5, 0.0, (0.1, 0.0, -0.05)), (2.25, 1.1, (-0.3, 0.2, 0.125))):
        st = _state([0.4, -0.7, z], yaw_quat([yaw])[0])
        r = ren.render_view(st, floor, 24, 32, math.radians(90), mount=(_pitch_quat(math.pi / 2), tm))
        assert np.all(r["id"] >= 0)
        assert np.allclose(r["depth"], z + tm[2], rtol=1e-12, atol=0)


def test_camera_mount_forward_offset_toward_a_wall():
    """A forward camera offset by t_m = (a, b, c) in a body yawed by psi, facing the wall x = L of a
    room: the centre ray leaves p + R_z(psi) t_m along (cos psi, sin psi, 0); at yaw 0 its depth is
    L - p_x - a, and for a camera yawed back by -psi on a body yawed by psi the image is the one of an
    unyawed body at the same camera position."""
    room = scenes.box_interior(np.array([0.0, 0.0, 0.0]), np.array([10.0, 10.0, 4.0]), split=2)
    st = _state([3.0, 5.0, 2.0], [1.0, 0.0, 0.0, 0.0])
    r = ren.render_view(st, room, 2, 2, math.radians(20), mount=((1.0, 0.0, 0.0, 0.0), (0.25, 0.1, -0.2)))
    # the four centre-adjacent pixels all hit the wall x = 10 with planar depth 10 - 3 - 0.25
    assert np.allclose(r["depth"], 10.0 - 3.0 - 0.25, rtol=1e-12)
    psi = 0.7
    body = _state([3.0, 5.0, 2.0], yaw_quat([psi])[0])
    tm = np.array([0.25, 0.1, -0.2])
    mounted = ren.render_view(body, room, 16, 16, math.radians(90), mount=(yaw_quat([-psi])[0], tm))
    c, s_ = math.cos(psi), math.sin(psi)
    cam = np.array([3.0 + c * tm[0] - s_ * tm[1], 5.0 + s_ * tm[0] + c * tm[1], 2.0 + tm[2]])
    plain = ren.render_view(_state(cam, [1.0, 0.0, 0.0, 0.0]), room, 16, 16, math.radians(90))
    assert np.allclose(mounted["depth"], plain["depth"], rtol=1e-12)


def test_box_entry_closed_form_and_orientation():
    """A member box straight ahead at distance D: the centre rays enter its near face at D - h_x; turned
    90 deg about z the near face is the one at h_y.  The entry point lies on the box surface and no
    earlier sample along the ray is inside the box (brute-force march)."""
    half = np.array([0.15, 0.1, 0.05])
    o = np.zeros(3)
    dirs = np.array([[1.0, 0.0, 0.0], [1.0, 0.01, 0.0], [1.0, -0.005, 0.004]])
    for yaw, face in ((0.0, half[0]), (math.pi / 2, half[1])):
        b = ren.cast_boxes(o, dirs, np.array([[4.0, 0.0, 0.0]]), np.array([yaw_quat([yaw])[0]]), half)
        assert np.all(b["k"] == 0)
        assert np.allclose(b["t"], 4.0 - face, rtol=1e-12)
    rng = np.random.default_rng(2)
    centers = rng.uniform(-3, 3, (4, 3))
    quats = rng.normal(size=(4, 4))
    quats /= np.linalg.norm(quats, axis=1, keepdims=True)
    half = np.array([0.8, 0.6, 0.5])
    d = np.concatenate([rng.normal(size=(200, 3)), centers[rng.integers(0, 4, 200)] + rng.normal(0, 0.5, (200, 3))])
    b = ren.cast_boxes(o, d, centers, quats, half, near=0.01, far=100.0)
    assert (b["k"] >= 0).sum() > 0
    for i in np.nonzero(b["k"] >= 0)[0]:
        k = b["k"][i]
        rot = ren.quat_to_rot(quats[k])
        x = (o + b["t"][i] * d[i] - centers[k]) @ rot
        assert abs(np.max(np.abs(x) / half) - 1.0) < 1e-9
    # brute force: march every ray and find the first sample inside any box
    ts = np.linspace(0.01, 10.0, 40001)
    for i in range(0, 400, 7):
        pts = o + ts[:, None] * d[i]
        inside = np.zeros(ts.shape, dtype=bool)
        for k in range(4):
            x = (pts - centers[k]) @ ren.quat_to_rot(quats[k])
            inside |= np.all(np.abs(x) <= half, axis=1)
        if inside.any():
            first = ts[np.argmax(inside)]
            assert b["k"][i] >= 0 and first - 5e-4 <= b["t"][i] <= first
        elif b["k"][i] >= 0:
            assert b["t"][i] > 10.0 or b["edge"][i] < 1e-3 or b["gap"][i] < 1e-3


def test_swarm_members_occlude_and_tie_to_the_mesh():
    """A member between the camera and a wall takes the pixel (its id and colour); a member behind the
    wall is hidden; a camera inside a member's box does not see that box."""
    wall = scenes.plane_quad((6.0, -5.0, -5.0), (0.0, 10.0, 0.0), (0.0, 0.0, 10.0))
    st = _state([0.0, 0.0, 0.0], [1.0, 0.0, 0.0, 0.0])
    half = (0.15, 0.15, 0.05)
    others = {"centers": np.array([[3.0, 0.0, 0.0], [8.0, 0.0, 0.0], [0.0, 0.0, 0.0]]),
              "quats": np.array([[1.0, 0, 0, 0]] * 3), "half": half, "rgb": (10, 20, 30), "ids": [100, 101, 102]}
    r = ren.render_view(st, wall, 9, 9, math.radians(10), others=others)
    c = r["depth"][4, 4]
    assert r["id"][4, 4] == 100 and abs(c - (3.0 - 0.15)) < 1e-12
    assert tuple(r["rgb"][:, 4, 4]) == (10, 20, 30)
    # corner pixels pass beside the member and hit the wall at its planar distance
    assert r["id"][0, 0] in (0, 1) and abs(r["depth"][0, 0] - 6.0) < 1e-12
    assert not np.any(r["id"] == 101) and not np.any(r["id"] == 102)
