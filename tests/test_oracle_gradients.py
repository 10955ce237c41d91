"""Pins of the oracle's finite-difference gradients and nearest-point query against closed forms."""
import math

import numpy as np

from oracle import dynamics as dyn
from oracle import gradients as grd
from oracle import render as ren
from workloads import default_params, scenes
from workloads.agents import make_states


def test_central_difference_is_exact_on_quadratics():
    a = np.array([[2.0, 0.5], [0.5, 1.0]])
    f = lambda x: 0.5 * x @ a @ x + x.sum()
    x = np.array([0.3, -1.2])
    for u in (np.array([1.0, 0.0]), np.array([0.6, 0.8])):
        assert math.isclose(grd.central_difference(f, x, u), (a @ x + 1) @ u, rel_tol=1e-8)


def test_step_jacobian_free_fall():
    """Free fall, no drag: dp'/dp = I, dp'/dv = dt I, dv'/dv = I (RK4 exact on this ODE)."""
    p = default_params(ctrl=dyn.SRT, k_lin=(0.0, 0.0, 0.0))
    s = make_states([[0.0, 0.0, 5.0]], p, vel=[[1.0, -2.0, 0.5]], rotor=[[0, 0, 0, 0]]).astype(np.float64)
    js, ja = grd.step_jacobian(s, np.zeros((1, 4)), p)
    assert np.allclose(js[0, 0:3, 0:3], np.eye(3), atol=1e-8)
    assert np.allclose(js[0, 0:3, 7:10], p["dt"] * np.eye(3), atol=1e-8)
    assert np.allclose(js[0, 7:10, 7:10], np.eye(3), atol=1e-8)
    assert np.allclose(js[0, 0:3, 3:7], 0.0, atol=1e-8)


def test_step_jacobian_linear_drag_velocity_block():
    """Isotropic linear drag: dv'/dv = P(-k dt / m) I with P the RK4 Taylor polynomial."""
    k = 0.1
    p = default_params(ctrl=dyn.SRT, k_lin=(k, k, k))
    s = make_states([[0.0, 0.0, 5.0]], p, vel=[[1.0, -2.0, 0.5]], rotor=[[0, 0, 0, 0]]).astype(np.float64)
    js, _ = grd.step_jacobian(s, np.zeros((1, 4)), p)
    z = -k * p["dt"] / p["mass"]
    amp = 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24
    assert np.allclose(js[0, 7:10, 7:10], amp * np.eye(3), atol=1e-8)


def test_depth_gradient_over_floor_closed_form():
    """Camera at height h pitched down by phi over z = 0: t = h / (sin phi - v cos phi) for the pixel ray."""
    floor = scenes.floor_quad(half=200.0)
    phi, h = 0.6, 2.0
    view = {"H": 8, "W": 8, "hfov": math.radians(90), "near": 0.01, "far": 100.0}
    s = np.zeros(17)
    s[0:3] = [0.4, -0.3, h]
    s[3:7] = [math.cos(phi / 2), 0.0, math.sin(phi / 2), 0.0]
    pixels = np.array([5 * 8 + 2, 7 * 8 + 6, 4 * 8 + 4])
    g = grd.depth_pose_gradient(s, floor, view, pixels)
    th = math.tan(view["hfov"] / 2)
    dq = 0.5 * np.array([-math.sin(phi / 2), 0.0, math.cos(phi / 2), 0.0])
    for k, pix in enumerate(pixels):
        r = pix // 8
        v = (1 - 2 * (r + 0.5) / 8) * th
        den = math.sin(phi) - v * math.cos(phi)
        assert abs(g[k, 0]) < 1e-7 and abs(g[k, 1]) < 1e-7
        assert math.isclose(g[k, 2], 1.0 / den, rel_tol=1e-7)
        assert math.isclose(g[k, 3:7] @ dq, -h * (math.cos(phi) + v * math.sin(phi)) / den ** 2, rel_tol=1e-6)
        # depth is invariant to the scale of q (the camera uses the normalised quaternion)
        assert abs(g[k, 3:7] @ s[3:7]) < 1e-6


def test_rollout_goal_term_gradient_closed_form():
    """With nothing in view the loss is the goal term only: dL/dp0 . u = sum_k 2 w (p_k - g) . u in free fall."""
    p = default_params(ctrl=dyn.SRT, k_lin=(0.0, 0.0, 0.0))
    far_tri = scenes.plane_quad([-50.0, 0.0, 0.0], [0.0, 0.1, 0.0], [0.0, 0.0, 0.1])   # behind the camera
    view = {"H": 4, "W": 4, "hfov": math.radians(90), "near": 0.01, "far": 100.0}
    s0 = make_states([[0.0, 0.0, 5.0]], p, vel=[[1.0, 0.0, 0.0]], rotor=[[0, 0, 0, 0]]).astype(np.float64)
    acts = np.zeros((5, 1, 4))
    goal = np.array([[3.0, 1.0, 4.0]])
    u_s = np.zeros_like(s0)
    u_s[0, 0:3] = [0.6, 0.0, 0.8]
    d, smooth, corr, nj = grd.rollout_directional(s0, acts, p, far_tri, goal, view, u_s, np.zeros_like(acts))
    assert smooth and nj == 0 and corr == d
    traj = dyn.rollout(s0, acts, p)
    expect = sum(2 * 0.01 * (traj[k, 0, 0:3] - goal[0]) @ u_s[0, 0:3] for k in range(1, 6))
    assert math.isclose(d, expect, rel_tol=1e-6)


def test_closest_point_closed_forms():
    """Nearest-obstacle distance (Sec. III-B spatial distance module): plane, edge and corner regions of a box."""
    v, t = scenes.boxes_mesh(np.array([[0.0, 0.0, 0.0]]), np.array([[2.0, 1.0, 3.0]]))
    pts = np.array([[1.0, 0.5, 4.0],      # above the top face: distance 1
                    [3.0, 2.0, 1.5],      # beside the vertical edge x=2,y=1: distance sqrt(2)
                    [-1.0, -1.0, -1.0],   # corner (0,0,0): sqrt(3)
                    [1.0, 0.5, 1.5]])     # inside: distance to the nearest face (y=0 or y=1): 0.5
    dist, pt, ids = ren.closest_points(pts, v, t)
    assert np.allclose(dist, [1.0, math.sqrt(2), math.sqrt(3), 0.5], atol=1e-14)
    assert np.allclose(pt[0], [1.0, 0.5, 3.0]) and np.allclose(pt[2], [0.0, 0.0, 0.0])
    assert np.all(ids >= 0)


def test_golden_box_room_regression():
    """The oracle reproduces its committed box-room fixture (guards against silent oracle edits)."""
    import json
    import os
    from oracle import render as ren2
    from workloads import agents, scenes as sc_mod
    with open(os.path.join(os.path.dirname(__file__), "golden", "box_room_oracle.json")) as f:
        gold = json.load(f)
    p = default_params()
    traj = dyn.rollout(agents.box_room_start(p), agents.random_actions(2, 100, 1, p), p)
    for k, row in gold["states"].items():
        assert np.allclose(traj[int(k), 0], row, rtol=0, atol=1e-12)
    r = ren2.render_view(traj[100, 0], sc_mod.box_room(seed=1), 64, 64, math.pi / 2,
                         pixels=np.array(gold["pixels"]))
    assert np.allclose(r["depth"], gold["depth"], rtol=1e-13)
    assert r["id"].tolist() == gold["id"]


def test_directional_derivative_flags_silhouette_jumps():
    """A perturbation that moves a wall edge across pixel rays makes the depth jump: flagged non-smooth."""
    p = default_params(ctrl=dyn.SRT, k_lin=(0.0, 0.0, 0.0))
    wall = scenes.plane_quad([5.0, -3.0, -3.0], [0.0, 3.0, 0.0], [0.0, 0.0, 13.0])   # y in [-3, 0], z in [-3, 10]
    back = scenes.plane_quad([9.0, -50.0, -50.0], [0.0, 100.0, 0.0], [0.0, 0.0, 100.0])
    sc = {"verts": np.concatenate([wall["verts"], back["verts"]]), "tris": np.concatenate([wall["tris"], back["tris"] + 4]),
          "rgb": np.concatenate([wall["rgb"], back["rgb"]])}
    view = {"H": 2, "W": 64, "hfov": math.radians(90), "near": 0.01, "far": 100.0}
    s0 = make_states([[0.0, 0.0, 5.0]], p, rotor=[[0, 0, 0, 0]]).astype(np.float64)
    acts = np.zeros((1, 1, 4))
    # the pixel column just right of the image centre sees the wall edge at y = 0 within ~1e-9 m
    u_s = np.zeros_like(s0)
    u_s[0, 1] = 1.0
    col = 32
    th = math.tan(view["hfov"] / 2)
    u = (2 * (col + 0.5) / 64 - 1) * th
    s0[0, 1] = u * 5.0 + 1e-9          # the ray meets the wall plane at y = s0_y - u * 5: the edge y = 0 is within +-h
    d, smooth, corr, nj = grd.rollout_directional(s0, acts, p, sc, np.zeros((1, 3)), view, u_s, np.zeros_like(acts),
                                                  w_goal=0.0)
    assert not smooth and abs(d) > 1.0 and nj == 2          # the edge column, in both image rows
    # with the jumped pixel removed, the rest of the image is a wall/backdrop seen head-on while the
    # camera moves sideways: depth is unchanged, so the corrected derivative vanishes
    assert abs(corr) < 1e-6


def _split_wall(x, y0):
    """A wall x = const made of two large triangles that share the vertical edge y = y0 (the other edges
    far outside a 90-degree view from near the origin)."""
    verts = np.array([[x, y0, -1000.0], [x, y0, 1000.0], [x, 2000.0, 0.0], [x, -2000.0, 0.0]])
    return {"verts": verts, "tris": np.array([[0, 1, 2], [0, 1, 3]]), "rgb": np.array([[200, 0, 0], [0, 200, 0]],
                                                                                      dtype=np.uint8)}


def test_edge_mask_flags_the_column_on_a_shared_edge():
    """Column 40's rays meet the wall at y = -5 u_40 exactly on the edge the two triangles share: that column
    is flagged in every row and step, no other pixel is (the next columns are 5/32 m away), and the
    columns either side hit different triangles."""
    p = default_params(ctrl=dyn.SRT, k_lin=(0.0, 0.0, 0.0))
    view = {"H": 4, "W": 64, "hfov": math.radians(90), "near": 0.01, "far": 100.0}
    u40 = 2 * (40 + 0.5) / 64 - 1
    sc = _split_wall(5.0, -5.0 * u40)
    s0 = make_states([[0.0, 0.0, 5.0]], p, rotor=[[0, 0, 0, 0]]).astype(np.float64)
    acts = np.zeros((2, 1, 4))                       # free fall: the camera keeps y = 0 and its attitude
    m = grd.rollout_edge_mask(s0, acts, p, sc, view, eps_edge=1e-4)
    assert m.shape == (2, 1, 4 * 64)
    expect = np.zeros((4, 64), dtype=bool)
    expect[:, 40] = True
    for k in range(2):
        assert np.array_equal(m[k, 0].reshape(4, 64), expect)
    ids = ren.render_view(dyn.rollout(s0, acts, p)[1, 0], sc, 4, 64, view["hfov"], with_mask=False)["id"]
    assert set(ids[:, 39]) != set(ids[:, 41])


def test_directional_derivative_removes_listed_pixel_steps():
    """Removing every pixel-step leaves the goal term alone: moving toward the wall changes every depth,
    yet the corrected derivative equals the goal term's closed form, sum_k 2 w (p_k - g) . u."""
    p = default_params(ctrl=dyn.SRT, k_lin=(0.0, 0.0, 0.0))
    view = {"H": 4, "W": 8, "hfov": math.radians(90), "near": 0.01, "far": 100.0}
    sc = _split_wall(5.0, 0.3)
    s0 = make_states([[0.0, 0.0, 5.0]], p, rotor=[[0, 0, 0, 0]]).astype(np.float64)
    acts = np.zeros((3, 1, 4))
    goal = np.array([[3.0, 1.0, 4.0]])
    u_s = np.zeros_like(s0)
    u_s[0, 0] = 1.0
    everything = np.ones((3, 1, 32), dtype=bool)
    d, smooth, corr, nj = grd.rollout_directional(s0, acts, p, sc, goal, view, u_s, np.zeros_like(acts),
                                                  remove=everything)
    traj = dyn.rollout(s0, acts, p)
    goal_only = sum(2 * 0.01 * (traj[k, 0, 0:3] - goal[0]) @ u_s[0, 0:3] for k in range(1, 4))
    assert nj == 96 and not smooth
    assert abs(d - goal_only) > 1e-3                  # the depth terms do change
    assert math.isclose(corr, goal_only, rel_tol=1e-6)
