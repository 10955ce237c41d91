"""Camera rigs (several mounted cameras per agent) on the device against the oracle.

Each view carries a camera mount (orientation and offset in the body frame); a
rig is several views whose env_idx entries name the same state slot.  Images
are compared with the oracle's brute-force render of the mounted camera
(ids and colours bit-exact off the edge/tie mask, depth within 1e-4), and the
depth adjoint of a mounted camera with central differences of the oracle.
"""
import math

import numpy as np
import pytest
import torch

from oracle import gradients as ograd
from oracle import render as oren
from workloads import agents, default_params, scenes
from tests.gpu_util import compare_render, header

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vf():
    from paper_2407_14783_amd import sim
    ctx = sim.Context(0)
    yield sim, ctx
    ctx.close()


def _pitch(angle):
    return np.array([math.cos(angle / 2), 0.0, math.sin(angle / 2), 0.0])


# front camera 10 cm ahead and 3 cm up; a down-facing camera; a rear camera turned 180 deg about z
RIG = [((1.0, 0.0, 0.0, 0.0), (0.10, 0.0, 0.03), (40, 56)),
       (tuple(_pitch(math.pi / 2)), (0.0, 0.02, -0.04), (24, 24)),
       ((0.0, 0.0, 0.0, 1.0), (-0.08, 0.0, 0.0), (33, 17))]


def _rig_views(sim, n, sid):
    k = len(RIG)
    qs = np.array([RIG[j % k][0] for j in range(n * k)], dtype=np.float32)
    ts = np.array([RIG[j % k][1] for j in range(n * k)], dtype=np.float32)
    hw = np.array([RIG[j % k][2] for j in range(n * k)])
    return sim.make_views(n * k, sid, hw, mount_q=qs, mount_t=ts), qs, ts, hw


def test_rig_render_matches_oracle(vf):
    sim, ctx = vf
    p = default_params()
    sc = scenes.box_room(seed=1)
    sid = ctx.build_scene(sc["verts"], sc["tris"], sc["rgb"])
    rng = np.random.default_rng(21)
    n = 5
    q = rng.normal(size=(n, 4))
    q[:, 1:3] *= 0.3                     # mostly upright bodies
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    st = agents.make_states(rng.uniform([1.5, 1.5, 1.0], [8.5, 8.5, 3.0], (n, 3)), p, quat=q)
    (views, npx, offs, mh, mw), qs, ts, hw = _rig_views(sim, n, sid)
    k = len(RIG)
    env = torch.as_tensor(np.repeat(np.arange(n), k).astype(np.int32)).cuda()
    depth = torch.empty(npx).cuda()
    ids = torch.empty(npx, dtype=torch.int32).cuda()
    rgb = torch.empty(3 * npx, dtype=torch.uint8).cuda()
    header(f"rig render: {n} agents x {k} mounted cameras")
    ctx.render(torch.as_tensor(st).cuda(), views, n=n * k, env_idx=env, max_hw=(mh, mw), depth=depth, tri_id=ids,
               rgb=rgb, out_pixels=npx)
    ctx.sync_check()
    depth, ids, rgb = depth.cpu().numpy(), ids.cpu().numpy(), rgb.cpu().numpy()
    masked = []
    for j in range(n * k):
        h, w = hw[j]
        a = j // k
        ref = oren.render_view(st[a].astype(np.float64), sc, h, w, math.pi / 2,
                               mount=(qs[j].astype(np.float64), ts[j].astype(np.float64)))
        sl = slice(offs[j], offs[j] + h * w)
        masked.append(compare_render(depth[sl], ids[sl], rgb[3 * offs[j]:3 * offs[j] + 3 * h * w], ref, 100.0,
                                     label=f"view {j}"))
    assert np.mean(masked) < 0.02
    # the down-facing camera of a level agent sees the floor below it
    ctx.free_scene(sid)


def test_step_with_mounted_views_fused_and_split(vf):
    """vf_step renders the mounted camera at the new state, the same in both launch forms."""
    sim, ctx = vf
    p = default_params()
    sc = scenes.box_room(seed=1)
    sid = ctx.build_scene(sc["verts"], sc["tris"], sc["rgb"])
    n = 3
    s0 = agents.make_states(np.array([[3.0, 4.0, 2.0], [6.0, 6.0, 1.5], [5.0, 2.5, 2.5]]), p,
                            quat=agents.yaw_quat([0.3, -1.0, 2.0]))
    acts = agents.random_actions(3, 1, n, p)[0]
    views, npx, offs, mh, mw = sim.make_views(n, sid, (20, 28), mount_q=RIG[1][0], mount_t=RIG[1][1])
    outs = []
    for fused in (True, False):
        ctx.set_launch_mode(fused)
        st = torch.as_tensor(s0).cuda()
        depth = torch.empty(npx).cuda()
        ids = torch.empty(npx, dtype=torch.int32).cuda()
        ctx.step(p, st, torch.as_tensor(acts).cuda(), views=views, max_hw=(mh, mw), depth=depth, tri_id=ids,
                 out_pixels=npx)
        ctx.sync_check()
        outs.append((st.cpu().numpy(), depth.cpu().numpy(), ids.cpu().numpy()))
    ctx.set_launch_mode(None)
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1]) and np.array_equal(outs[0][2], outs[1][2])
    s1 = outs[0][0]
    for i in range(n):
        ref = oren.render_view(s1[i].astype(np.float64), sc, 20, 28, math.pi / 2,
                               mount=(np.array(RIG[1][0], dtype=np.float32).astype(np.float64),
                                      np.array(RIG[1][1], dtype=np.float32).astype(np.float64)))
        sl = slice(offs[i], offs[i] + 560)
        compare_render(outs[0][1][sl], outs[0][2][sl], None, ref, 100.0, label=f"agent {i}")
    ctx.free_scene(sid)


def test_render_backward_with_mount_matches_fd(vf):
    sim, ctx = vf
    p = default_params()
    sc = scenes.box_room(seed=1)
    sid = ctx.build_scene(sc["verts"], sc["tris"], sc["rgb"])
    rng = np.random.default_rng(33)
    n, h, w = 3, 12, 12
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    st = agents.make_states(rng.uniform([2, 2, 1], [8, 8, 3], size=(n, 3)), p, quat=q)
    mq = np.array([_pitch(0.6), (1.0, 0.0, 0.0, 0.0), (0.0, 0.0, 0.0, 1.0)], dtype=np.float32)
    mq /= np.linalg.norm(mq, axis=1, keepdims=True)
    mt = np.array([(0.12, -0.05, 0.04), (0.3, 0.2, -0.1), (-0.1, 0.0, 0.05)], dtype=np.float32)
    views, npx, offs, mh, mw = sim.make_views(n, sid, (h, w), mount_q=mq, mount_t=mt)
    ids = torch.zeros(npx, dtype=torch.int32).cuda()
    depth = torch.zeros(npx).cuda()
    ctx.render(torch.as_tensor(st).cuda(), views, max_hw=(mh, mw), depth=depth, tri_id=ids, out_pixels=npx)
    g = rng.normal(size=npx).astype(np.float32)
    for i in range(n):
        ref = oren.render_view(st[i].astype(np.float64), sc, h, w, math.pi / 2, eps_edge=1e-3,
                               mount=(mq[i].astype(np.float64), mt[i].astype(np.float64)))
        g[offs[i]:offs[i] + h * w][ref["mask"].reshape(-1)] = 0.0
    grad_state = torch.zeros((n, 17)).cuda()
    header("render_backward with mounted cameras")
    ctx.render_backward(torch.as_tensor(st).cuda(), views, (mh, mw), ids, torch.as_tensor(g).cuda(), npx,
                        grad_state)
    ctx.sync_check()
    got = grad_state.cpu().numpy()
    for i in range(n):
        view = {"H": h, "W": w, "hfov": math.pi / 2, "near": 0.01, "far": 100.0,
                "mount": (mq[i].astype(np.float64), mt[i].astype(np.float64))}
        fd = ograd.depth_pose_gradient(st[i].astype(np.float64), sc, view, np.arange(h * w))
        expect = g[offs[i]:offs[i] + h * w].astype(np.float64) @ fd
        rel = np.linalg.norm(got[i, 0:7] - expect) / max(np.linalg.norm(expect), 1e-12)
        assert rel <= 1e-3, f"view {i}: rel err {rel:.2e}"
    ctx.free_scene(sid)
