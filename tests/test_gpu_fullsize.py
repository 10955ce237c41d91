"""Parity at full benchmark sizes, in the launch configuration the benchmark times.

The oracle cannot brute-force every frame of a full batch, so these tests
sample outputs it can compute one by one: after running the benchmark's own
workloads through vf_step (default launch form: split with spatial order), a
seeded sample of pixels of a seeded sample of agents is rendered by the oracle
at the GPU's float32 poses and compared element by element (ids and colours
bit-exact off the edge/tie mask, depth within 1e-4), and every agent's last
step is checked against the oracle stepped from the GPU's previous state.
Also the largest image (1,024 x 1,024) and the degenerate 1 x 1,024 strips.
"""
import math

import numpy as np
import pytest
import torch

from oracle import dynamics as odyn
from oracle import render as oren
from workloads import agents, default_params, device_params, scenes
from tests.gpu_util import compare_render, header, state_close

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vf():
    from paper_2407_14783_amd import sim
    ctx = sim.Context(0)
    yield sim, ctx
    ctx.close()


def _sampled_check(scene, state_row, depth, ids, rgb, off, hw, pixels, label):
    h, w = hw
    ref = oren.render_view(state_row.astype(np.float64), scene, h, w, math.pi / 2, pixels=pixels)
    rgb_px = None
    if rgb is not None:
        rgb_px = np.stack([rgb[3 * off + c * h * w + pixels] for c in range(3)])
    return compare_render(depth[off + pixels], ids[off + pixels], rgb_px, ref, 100.0, label)


def test_forest256_benchmark_configuration_sampled(vf):
    sim, ctx = vf
    p = default_params()
    sc = scenes.forest(seed=3)
    sid = ctx.build_scene(sc["verts"], sc["tris"], sc["rgb"])
    n, steps = 256, 10
    s0 = agents.forest_starts(4, n, sc, p)
    acts = agents.random_actions(5, 200, n, p)
    views, npx, offs, mh, mw = sim.make_views(n, sid, (64, 64))
    state = torch.as_tensor(s0).cuda()
    depth = torch.empty(npx).cuda()
    ids = torch.empty(npx, dtype=torch.int32).cuda()
    rgb = torch.empty(3 * npx, dtype=torch.uint8).cuda()
    header(f"full size: forest-256, {steps} steps, sampled pixels")
    for k in range(steps):
        prev = state.cpu().numpy()
        ctx.step(p, state, torch.as_tensor(acts[k]).cuda(), views=views, max_hw=(mh, mw), depth=depth,
                 tri_id=ids, rgb=rgb, out_pixels=npx)
    ctx.sync_check()
    s1 = state.cpu().numpy()
    ref = odyn.step(prev.astype(np.float64), acts[steps - 1], device_params(p))
    assert state_close(s1, ref) <= 1e-5
    d, i, c = depth.cpu().numpy(), ids.cpu().numpy(), rgb.cpu().numpy()
    rng = np.random.default_rng(21)
    masked = []
    for a in rng.choice(n, 12, replace=False):
        px = rng.choice(4096, 160, replace=False)
        masked.append(_sampled_check(sc, s1[a], d, i, c, offs[a], (64, 64), px, f"agent {a}"))
    assert np.mean(masked) < 0.02
    ctx.free_scene(sid)


def test_multi_scene_4096_sampled(vf):
    """The multi-scene benchmark batch: 4,096 agents over 8 room graphs (20k to 2M triangles), half
    64x64, half 128x128, in one launch."""
    sim, ctx = vf
    p = default_params()
    from paper_2407_14783_amd.serving import ROOM_LEAF_SIZE
    scs = scenes.multi_scene_set(seed=6)
    ctx.set_bvh_leaf_size(ROOM_LEAF_SIZE)          # as the benchmark builds the room graphs
    sids = [ctx.build_scene(s["verts"], s["tris"], s["rgb"]) for s in scs]
    ctx.set_bvh_leaf_size(4)
    counts = agents.multi_scene_split(6, 4096, 8)
    st = np.concatenate([agents.room_graph_starts(60 + j, int(c), scs[j], p) for j, c in enumerate(counts)])
    scene_of = np.repeat(np.arange(8), counts)
    big = np.random.default_rng(6).permutation(4096) < 2048
    hw = np.where(big, 128, 64)
    views, npx, offs, mh, mw = sim.make_views(4096, np.asarray(sids)[scene_of], np.stack([hw, hw], 1))
    state = torch.as_tensor(st).cuda()
    acts = agents.random_actions(6, 2, 4096, p)
    depth = torch.empty(npx).cuda()
    ids = torch.empty(npx, dtype=torch.int32).cuda()
    header("full size: multi-scene 4,096 agents, sampled pixels")
    for k in range(2):
        prev = state.cpu().numpy()
        ctx.step(p, state, torch.as_tensor(acts[k]).cuda(), views=views, max_hw=(mh, mw), depth=depth,
                 tri_id=ids, out_pixels=npx)
    ctx.sync_check()
    s1 = state.cpu().numpy()
    assert state_close(s1, odyn.step(prev.astype(np.float64), acts[1], device_params(p))) <= 1e-5
    d, i = depth.cpu().numpy(), ids.cpu().numpy()
    rng = np.random.default_rng(22)
    masked = []
    for j in range(8):                       # two agents of every scene
        for a in rng.choice(np.nonzero(scene_of == j)[0], 2, replace=False):
            h = int(hw[a])
            px = rng.choice(h * h, 24, replace=False)
            masked.append(_sampled_check(scs[j], s1[a], d, i, None, offs[a], (h, h), px, f"scene {j} agent {a}"))
    assert np.mean(masked) < 0.05
    for s in sids:
        ctx.free_scene(s)


def test_largest_and_degenerate_images(vf):
    sim, ctx = vf
    p = default_params()
    sc = scenes.box_room(seed=1)
    sid = ctx.build_scene(sc["verts"], sc["tris"], sc["rgb"])
    rng = np.random.default_rng(23)
    q = rng.normal(size=(3, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    states = agents.make_states(rng.uniform([2, 2, 1], [8, 8, 3], (3, 3)), p, quat=q)
    hws = np.array([(1024, 1024), (1, 1024), (1024, 1)])
    views, npx, offs, mh, mw = sim.make_views(3, sid, hws)
    depth = torch.empty(npx).cuda()
    ids = torch.empty(npx, dtype=torch.int32).cuda()
    rgb = torch.empty(3 * npx, dtype=torch.uint8).cuda()
    header("full size: 1024x1024 and 1x1024 / 1024x1 images")
    ctx.render(torch.as_tensor(states).cuda(), views, max_hw=(mh, mw), depth=depth, tri_id=ids, rgb=rgb,
               out_pixels=npx)
    ctx.sync_check()
    d, i, c = depth.cpu().numpy(), ids.cpu().numpy(), rgb.cpu().numpy()
    for a in range(3):
        h, w = hws[a]
        px = rng.choice(h * w, min(h * w, 1500), replace=False)
        # the tile grid's last row and column, where a ragged edge would show
        px = np.unique(np.concatenate([px, [h * w - 1, w - 1, (h - 1) * w]]))
        _sampled_check(sc, states[a], d, i, c, offs[a], (h, w), px, f"{h}x{w}")
    ctx.free_scene(sid)
