"""Swarm mode on the device against the oracle (the swarm example of Sec. IV).

Agents of a swarm see the other members as boxes turned with their attitude
(ids past the mesh's triangle count, one flat colour); images are compared with
the oracle's brute-force render of mesh plus member boxes (ids and colours
bit-exact off the edge/tie mask, depth within 1e-4).  The collision check
reports the nearer of the mesh and the other members' bounding spheres.
"""
import math

import numpy as np
import pytest
import torch

from oracle import dynamics as odyn
from oracle import render as oren
from workloads import agents, default_params, device_params, scenes
from tests.gpu_util import compare_render, header, record

pytestmark = pytest.mark.gpu

HALF = (0.3, 0.25, 0.1)
RGB = (250, 40, 10)


@pytest.fixture(scope="module")
def vf():
    from paper_2407_14783_amd import sim
    ctx = sim.Context(0)
    yield sim, ctx
    ctx.set_swarms([])
    ctx.close()


def _swarm_states(p, rng, n):
    """n agents within a few metres of each other in the box room, random attitudes near level."""
    q = rng.normal(size=(n, 4))
    q[:, 1:3] *= 0.2
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    pos = np.array([4.0, 5.0, 2.0]) + rng.uniform(-1.5, 1.5, (n, 3)) * np.array([1.0, 1.0, 0.5])
    return agents.make_states(pos, p, quat=q)


def _others(states, members, self_slot, n_tris):
    idx = [j for j, m in enumerate(members) if m != self_slot]
    return {"centers": states[[members[j] for j in idx], 0:3].astype(np.float64),
            "quats": states[[members[j] for j in idx], 3:7].astype(np.float64),
            "half": np.asarray(HALF, dtype=np.float32).astype(np.float64), "rgb": RGB,
            "ids": [n_tris + j for j in idx]}


def test_swarm_render_matches_oracle(vf):
    sim, ctx = vf
    p = default_params()
    sc = scenes.box_room(seed=1)
    sid = ctx.build_scene(sc["verts"], sc["tris"], sc["rgb"])
    n_tris = sc["tris"].shape[0]
    rng = np.random.default_rng(41)
    n = 8
    st = _swarm_states(p, rng, n)
    # two swarms over the slots; slot 7 flies alone
    groups = [[0, 2, 4, 6], [5, 1, 3]]
    ctx.set_swarms(groups, half_extent=HALF, rgb=RGB)
    swarm_of = {m: g for g, mem in enumerate(groups) for m in mem}
    sw = np.array([swarm_of.get(i, -1) for i in range(n)])
    views, npx, offs, mh, mw = sim.make_views(n, sid, (48, 48), swarm=sw)
    depth = torch.empty(npx).cuda()
    ids = torch.empty(npx, dtype=torch.int32).cuda()
    rgb = torch.empty(3 * npx, dtype=torch.uint8).cuda()
    header("swarm render: 8 agents, swarms of 4 and 3")
    ctx.render(torch.as_tensor(st).cuda(), views, max_hw=(mh, mw), depth=depth, tri_id=ids, rgb=rgb,
               out_pixels=npx)
    ctx.sync_check()
    depth, ids, rgb = depth.cpu().numpy(), ids.cpu().numpy(), rgb.cpu().numpy()
    seen = 0
    for i in range(n):
        others = _others(st, groups[sw[i]], i, n_tris) if sw[i] >= 0 else None
        ref = oren.render_view(st[i].astype(np.float64), sc, 48, 48, math.pi / 2, others=others)
        sl = slice(offs[i], offs[i] + 48 * 48)
        masked = compare_render(depth[sl], ids[sl], rgb[3 * offs[i]:3 * offs[i] + 3 * 48 * 48], ref, 100.0,
                                label=f"agent {i}")
        assert masked < 0.05
        seen += int((ids[sl] >= n_tris).sum())
        if sw[i] < 0:
            assert not np.any(ids[sl] >= n_tris)
    assert seen > 0, "no agent saw a swarm member"
    # segmentation labels member pixels -2 - j
    seg = ctx.segmentation(views, n, (mh, mw), torch.as_tensor(ids).cuda(), npx).cpu().numpy()
    ctx.sync_check()
    assert np.array_equal(seg, np.where(ids >= n_tris, -2 - (ids - n_tris), np.where(ids >= 0, ids, -1)))
    ctx.set_swarms([])
    ctx.free_scene(sid)


def test_swarm_step_and_collision(vf):
    """vf_step with swarms renders every member at its new state (split launch), and the collision
    check takes the nearer of the mesh and the members' bounding spheres."""
    sim, ctx = vf
    p = default_params()
    sc = scenes.box_room(seed=1)
    sid = ctx.build_scene(sc["verts"], sc["tris"], sc["rgb"])
    n_tris = sc["tris"].shape[0]
    rng = np.random.default_rng(42)
    n = 5
    st0 = _swarm_states(p, rng, n)
    groups = [list(range(n))]
    ctx.set_swarms(groups, half_extent=HALF, rgb=RGB)
    views, npx, offs, mh, mw = sim.make_views(n, sid, (32, 40), swarm=0)
    acts = agents.random_actions(7, 1, n, p)[0]
    st = torch.as_tensor(st0).cuda()
    ctx.set_launch_mode(True)          # asks for the fused form; swarms force the split one
    depth = torch.empty(npx).cuda()
    ids = torch.empty(npx, dtype=torch.int32).cuda()
    ctx.step(p, st, torch.as_tensor(acts).cuda(), views=views, max_hw=(mh, mw), depth=depth, tri_id=ids,
             out_pixels=npx)
    ctx.sync_check()
    ctx.set_launch_mode(None)
    s1 = st.cpu().numpy()
    ref_s1 = odyn.step(st0, acts, device_params(p))
    assert np.abs(s1 - ref_s1).max() < 1e-5
    depth, ids = depth.cpu().numpy(), ids.cpu().numpy()
    for i in range(n):
        ref = oren.render_view(s1[i].astype(np.float64), sc, 32, 40, math.pi / 2,
                               others=_others(s1, groups[0], i, n_tris))
        sl = slice(offs[i], offs[i] + 32 * 40)
        compare_render(depth[sl], ids[sl], None, ref, 100.0, label=f"agent {i}")
    radius = 0.5
    rel = torch.empty((n, 3)).cuda()
    col = torch.empty(n, dtype=torch.uint8).cuda()
    d = ctx.collision(torch.as_tensor(s1).cuda(), views, radius, rel=rel, collided=col)
    ctx.sync_check()
    d, rel, col = d.cpu().numpy(), rel.cpu().numpy(), col.cpu().numpy()
    r_b = float(np.linalg.norm(np.asarray(HALF, dtype=np.float32)))
    for i in range(n):
        pos = s1[i, 0:3].astype(np.float64)
        mesh, pt, _ = oren.closest_points(pos[None], sc["verts"], sc["tris"])
        cen = np.linalg.norm(s1[:, 0:3].astype(np.float64) - pos, axis=1)
        cen[i] = np.inf
        expect = min(mesh[0], cen.min() - r_b)
        assert abs(d[i] - expect) <= 2e-5 * max(1.0, abs(expect))
        assert abs(np.linalg.norm(rel[i]) - abs(expect)) <= 1e-4
        if abs(expect - radius) > 1e-4:
            assert col[i] == (expect <= radius)
    ctx.set_swarms([])
    ctx.free_scene(sid)


def _swarm_of_100(p, rng, n=100):
    """n drones on a jittered 5 x 5 x 4 lattice in the box room, attitudes near level."""
    g = np.stack(np.meshgrid(np.arange(5), np.arange(5), np.arange(4), indexing="ij"), -1).reshape(-1, 3)[:n]
    pos = np.array([2.0, 2.0, 0.8]) + g * np.array([1.5, 1.5, 0.8]) + rng.uniform(-0.3, 0.3, (n, 3))
    q = rng.normal(size=(n, 4))
    q[:, 1:4] *= 0.3
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return agents.make_states(pos, p, quat=q)


def test_swarm_of_100_through_the_tree(vf):
    """A swarm of 100 members (the paper's 100-drone example): every member's 32x32 view against the
    oracle's brute-force render of the mesh and the 99 other boxes, before and after three steps (the
    tree is rebuilt from the new states); member tests per ray with the tree against the 99 without."""
    sim, ctx = vf
    p = default_params()
    sc = scenes.box_room(seed=1)
    sid = ctx.build_scene(sc["verts"], sc["tris"], sc["rgb"])
    n_tris = sc["tris"].shape[0]
    rng = np.random.default_rng(100)
    n = 100
    st0 = _swarm_of_100(p, rng, n)
    groups = [list(range(n))]
    ctx.set_swarms(groups, half_extent=HALF, rgb=RGB)
    views, npx, offs, mh, mw = sim.make_views(n, sid, (32, 32), swarm=0)
    st = torch.as_tensor(st0).cuda()
    depth = torch.empty(npx).cuda()
    ids = torch.empty(npx, dtype=torch.int32).cuda()
    acts = agents.random_actions(9, 3, n, p, c_range=(0.95, 1.05), rate=0.5)
    header("swarm of 100: views through the member tree, before and after 3 steps")
    for phase in ("start", "after 3 steps"):
        if phase != "start":
            for k in range(3):
                ctx.step(p, st, torch.as_tensor(acts[k]).cuda(), views=views, max_hw=(mh, mw), depth=depth,
                         tri_id=ids, out_pixels=npx)
        ctx.read_stats(reset=True)
        ctx.set_stats(True)
        ctx.render(st, views, max_hw=(mh, mw), depth=depth, tri_id=ids, out_pixels=npx)
        ctx.set_stats(False)
        stats = ctx.read_stats(reset=True)
        ctx.sync_check()
        s_now = st.cpu().numpy()
        dd, ii = depth.cpu().numpy(), ids.cpu().numpy()
        masked, seen = [], 0
        for i in range(n):
            ref = oren.render_view(s_now[i].astype(np.float64), sc, 32, 32, math.pi / 2,
                                   others=_others(s_now, groups[0], i, n_tris))
            sl = slice(offs[i], offs[i] + 1024)
            masked.append(compare_render(dd[sl], ii[sl], None, ref, 100.0, label=f"{phase} agent {i}"))
            seen += int((ii[sl] >= n_tris).sum())
        per_ray = stats["member_tests"] / max(stats["rays"], 1)
        record(f"swarm100[{phase}]", member_tests_per_ray=per_ray, brute_force_per_ray=n - 1,
               member_pixels=seen, masked=float(np.mean(masked)))
        assert np.mean(masked) < 0.02
        assert seen > 1000, "the members should fill part of the views"
        assert per_ray < 0.5 * (n - 1)
    ctx.set_swarms([])
    ctx.free_scene(sid)


def test_swarm_limits(vf):
    sim, ctx = vf
    with pytest.raises(sim.capi.VfError):
        ctx.set_swarms([list(range(4097))])
    ctx.set_swarms([list(range(4096))])     # the largest swarm builds
    ctx.set_swarms([])
