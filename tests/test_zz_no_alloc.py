"""vf_step_noalloc (the allocation-free step) against vf_step through the C ABI: the same states, depth,
ids and colours bit for bit, on two calls in a row with the second smaller, for fused, split (with the
cost order's recorded work) and automatic launches; and its limits (a fused launch beyond 262,144 state
slots and swarm mode are refused with VF_EINVAL)."""
import numpy as np
import pytest
import torch

from workloads import agents, default_params, scenes
from tests.gpu_util import header

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    from paper_2407_14783_amd import capi, sim
    ctx = sim.Context(0)
    p = default_params()
    sc = scenes.forest(seed=3, n_trees=300)
    sid = ctx.build_scene(sc["verts"], sc["tris"], sc["rgb"])
    s0 = agents.forest_starts(4, 300, sc, p)
    yield {"ctx": ctx, "sim": sim, "capi": capi, "p": p, "sid": sid, "s0": s0}
    ctx.set_launch_mode(None)
    ctx.free_scene(sid)
    ctx.close()


def _outputs(fn, env, n, hw, seed):
    sim, p = env["sim"], env["p"]
    views, npx, offs, mh, mw = sim.make_views(n, env["sid"], hw)
    st = torch.as_tensor(env["s0"][:n]).cuda()
    acts = torch.as_tensor(agents.random_actions(seed, 1, n, p)[0]).cuda()
    depth = torch.full((npx,), -3.0, device="cuda")
    ids = torch.full((npx,), -9, dtype=torch.int32, device="cuda")
    rgb = torch.zeros(3 * npx, dtype=torch.uint8, device="cuda")
    fn(p, st, acts, views=views, max_hw=(mh, mw), depth=depth, tri_id=ids, rgb=rgb, out_pixels=npx)
    env["ctx"].sync_check()
    return [t.cpu().numpy() for t in (st, depth, ids, rgb)]


@pytest.mark.parametrize("mode,sizes", [("fused", [(12, (64, 64)), (5, (40, 56))]),
                                        ("split", [(300, (64, 64)), (120, (64, 64)), (120, (64, 64))]),
                                        ("auto", [(40, (64, 64)), (7, (33, 47))])])
def test_step_noalloc_equals_step(env, mode, sizes):
    ctx = env["ctx"]
    ctx.set_launch_mode({"fused": True, "split": False, "auto": None}[mode])
    header(f"allocation-free step vs vf_step: {mode}, calls of {[n for n, _ in sizes]} agents")
    try:
        for k, (n, hw) in enumerate(sizes):
            ref = _outputs(ctx.step, env, n, hw, 50 + k)
            got = _outputs(ctx.step_noalloc, env, n, hw, 50 + k)
            for name, a, b in zip(("state", "depth", "ids", "rgb"), ref, got):
                assert np.array_equal(a, b), f"{mode} call {k} ({n} agents): {name} differs"
    finally:
        ctx.set_launch_mode(None)


def test_step_noalloc_limits(env):
    ctx, sim, capi, p = env["ctx"], env["sim"], env["capi"], env["p"]
    big = torch.zeros((262_145, 17), device="cuda")
    big[:, 3] = 1.0
    n = 2
    views, npx, offs, mh, mw = sim.make_views(n, env["sid"], (16, 16))
    idx = torch.tensor([0, 262_144], dtype=torch.int32, device="cuda")
    acts = torch.as_tensor(agents.random_actions(3, 1, n, p)[0]).cuda()
    depth = torch.empty(npx, device="cuda")
    ctx.set_launch_mode(True)
    try:
        with pytest.raises(capi.VfError):
            ctx.step_noalloc(p, big, acts, views=views, env_idx=idx, max_hw=(mh, mw), depth=depth, out_pixels=npx)
        ctx.step(p, big, acts, views=views, env_idx=idx, max_hw=(mh, mw), depth=depth, out_pixels=npx)
        ctx.sync_check()
    finally:
        ctx.set_launch_mode(None)
    ctx.set_swarms([[0, 1]])
    try:
        st = torch.as_tensor(env["s0"][:n]).cuda()
        with pytest.raises(capi.VfError):
            ctx.step_noalloc(p, st, acts, views=views, max_hw=(mh, mw), depth=depth, out_pixels=npx)
    finally:
        ctx.set_swarms([])
