"""vf_step_noalloc under HIP graph capture (the callers it is for): a captured fused step and a captured split
step (cost-ordered after its first replay's shape is known) are replayed several times, with new actions
written into the captured action buffer and eager steps in between, and every replay's states, depth and ids
equal those of eager vf_step calls from the same states."""
import numpy as np
import pytest
import torch

from workloads import agents, default_params, scenes
from tests.gpu_util import header

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("mode,n", [("fused", 4), ("split", 300)])
def test_captured_noalloc_step_replays_equal_eager_steps(mode, n):
    from paper_2407_14783_amd import sim
    ctx = sim.Context(0)
    p = default_params()
    sc = scenes.forest(seed=3, n_trees=300)
    sid = ctx.build_scene(sc["verts"], sc["tris"], sc["rgb"])
    s0 = agents.forest_starts(44, n, sc, p)
    acts = agents.random_actions(45, 4, n, p)
    views, npx, offs, mh, mw = sim.make_views(n, sid, (64, 64))
    header(f"graph capture of vf_step_noalloc: {mode}, {n} agents, 4 replays")
    ctx.set_launch_mode(mode == "fused")
    try:
        # the captured step's buffers
        st = torch.as_tensor(s0).cuda()
        a_buf = torch.as_tensor(acts[0]).cuda()
        depth = torch.zeros(npx, device="cuda")
        ids = torch.zeros(npx, dtype=torch.int32, device="cuda")
        # the eager reference
        st_ref = torch.as_tensor(s0).cuda()
        depth_ref = torch.zeros(npx, device="cuda")
        ids_ref = torch.zeros(npx, dtype=torch.int32, device="cuda")
        if mode == "split":
            # one eager step of the same shape first, so the captured launch includes the cost order
            warm = torch.as_tensor(s0).cuda()
            ctx.step_noalloc(p, warm, a_buf, views=views, max_hw=(mh, mw), depth=depth, tri_id=ids, out_pixels=npx)
            torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            ctx.step_noalloc(p, st, a_buf, views=views, max_hw=(mh, mw), depth=depth, tri_id=ids, out_pixels=npx)
        torch.cuda.synchronize()
        assert torch.equal(st, torch.as_tensor(s0).cuda())        # capture runs nothing
        for k in range(4):
            a_buf.copy_(torch.as_tensor(acts[k]).cuda())
            g.replay()
            torch.cuda.synchronize()
            ctx.step(p, st_ref, torch.as_tensor(acts[k]).cuda(), views=views, max_hw=(mh, mw), depth=depth_ref,
                     tri_id=ids_ref, out_pixels=npx)
            ctx.sync_check()
            assert torch.equal(st, st_ref), f"{mode} replay {k}: states differ"
            assert torch.equal(depth, depth_ref) and torch.equal(ids, ids_ref), f"{mode} replay {k}: images differ"
    finally:
        ctx.set_launch_mode(None)
        ctx.free_scene(sid)
        ctx.close()
