"""Differentiable rollout (Sec. III-A: differentiable dynamics) with checkpointed BPTT.

``rollout(ctx, params, s0, actions, views, ...)`` runs H steps of vf_step and
returns the states after every step [H, N, 17] and the depth images [H, P].
Backward walks the horizon in segments of ``checkpoint_every`` steps from the
end: it re-runs the segment's dynamics from the saved state checkpoint, then for
each step in reverse adds the state-output gradient, accumulates the
depth-to-pose adjoint (vf_render_backward) into the state cotangent and applies
the RK4 step adjoint (vf_step_backward).  The depth adjoint needs each frame's
hit ids, H x P int32 for the horizon (1 GiB for 1,024 agents x 64 steps of
64x64).  ``keep_ids``: True keeps them from the forward and backward renders
nothing; False keeps one segment's worth and backward re-renders each segment
(about twice the rollout time); None (the default) keeps them while they fit
``ids_budget_bytes`` (4 GiB) and re-renders beyond.  State checkpoints take
N x 17 floats each.
All arithmetic runs in the library's kernels; torch only holds the buffers.
"""
import torch

from . import capi


class _Rollout(torch.autograd.Function):
    @staticmethod
    def forward(fctx, s0, actions, sim_ctx, params, views, max_hw, out_pixels, k, keep_ids):
        H, N = actions.shape[0], actions.shape[1]
        p = params if isinstance(params, capi.DynParams) else capi.params_struct(params)
        s = s0.detach().clone().contiguous()
        states = torch.empty((H, N, 17), dtype=torch.float32, device=s0.device)
        depths = torch.empty((H, out_pixels), dtype=torch.float32, device=s0.device)
        ids = torch.empty((H if keep_ids else 1, out_pixels), dtype=torch.int32, device=s0.device)
        ckpts = [s.clone()]
        acts = actions.detach().contiguous()
        for t in range(H):
            sim_ctx.step(p, s, acts[t], views=views, max_hw=max_hw, depth=depths[t],
                         tri_id=ids[t if keep_ids else 0], out_pixels=out_pixels)
            states[t].copy_(s)
            if (t + 1) % k == 0 and t + 1 < H:
                ckpts.append(s.clone())
        fctx.sim_ctx, fctx.p, fctx.views, fctx.max_hw, fctx.out_pixels, fctx.k = sim_ctx, p, views, max_hw, \
            out_pixels, k
        fctx.keep_ids = keep_ids
        fctx.save_for_backward(acts, ids if keep_ids else ids[:0], *ckpts)
        return states, depths

    @staticmethod
    def backward(fctx, g_states, g_depths):
        acts, kept_ids, *ckpts = fctx.saved_tensors
        sim_ctx, p, views, max_hw, npx, k = fctx.sim_ctx, fctx.p, fctx.views, fctx.max_hw, fctx.out_pixels, fctx.k
        H, N = acts.shape[0], acts.shape[1]
        dev = acts.device
        g_states = torch.zeros((H, N, 17), device=dev) if g_states is None else g_states.contiguous()
        g_depths = torch.zeros((H, npx), device=dev) if g_depths is None else g_depths.contiguous()
        lam = torch.zeros((N, 17), dtype=torch.float32, device=dev)
        lam_prev = torch.empty_like(lam)
        g_act = torch.zeros_like(acts)
        scratch_depth = torch.empty(npx, dtype=torch.float32, device=dev)
        n_seg = len(ckpts)
        for seg in reversed(range(n_seg)):
            a, b = seg * k, min((seg + 1) * k, H)
            # recompute the segment: seg_states[j] = s_{a+j}, ids[j] = hit ids of the frame after step a+j
            s = ckpts[seg].clone()
            seg_states = [s.clone()]
            if fctx.keep_ids:
                seg_ids = kept_ids[a:b]
                for t in range(a, b):
                    sim_ctx.step(p, s, acts[t])          # dynamics only: the ids were kept
                    seg_states.append(s.clone())
            else:
                seg_ids = torch.empty((b - a, npx), dtype=torch.int32, device=dev)
                for t in range(a, b):
                    sim_ctx.step(p, s, acts[t], views=views, max_hw=max_hw, depth=scratch_depth,
                                 tri_id=seg_ids[t - a], out_pixels=npx)
                    seg_states.append(s.clone())
            for t in reversed(range(a, b)):
                lam += g_states[t]
                sim_ctx.render_backward(seg_states[t + 1 - a], views, max_hw, seg_ids[t - a], g_depths[t], npx, lam)
                sim_ctx.step_backward(p, seg_states[t - a], acts[t], lam, lam_prev, g_act[t])
                lam, lam_prev = lam_prev, lam
        return lam.clone(), g_act, None, None, None, None, None, None, None


IDS_BUDGET_BYTES = 4 << 30


def rollout(sim_ctx, params, s0, actions, views, max_hw, out_pixels, checkpoint_every=8, keep_ids=None,
            ids_budget_bytes=IDS_BUDGET_BYTES):
    """States [H, N, 17] and depth images [H, out_pixels] of an H-step rollout, differentiable in s0 and actions.
    keep_ids: keep every frame's hit ids for the backward pass (True), re-render each segment there (False), or
    keep them while H x out_pixels x 4 bytes fit ids_budget_bytes (None)."""
    if keep_ids is None:
        keep_ids = actions.shape[0] * int(out_pixels) * 4 <= ids_budget_bytes
    return _Rollout.apply(s0, actions, sim_ctx, params, views, tuple(max_hw), int(out_pixels),
                          int(checkpoint_every), bool(keep_ids))
