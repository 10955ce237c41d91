"""Rollout loss and its FP64 central finite differences (differentiable dynamics, Sec. III-A).

The paper differentiates its dynamics through autograd; the device path uses
hand-written adjoints.  The oracle provides the reference derivative the plain
way: central differences of an FP64 rollout.

Loss (the obstacle-proximity + goal loss of the differentiable workload; the
paper fixes none, this reading is used):
    L = sum_agents sum_{k=1..H} [ mean_pixels exp(-D_k / d0) + w_goal |p_k - goal|^2 ],
with D_k the depth image rendered at the state after step k, d0 = 1 m and
w_goal = 0.01.  Missed pixels have the constant miss depth.
"""
import numpy as np

from . import dynamics, render


def rollout_loss(state0, actions, params, scene, goals, view, d0=1.0, w_goal=0.01, return_images=False):
    """L(s0, a_0..a_{H-1}) in FP64; optionally the per-step depth images (for discontinuity screening)."""
    s = np.asarray(state0, dtype=np.float64)
    goals = np.asarray(goals, dtype=np.float64)
    total = 0.0
    images = []
    for a in actions:
        s = dynamics.step(s, a, params)
        for i in range(s.shape[0]):
            r = render.render_view(s[i], scene, view["H"], view["W"], view["hfov"], view["near"], view["far"],
                                   view.get("miss_depth"), with_mask=False)
            total += float(np.mean(np.exp(-r["depth"] / d0)))
            if return_images:
                images.append(r["depth"])
        total += w_goal * float(np.sum((s[:, 0:3] - goals) ** 2))
    if return_images:
        return total, np.stack(images) if images else np.zeros((0,))
    return total


def central_difference(fun, x, direction, h=1e-6):
    """(f(x + h u) - f(x - h u)) / (2h) for a flat FP64 vector x and direction u."""
    x = np.asarray(x, dtype=np.float64)
    u = np.asarray(direction, dtype=np.float64)
    return (fun(x + h * u) - fun(x - h * u)) / (2.0 * h)


def rollout_edge_mask(state0, actions, params, scene, view, eps_edge=1e-4):
    """Pixel-steps [H, N, pixels] of the rollout from state0 whose closest hit is not decided robustly:
    the comparison mask of render_view (edges, near misses, ties, clip planes) with eps_edge.  At a
    triangle edge the depth stays continuous but its derivative jumps from one plane to the other, and
    which plane a ray in finite precision meets there is not decided: the gradient of such a pixel is
    not defined to compare."""
    s = np.asarray(state0, dtype=np.float64)
    masks = []
    for a in np.asarray(actions, dtype=np.float64):
        s = dynamics.step(s, a, params)
        for i in range(s.shape[0]):
            r = render.render_view(s[i], scene, view["H"], view["W"], view["hfov"], view["near"], view["far"],
                                   view.get("miss_depth"), eps_edge=eps_edge)
            masks.append(r["mask"].reshape(-1))
    n = s.shape[0]
    return np.stack(masks).reshape(-1, n, masks[0].size) if masks else np.zeros((0, n, 0), dtype=bool)


def rollout_directional(state0, actions, params, scene, goals, view, u_state, u_actions, h=1e-6, d0=1.0,
                        w_goal=0.01, jump_abs=1e-2, jump_rel=1e-3, return_jumps=False, remove=None):
    """Directional derivative of the rollout loss along (u_state, u_actions) by central differences.

    Returns (derivative, smooth, corrected, n_jumps).  The loss is piecewise
    smooth: a pixel whose ray crosses a silhouette between the +h and -h rollouts
    changes depth by a finite jump (flagged when |D+ - D-| > jump_abs + jump_rel D),
    and the plain difference quotient then measures that jump.  `smooth` says no
    pixel jumped.  `corrected` removes exactly the jumped pixels' terms
    exp(-D/d0)/P from both rollouts before differencing: the derivative of the
    loss restricted to the pixels that stay on one smooth branch (a change of hit
    triangle across a shared edge keeps the depth continuous and is kept).  With return_jumps the flags
    of the removed pixel-steps come back too, [H, N, pixels] (step, agent, pixel), so that the gradient
    being checked can be taken of the same restricted loss.  remove [H, N, pixels] (say rollout_edge_mask)
    names more pixel-steps to leave out the same way; they are counted and returned with the jumped ones.
    """
    s0 = np.asarray(state0, dtype=np.float64)
    a = np.asarray(actions, dtype=np.float64)
    lp, dp = rollout_loss(s0 + h * u_state, a + h * u_actions, params, scene, goals, view, d0=d0, w_goal=w_goal,
                          return_images=True)
    lm, dm = rollout_loss(s0 - h * u_state, a - h * u_actions, params, scene, goals, view, d0=d0, w_goal=w_goal,
                          return_images=True)
    raw = (lp - lm) / (2.0 * h)
    if dp.size == 0:
        return (raw, True, raw, 0, np.zeros((0,), dtype=bool)) if return_jumps else (raw, True, raw, 0)
    jumped = np.abs(dp - dm) > jump_abs + jump_rel * np.minimum(np.abs(dp), np.abs(dm))
    if remove is not None:
        jumped = jumped | np.asarray(remove, dtype=bool).reshape(jumped.shape)
    n_pix = dp[0].size
    cp = float(np.sum(np.exp(-dp[jumped] / d0)) / n_pix)
    cm = float(np.sum(np.exp(-dm[jumped] / d0)) / n_pix)
    corrected = ((lp - cp) - (lm - cm)) / (2.0 * h)
    if return_jumps:
        n_agents = np.asarray(state0).shape[0]
        return raw, not bool(jumped.any()), corrected, int(jumped.sum()), jumped.reshape(-1, n_agents, n_pix)
    return raw, not bool(jumped.any()), corrected, int(jumped.sum())


def step_jacobian(state, action, params, h=1e-6):
    """Central-difference Jacobians of one control step: d s' / d s [N,17,17] and d s' / d a [N,17,4]."""
    s = np.asarray(state, dtype=np.float64)
    a = np.asarray(action, dtype=np.float64)
    n = s.shape[0]
    js = np.empty((n, 17, 17))
    ja = np.empty((n, 17, 4))
    for j in range(17):
        e = np.zeros_like(s)
        e[:, j] = h
        js[:, :, j] = (dynamics.step(s + e, a, params) - dynamics.step(s - e, a, params)) / (2 * h)
    for j in range(4):
        e = np.zeros_like(a)
        e[:, j] = h
        ja[:, :, j] = (dynamics.step(s, a + e, params) - dynamics.step(s, a - e, params)) / (2 * h)
    return js, ja


def depth_pose_gradient(state_row, scene, view, pixels, h=1e-6):
    """Central differences of each listed pixel's depth with respect to p (3) and q (4): [P, 7]."""
    s = np.asarray(state_row, dtype=np.float64)
    g = np.empty((len(pixels), 7))
    for j in range(7):
        e = np.zeros(17)
        e[j] = h
        dp = render.render_view(s + e, scene, view["H"], view["W"], view["hfov"], view["near"], view["far"],
                                view.get("miss_depth"), with_mask=False, pixels=pixels,
                                mount=view.get("mount"))["depth"]
        dm = render.render_view(s - e, scene, view["H"], view["W"], view["hfov"], view["near"], view["far"],
                                view.get("miss_depth"), with_mask=False, pixels=pixels,
                                mount=view.get("mount"))["depth"]
        g[:, j] = (dp - dm) / (2 * h)
    return g
