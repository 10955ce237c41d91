"""GPU adjoint kernels against FP64 central finite differences of the oracle.

vf_step_backward: J_s^T lam and J_a^T lam of one control step against the
oracle's central-difference Jacobians (h = 1e-6) at the same float32 inputs.
vf_render_backward: sum_pixels g * d depth / d (p, q) against central
differences of the oracle's brute-force depth, off the edge mask.
Rollout: the checkpointed BPTT of the differentiable rollout against central
differences of the oracle's rollout loss, along 8 seeded random directions and
per coordinate (actions at steps 0, 31, 63 and the start state).  Pixel-steps
whose depth jumps between the +h and -h rollouts (a silhouette crossing) are
removed from both sides: from the oracle's difference and from the loss the
device gradient is taken of.
"""
import math

import numpy as np
import pytest
import torch

from oracle import dynamics as odyn
from oracle import gradients as ograd
from oracle import render as oren
from workloads import agents, default_params, device_params, scenes
from tests.gpu_util import header, record

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vf():
    from paper_2407_14783_amd import sim
    ctx = sim.Context(0)
    yield sim, ctx
    ctx.close()


def _dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to(dtype).cuda()


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-12))


def _random_states(rng, n, p, rate=1.0, speed=1.5):
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return agents.make_states(rng.uniform(-5, 5, (n, 3)), p, quat=q, vel=rng.normal(scale=speed, size=(n, 3)),
                              omega=rng.uniform(-rate, rate, (n, 3)),
                              rotor=np.sqrt(p["mass"] * p["g"] / 4) * rng.uniform(0.8, 1.2, (n, 4)))


@pytest.mark.parametrize("variant", ["ctbr", "ctbr_saturating", "srt", "euler_nsub2", "rk4_nsub3", "quad_drag",
                                     "quad_drag_srt", "ps", "lv", "ps_euler_nsub2_drag"])
def test_step_backward_matches_fd_jacobian(vf, variant):
    """J_s^T lam and J_a^T lam of one control step against the oracle's central-difference Jacobians.  CTBR
    and SRT take the hand-written reverse-mode kernel, PS and LV the forward-mode (dual number) one."""
    sim, ctx = vf
    rng = np.random.default_rng({"ctbr": 1, "ctbr_saturating": 2, "srt": 3, "euler_nsub2": 4, "rk4_nsub3": 5,
                                 "quad_drag": 6, "quad_drag_srt": 7, "ps": 8, "lv": 9,
                                 "ps_euler_nsub2_drag": 10}[variant])
    speed = 1.5
    if variant == "ps":
        p = default_params(ctrl=odyn.PS)
    elif variant == "lv":
        p = default_params(ctrl=odyn.LV)
    elif variant == "ps_euler_nsub2_drag":
        p = default_params(ctrl=odyn.PS, integrator=odyn.EULER, n_sub=2, c_quad=(0.04, 0.06, 0.1))
    elif variant == "quad_drag":
        # Eq. 2 with both terms, at body speeds (about 7 m/s) where the quadratic term dominates
        p = default_params(c_quad=(0.04, 0.06, 0.1))
        speed = 4.0
    elif variant == "quad_drag_srt":
        p = default_params(ctrl=odyn.SRT, c_quad=(0.1, 0.1, 0.1), k_lin=(0.0, 0.0, 0.0))
        speed = 4.0
    elif variant == "srt":
        p = default_params(ctrl=odyn.SRT)
    elif variant == "euler_nsub2":
        p = default_params(integrator=odyn.EULER, n_sub=2)
    elif variant == "rk4_nsub3":
        p = default_params(n_sub=3)
    else:
        p = default_params()
    n = 32
    s = _random_states(rng, n, p, speed=speed)
    if variant in ("srt", "quad_drag_srt"):
        a = (p["mass"] * p["g"] / 4 * rng.uniform(0.7, 1.3, (n, 4))).astype(np.float32)
    elif variant == "ctbr_saturating":
        a = agents.random_actions(int(rng.integers(1 << 30)), 1, n, p)[0]
    elif variant.startswith("ps"):
        # position setpoints within 3 m of the agent and a yaw setpoint
        a = np.concatenate([s[:, 0:3] + rng.uniform(-3, 3, (n, 3)), rng.uniform(-np.pi, np.pi, (n, 1))], 1).astype(
            np.float32)
    elif variant == "lv":
        a = np.concatenate([rng.uniform(-2, 2, (n, 3)), rng.uniform(-np.pi, np.pi, (n, 1))], 1).astype(np.float32)
    else:
        a = np.concatenate([rng.uniform(0.8, 1.2, (n, 1)) * p["g"], rng.uniform(-0.5, 0.5, (n, 3))], 1).astype(
            np.float32)
    lam = rng.normal(size=(n, 17)).astype(np.float32)
    g_in = torch.zeros((n, 17)).cuda()
    g_a = torch.zeros((n, 4)).cuda()
    header(f"step_backward: {variant}")
    ctx.step_backward(p, _dev(s), _dev(a), _dev(lam), g_in, g_a)
    torch.cuda.synchronize()
    js, ja = ograd.step_jacobian(s.astype(np.float64), a.astype(np.float64), device_params(p))
    ref_in = np.einsum("nij,ni->nj", js, lam.astype(np.float64))
    ref_a = np.einsum("nij,ni->nj", ja, lam.astype(np.float64))
    gi, ga = g_in.cpu().numpy(), g_a.cpu().numpy()
    record(f"step_backward[{variant}]", state_rel=max(_rel(gi[i], ref_in[i]) for i in range(n)),
           action_rel=max(_rel(ga[i], ref_a[i]) for i in range(n) if np.linalg.norm(ref_a[i]) > 1e-6),
           bound=2e-4)
    for i in range(n):
        assert _rel(gi[i], ref_in[i]) <= 2e-4, f"{variant} agent {i}: state cotangent rel err {_rel(gi[i], ref_in[i]):.2e}"
        if np.linalg.norm(ref_a[i]) > 1e-6:
            assert _rel(ga[i], ref_a[i]) <= 2e-4, f"{variant} agent {i}: action cotangent rel err {_rel(ga[i], ref_a[i]):.2e}"
        else:
            assert np.linalg.norm(ga[i]) <= 1e-5


@pytest.mark.parametrize("h,w", [(16, 16), (12, 20), (40, 26)])
def test_render_backward_matches_fd(vf, h, w):
    """Square and non-square views; 40 x 26 spans two pixel batches of a workgroup and a ragged third."""
    sim, ctx = vf
    p = default_params()
    sc = scenes.box_room(seed=1)
    sid = ctx.build_scene(sc["verts"], sc["tris"], sc["rgb"])
    rng = np.random.default_rng(31)
    n = 4
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    st = agents.make_states(rng.uniform([1, 1, 0.5], [9, 9, 3.5], size=(n, 3)), p, quat=q)
    views, npx, offs, mh, mw = sim.make_views(n, sid, (h, w))
    ids = torch.zeros(npx, dtype=torch.int32).cuda()
    depth = torch.zeros(npx).cuda()
    ctx.render(_dev(st), views, max_hw=(mh, mw), depth=depth, tri_id=ids, out_pixels=npx)
    g = rng.normal(size=npx).astype(np.float32)
    view = {"H": h, "W": w, "hfov": math.pi / 2, "near": 0.01, "far": 100.0}
    # zero the weight of pixels near edges (finite differences would straddle two triangles there)
    for i in range(n):
        ref = oren.render_view(st[i].astype(np.float64), sc, h, w, math.pi / 2, eps_edge=1e-3)
        g[offs[i]:offs[i] + h * w][ref["mask"].reshape(-1)] = 0.0
    base = rng.normal(size=(n, 17)).astype(np.float32)
    grad_state = _dev(base)
    header(f"render_backward: box room, 4 agents, {h}x{w}")
    ctx.render_backward(_dev(st), views, (mh, mw), ids, _dev(g), npx, grad_state)
    ctx.sync_check()
    got = grad_state.cpu().numpy() - base
    for i in range(n):
        fd = ograd.depth_pose_gradient(st[i].astype(np.float64), sc, view, np.arange(h * w))
        expect = g[offs[i]:offs[i] + h * w].astype(np.float64) @ fd
        assert _rel(got[i, 0:7], expect) <= 1e-3, f"agent {i}: rel err {_rel(got[i, 0:7], expect):.2e}"
        assert np.allclose(got[i, 7:], 0.0, atol=1e-6)
    ctx.free_scene(sid)


def _crop_forest(sc, centers, radius):
    """Ground plus the trees within `radius` (xy) of any of the given points."""
    trees = sc["trees"]
    d = np.min(np.hypot(trees[:, 0][:, None] - centers[None, :, 0], trees[:, 1][:, None] - centers[None, :, 1]), axis=1)
    keep = np.nonzero(d < radius)[0]
    tri_sel = [np.arange(2)] + [2 + 64 * k + np.arange(64) for k in keep]
    tri_sel = np.concatenate(tri_sel)
    return {"verts": sc["verts"], "tris": sc["tris"][tri_sel], "rgb": sc["rgb"][tri_sel]}


BPTT_TOL = 1e-3        # relative, per direction and per coordinate
N_DIRECTIONS = 8


def _bptt_setup(agent=None):
    """4 agents in a forest (or one of them in a crop around it alone), horizon 64, hover-range actions,
    goals 12 m away: the differentiable workload's configuration on the FD-checkable scale."""
    p = default_params()
    full = scenes.forest(seed=3)
    n, H = 4, 64
    s0 = agents.forest_starts(8, n, full, p)
    rng = np.random.default_rng(8)
    acts = np.concatenate([rng.uniform(0.9, 1.15, (H, n, 1)) * p["g"], rng.uniform(-0.6, 0.6, (H, n, 3))],
                          axis=2).astype(np.float32)
    ang = rng.uniform(0, 2 * np.pi, n)
    goals = (s0[:, 0:3] + np.stack([12 * np.cos(ang), 12 * np.sin(ang), np.zeros(n)], 1)).astype(np.float32)
    if agent is not None:
        s0, acts, goals = s0[agent:agent + 1], acts[:, agent:agent + 1], goals[agent:agent + 1]
    sc = _crop_forest(full, s0[:, 0:3], 6.0)
    return p, sc, s0, acts, goals, rng


def _gpu_gradient(ctx, sim, vag, p, sid, s0, acts, goals, w_goal, keep=None, d0=1.0):
    """Loss and its gradient through the checkpointed BPTT (k = 8).  keep [H, N, 4096] (0/1) drops
    pixel-steps from the depth term, as the oracle's jump-corrected differences do."""
    H, n = acts.shape[0], acts.shape[1]
    views, npx, offs, mh, mw = sim.make_views(n, sid, (64, 64))
    s0_t = _dev(s0).requires_grad_(True)
    a_t = _dev(acts).requires_grad_(True)
    states, depths = vag.rollout(ctx, p, s0_t, a_t, views, (mh, mw), npx, checkpoint_every=8)
    e = torch.exp(-depths.double() / d0).view(H, n, 64 * 64)
    if keep is not None:
        e = e * torch.as_tensor(keep, dtype=torch.float64).cuda()
    loss = e.mean(dim=2).sum() + w_goal * ((states[:, :, 0:3].double() - _dev(goals).double()) ** 2).sum()
    loss.backward()
    return loss.item(), s0_t.grad.cpu().numpy().astype(np.float64), a_t.grad.cpu().numpy().astype(np.float64)


VIEW64 = {"H": 64, "W": 64, "hfov": math.pi / 2, "near": 0.01, "far": 100.0}


@pytest.mark.timeout(900)
@pytest.mark.parametrize("w_goal", [0.01, 0.0])
def test_bptt_rollout_gradient_vs_oracle_fd(vf, w_goal):
    """Differentiable rollout: 4 agents in a forest, horizon 64, checkpoints every 8, 64x64 depth.  The
    directional derivative along 8 seeded unit directions (start states and all actions) against FP64
    central differences (h = 1e-6) of the oracle's rollout loss, within 1e-3 relative, every direction.
    Pixel-steps whose depth jumps between the two oracle rollouts (a silhouette crossing) are removed
    from both sides: the oracle's difference leaves out their terms and the device gradient is taken of
    the loss without them."""
    sim, ctx = vf
    from paper_2407_14783_amd import autograd as vag
    p, sc, s0, acts, goals, rng = _bptt_setup()
    n, H = s0.shape[0], acts.shape[0]
    sid = ctx.build_scene(sc["verts"], sc["tris"], sc["rgb"])
    header(f"BPTT: 4 agents x 64 steps, k = 8, w_goal = {w_goal}, {N_DIRECTIONS} directions")
    loss, g_s0, g_a = _gpu_gradient(ctx, sim, vag, p, sid, s0, acts, goals, w_goal)
    pd = device_params(p)      # the oracle runs on the parameter values the device receives
    l_ref = ograd.rollout_loss(s0, acts, pd, sc, goals, VIEW64, w_goal=w_goal)
    assert abs(loss - l_ref) <= 1e-4 * abs(l_ref)
    worst, jumps = 0.0, []
    for j in range(N_DIRECTIONS):
        u_s = rng.normal(size=s0.shape)
        u_a = rng.normal(size=acts.shape)
        norm = math.sqrt((u_s ** 2).sum() + (u_a ** 2).sum())
        u_s, u_a = u_s / norm, u_a / norm
        fd, smooth, fd_c, n_jumps, jumped = ograd.rollout_directional(s0, acts, pd, sc, goals, VIEW64, u_s, u_a,
                                                                      h=1e-6, w_goal=w_goal, return_jumps=True)
        if n_jumps:
            _, gs, ga = _gpu_gradient(ctx, sim, vag, p, sid, s0, acts, goals, w_goal, keep=~jumped)
        else:
            gs, ga = g_s0, g_a
        ad = float((gs * u_s).sum() + (ga * u_a).sum())
        rel = abs(ad - fd_c) / max(abs(fd_c), 1e-3)
        print(f"[gpu-test] direction {j}: adjoint {ad:.6e} fd {fd_c:.6e} rel {rel:.2e} "
              f"({n_jumps} jumped pixel-steps of {H * n * 4096} removed)", flush=True)
        assert rel <= BPTT_TOL, f"direction {j}: adjoint {ad} vs fd {fd_c} (rel {rel:.2e})"
        worst = max(worst, rel)
        jumps.append(n_jumps)
    record(f"bptt_directions[w_goal={w_goal}]", compared=N_DIRECTIONS, of=N_DIRECTIONS, worst_rel=worst,
           bound=BPTT_TOL, jumped_pixel_steps=jumps)
    ctx.free_scene(sid)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("ctrl", ["ps", "lv"])
def test_bptt_outer_loop_controllers_vs_oracle_fd(vf, ctrl):
    """The checkpointed BPTT through the PS and LV controllers (forward-mode step adjoint): 2 agents of the
    differentiable configuration's forest, horizon 16, position (PS) or velocity (LV) setpoints; the
    directional derivative along 4 seeded directions against the oracle's FP64 central differences,
    within 1e-3 relative (jumped and edge pixel-steps removed from both sides, as above)."""
    sim, ctx = vf
    from paper_2407_14783_amd import autograd as vag
    p0, _, s0_all, _, goals_all, _ = _bptt_setup()
    p = default_params(ctrl=odyn.PS if ctrl == "ps" else odyn.LV)
    n, H = 2, 16
    s0, goals = s0_all[:n], goals_all[:n]
    rng = np.random.default_rng({"ps": 41, "lv": 42}[ctrl])
    if ctrl == "ps":
        target = s0[:, 0:3] + rng.uniform(-2.0, 2.0, (n, 3))
        acts = np.repeat(np.concatenate([target, rng.uniform(-1, 1, (n, 1))], 1)[None], H, 0)
    else:
        acts = np.repeat(np.concatenate([rng.uniform(-1.5, 1.5, (n, 3)), rng.uniform(-1, 1, (n, 1))], 1)[None], H, 0)
    acts = (acts + rng.normal(scale=0.05, size=acts.shape)).astype(np.float32)
    full = scenes.forest(seed=3)
    sc = _crop_forest(full, s0[:, 0:3], 6.0)
    sid = ctx.build_scene(sc["verts"], sc["tris"], sc["rgb"])
    header(f"BPTT through {ctrl.upper()}: {n} agents x {H} steps, {sc['tris'].shape[0]} triangles")
    pd = device_params(p)
    traj_ok = odyn.rollout(s0.astype(np.float64), acts.astype(np.float64), pd)
    assert np.isfinite(traj_ok).all()
    edges = ograd.rollout_edge_mask(s0, acts, pd, sc, VIEW64, eps_edge=1e-4)
    worst = 0.0
    for j in range(4):
        u_s = rng.normal(size=s0.shape)
        u_a = rng.normal(size=acts.shape)
        norm = math.sqrt((u_s ** 2).sum() + (u_a ** 2).sum())
        u_s, u_a = u_s / norm, u_a / norm
        _, _, fd_c, n_removed, removed = ograd.rollout_directional(s0, acts, pd, sc, goals, VIEW64, u_s, u_a, h=1e-6,
                                                                    w_goal=0.01, return_jumps=True, remove=edges)
        _, gs, ga = _gpu_gradient(ctx, sim, vag, p, sid, s0, acts, goals, 0.01, keep=~removed)
        ad = float((gs * u_s).sum() + (ga * u_a).sum())
        rel = abs(ad - fd_c) / max(abs(fd_c), 1e-3)
        print(f"[gpu-test] {ctrl} direction {j}: adjoint {ad:.6e} fd {fd_c:.6e} rel {rel:.2e} "
              f"({n_removed} pixel-steps removed)", flush=True)
        assert rel <= BPTT_TOL, f"{ctrl} direction {j}: adjoint {ad} vs fd {fd_c} (rel {rel:.2e})"
        worst = max(worst, rel)
    record(f"bptt_outer_loop[{ctrl}]", directions=4, worst_rel=worst, bound=BPTT_TOL)
    ctx.free_scene(sid)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("agent", [0, 1, 2, 3])
def test_bptt_coordinates_vs_oracle_fd(vf, agent):
    """Per-coordinate gradients of the rollout loss (w_goal = 0.01) for one agent of the differentiable
    configuration, in a crop of the forest around it: the 4 action components at steps 0, 31 and 63 and
    the 17 start-state components, each against FP64 central differences (h = 1e-6) of the oracle,
    within 1e-3 relative.  A coordinate whose derivative is under 1% of the largest of its group (the
    actions of one step, or the start state) is held to 1e-3 of that 1%: float32 adjoint errors scale
    with the group's largest terms.  Jumped pixel-steps are removed from both sides as above, and so are
    the pixel-steps whose ray passes within 1e-4 max(1, t) of an edge of the triangle it hits in the
    oracle's rollout (rollout_edge_mask): the depth derivative changes plane there, and a single
    coordinate's derivative, which the pixel sums can cancel to a few percent of its terms, moves by
    more than the bound when a float32 ray and an FP64 ray take different sides."""
    sim, ctx = vf
    from paper_2407_14783_amd import autograd as vag
    p, sc, s0, acts, goals, _ = _bptt_setup(agent)
    H = acts.shape[0]
    w_goal = 0.01
    sid = ctx.build_scene(sc["verts"], sc["tris"], sc["rgb"])
    header(f"BPTT coordinates: agent {agent}, {sc['tris'].shape[0]} triangles, 64 steps")
    # FP64 oracle states s_k (dynamics only) to start the differences at step k from
    pd = device_params(p)      # the oracle runs on the parameter values the device receives
    traj = odyn.rollout(s0.astype(np.float64), acts.astype(np.float64), pd)
    groups = [("a0", 0), ("a31", 31), ("a63", 63), ("s0", None)]
    worst = 0.0
    n_checked = 0
    removed_steps = []
    grads = {}
    for name, k in groups:
        start = 0 if k is None else k
        dim = 17 if k is None else 4
        edges = ograd.rollout_edge_mask(traj[start], acts[start:], pd, sc, VIEW64, eps_edge=1e-4)
        fds, ads = [], []
        for c in range(dim):
            u_s = np.zeros((1, 17))
            u_a = np.zeros((H - start, 1, 4))
            if k is None:
                u_s[0, c] = 1.0
            else:
                u_a[0, 0, c] = 1.0
            fd, smooth, fd_c, n_removed, removed = ograd.rollout_directional(
                traj[start], acts[start:], pd, sc, goals, VIEW64, u_s, u_a, h=1e-6, w_goal=w_goal,
                return_jumps=True, remove=edges)
            keep = np.ones((H, 1, 4096), dtype=bool)
            keep[start:] = ~removed
            key = keep.tobytes()
            if key not in grads:
                grads[key] = _gpu_gradient(ctx, sim, vag, p, sid, s0, acts, goals, w_goal, keep=keep)[1:]
            gs, ga = grads[key]
            fds.append(fd_c)
            ads.append(gs[0, c] if k is None else ga[k, 0, c])
            removed_steps.append(n_removed)
        fds, ads = np.asarray(fds), np.asarray(ads)
        floor = 1e-2 * np.abs(fds).max()
        rel = np.abs(ads - fds) / np.maximum(np.abs(fds), floor)
        print(f"[gpu-test] agent {agent} {name}: fd {np.array2string(fds, precision=4)} "
              f"max rel {rel.max():.2e} ({int(edges.sum())} edge pixel-steps of {edges.size} removed)", flush=True)
        assert rel.max() <= BPTT_TOL, f"agent {agent} {name}: component {int(np.argmax(rel))} rel {rel.max():.2e}"
        worst = max(worst, float(rel.max()))
        n_checked += dim
    record(f"bptt_coordinates[agent {agent}]", coordinates=n_checked, worst_rel=worst, bound=BPTT_TOL,
           removed_pixel_steps_max=max(removed_steps))
    ctx.free_scene(sid)


def test_bptt_kept_ids_equal_rerendered(vf):
    """Keeping every frame's hit ids in the forward (no renders in backward) and re-rendering each segment in
    backward give the same gradients bit for bit: the same kernels see the same states and ids."""
    sim, ctx = vf
    from paper_2407_14783_amd import autograd as vag
    p = default_params()
    sc = scenes.forest(seed=3, n_trees=400)
    n, H = 6, 20
    s0 = agents.forest_starts(8, n, sc, p)
    rng = np.random.default_rng(31)
    acts = np.concatenate([rng.uniform(0.9, 1.15, (H, n, 1)) * p["g"], rng.uniform(-0.6, 0.6, (H, n, 3))],
                          axis=2).astype(np.float32)
    sid = ctx.build_scene(sc["verts"], sc["tris"], sc["rgb"])
    views, npx, offs, mh, mw = sim.make_views(n, sid, (64, 64))
    header("BPTT: kept hit ids vs re-rendered segments, 6 agents x 20 steps, k = 8")
    grads = []
    # kept, re-rendered, and the default's choice under a budget too small for the ids (re-rendered)
    for keep, budget in ((True, 0), (False, 0), (None, 1024)):
        s0_t = _dev(s0).requires_grad_(True)
        a_t = _dev(acts).requires_grad_(True)
        states, depths = vag.rollout(ctx, p, s0_t, a_t, views, (mh, mw), npx, checkpoint_every=8, keep_ids=keep,
                                     ids_budget_bytes=budget)
        loss = torch.exp(-depths).view(H, n, -1).mean(2).sum() + 0.01 * (states[:, :, 0:3] ** 2).sum()
        loss.backward()
        grads.append((s0_t.grad.cpu().numpy(), a_t.grad.cpu().numpy(), loss.item()))
    for other in grads[1:]:
        assert grads[0][2] == other[2]
        assert np.array_equal(grads[0][0], other[0]) and np.array_equal(grads[0][1], other[1])
    assert np.abs(grads[0][1]).max() > 0
    ctx.free_scene(sid)
