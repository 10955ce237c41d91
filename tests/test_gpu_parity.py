"""GPU (gfx950) parity of the HIP path against the FP64 oracle, through the C ABI.

Dynamics: trajectories from the same float32 start states and actions, state
within 1e-5 * max(1, |s|) per component after every one of 100 steps.
Render: the oracle renders at the GPU's float32 poses (upcast); off the oracle's
edge/tie mask the hit ids and colours are bit-exact and depth is within 1e-4
relative.  Sizes span several 16x4 packets, ragged image edges and many BVH levels.
"""
import math

import numpy as np
import pytest
import torch

from oracle import dynamics as odyn
from oracle import render as oren
from workloads import agents, default_params, device_params, scenes
from tests.gpu_util import compare_render, header, record, state_close, STATE_TOL

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vf():
    from paper_2407_14783_amd import sim
    ctx = sim.Context(0)
    yield sim, ctx
    ctx.close()


def _dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to(dtype).cuda()


def _gpu_rollout(ctx, params, s0, acts, stride=1):
    """Dynamics-only rollout through vf_step (views = NULL): returns states [H+1, N, 17]."""
    st = _dev(s0)
    out = [s0.astype(np.float32)]
    for k in range(acts.shape[0]):
        ctx.step(params, st, _dev(acts[k]))
        if (k + 1) % stride == 0:
            out.append(st.cpu().numpy())
    torch.cuda.synchronize()
    return np.stack(out)


# ---------------------------------------------------------------------------
# dynamics
# ---------------------------------------------------------------------------

def test_dynamics_box_room_100_steps(vf):
    sim, ctx = vf
    p = default_params()
    s0 = agents.box_room_start(p)
    acts = agents.random_actions(2, 100, 1, p)
    header("dynamics: box-room agent, 100 CTBR steps")
    gpu = _gpu_rollout(ctx, p, s0, acts)
    ref = odyn.rollout(s0, acts, device_params(p))
    errs = [state_close(gpu[k], ref[k]) for k in range(101)]
    assert max(errs) <= STATE_TOL, f"max state error {max(errs):.3e} at step {int(np.argmax(errs))}"


def _rounding_amplification(s0, acts, p):
    """Growth over the horizon of a one-ulp (2^-24 relative) start perturbation, in the FP64 oracle."""
    rng = np.random.default_rng(1)
    s = s0.astype(np.float64)
    pert = s * (1 + rng.choice([-1, 1], size=s.shape) * 2.0 ** -24)
    a = odyn.rollout(s, acts, p)[-1]
    b = odyn.rollout(pert, acts, p)[-1]
    return float((np.abs(a - b) / np.maximum(1.0, np.abs(a))).max())


DYN_VARIANTS = ["ctbr_forest", "rk4_nsub4", "quad_drag", "srt", "euler_nsub4", "hover", "ps", "lv",
                "ps_euler_nsub2"]


def _variant_params(variant):
    if variant == "srt":
        return default_params(ctrl=odyn.SRT)
    if variant == "euler_nsub4":
        return default_params(integrator=odyn.EULER, n_sub=4)
    if variant == "rk4_nsub4":
        return default_params(n_sub=4)
    if variant == "quad_drag":
        # Eq. 2 with both terms: anisotropic quadratic coefficients (N s^2 / m^2) beside the linear ones
        return default_params(c_quad=(0.04, 0.06, 0.1))
    if variant == "ps":
        return default_params(ctrl=odyn.PS)
    if variant == "ps_euler_nsub2":
        return default_params(ctrl=odyn.PS, integrator=odyn.EULER, n_sub=2)
    if variant == "lv":
        return default_params(ctrl=odyn.LV)
    return default_params()


def _component_name(j):
    names = ["px", "py", "pz", "qw", "qx", "qy", "qz", "vx", "vy", "vz", "wx", "wy", "wz", "r0", "r1", "r2", "r3"]
    return names[j]


def _worst(s_gpu, s_ref):
    err = np.abs(np.asarray(s_gpu, np.float64) - s_ref) / np.maximum(1.0, np.abs(s_ref))
    i, j = np.unravel_index(int(np.argmax(err)), err.shape)
    return float(err[i, j]), int(i), _component_name(int(j))


@pytest.mark.parametrize("variant", DYN_VARIANTS)
def test_dynamics_batch_variants(vf, variant):
    """Local parity (the oracle stepped from every GPU state) at 1e-5 for every variant.  100-step
    trajectories at 1e-5 for the CTBR/RK4 configurations (one and four sub-steps, with and without
    quadratic drag); the open-loop SRT and the closed-loop Euler, PS and LV variants within 32x the
    oracle's own growth of a one-ulp start perturbation (their conditioning), never below 1e-5.  Every
    variant's errors, bounds and worst component are recorded."""
    sim, ctx = vf
    p = _variant_params(variant)
    forest = scenes.forest(seed=3, n_trees=300)
    n = 200
    s0 = agents.forest_starts(4, n, forest, p)
    rng = np.random.default_rng(12)
    if variant == "srt":
        # single-rotor thrusts around hover (+-10 %); open loop, so the attitude random-walks
        rng = np.random.default_rng(9)
        f_hover = p["mass"] * p["g"] / 4
        acts = (f_hover * rng.uniform(0.9, 1.1, size=(100, n, 4))).astype(np.float32)
    elif variant == "hover":
        acts = np.tile(np.array([p["g"], 0, 0, 0], dtype=np.float32), (100, n, 1))
    elif variant.startswith("ps"):
        # step commands: a goal within 3 m per axis and a yaw, held for 50 steps, then a second one
        goal = np.concatenate([s0[:, 0:3] + rng.uniform(-3, 3, (n, 3)), rng.uniform(-np.pi, np.pi, (n, 1))], 1)
        goal2 = np.concatenate([goal[:, 0:3] + rng.uniform(-3, 3, (n, 3)), rng.uniform(-np.pi, np.pi, (n, 1))], 1)
        acts = np.concatenate([np.tile(goal, (50, 1, 1)), np.tile(goal2, (50, 1, 1))]).astype(np.float32)
    elif variant == "lv":
        cmd = np.concatenate([rng.uniform(-2, 2, (4, n, 3)), rng.uniform(-np.pi, np.pi, (4, n, 1))], 2)
        acts = np.repeat(cmd, 25, axis=0).astype(np.float32)
    else:
        acts = agents.random_actions(5, 100, n, p)
    header(f"dynamics: {variant}, {n} agents x 100 steps")
    gpu = _gpu_rollout(ctx, p, s0, acts)
    pd = device_params(p)      # the oracle runs on the float32 parameter values the device receives
    local, local_at = 0.0, None
    for k in range(100):
        e, i, comp = _worst(gpu[k + 1], odyn.step(gpu[k].astype(np.float64), acts[k], pd))
        if e > local:
            local, local_at = e, (k, i, comp)
    ref = odyn.rollout(s0, acts, pd)
    err, err_at = 0.0, None
    for k in range(101):
        e, i, comp = _worst(gpu[k], ref[k])
        if e > err:
            err, err_at = e, (k, i, comp)
    tol = STATE_TOL
    if variant not in ("ctbr_forest", "hover", "rk4_nsub4", "quad_drag"):
        tol = max(STATE_TOL, 32 * _rounding_amplification(s0, acts, pd))
    speed = float(np.linalg.norm(ref[:, :, 7:10], axis=2).max())
    record(f"dynamics[{variant}]", one_step=local, one_step_bound=STATE_TOL, one_step_worst=local_at,
           trajectory=err, trajectory_bound=tol, trajectory_worst=err_at, max_speed=speed)
    assert local <= STATE_TOL, f"{variant}: one-step error {local:.3e} at {local_at}"
    assert err <= tol, f"{variant}: max state error {err:.3e} (bound {tol:.3e}) at {err_at}"
    if variant == "hover":
        assert np.abs(gpu[-1][:, 0:3] - s0[:, 0:3]).max() <= 1e-5
    if variant == "quad_drag":
        # the quadratic term is exercised: body speeds where c |v| v is comparable to the linear term
        assert speed > 5.0


def test_dynamics_env_idx_and_n0(vf):
    """Resident slots: only the listed rows change; n = 0 is a no-op."""
    sim, ctx = vf
    p = default_params()
    s = agents.make_states(np.arange(30).reshape(10, 3), p)
    st = _dev(s)
    idx = torch.tensor([7, 2, 5], dtype=torch.int32).cuda()
    a = agents.random_actions(1, 1, 3, p)[0]
    ctx.step(p, st, _dev(a), env_idx=idx)
    got = st.cpu().numpy()
    ref = odyn.step(s[[7, 2, 5]], a, device_params(p))
    for j, row in enumerate([7, 2, 5]):
        assert state_close(got[row], ref[j]) <= 1e-6
    untouched = [i for i in range(10) if i not in (7, 2, 5)]
    assert np.array_equal(got[untouched], s[untouched])
    ctx.step(p, st, torch.zeros((0, 4), dtype=torch.float32).cuda())
    assert np.array_equal(st.cpu().numpy(), got)


# ---------------------------------------------------------------------------
# render
# ---------------------------------------------------------------------------

def _render(ctx, sim, sid, states, hw=(64, 64), hfov=math.pi / 2, with_rgb=True):
    n = states.shape[0]
    views, npx, offs, mh, mw = sim.make_views(n, sid, hw, hfov=hfov)
    depth = torch.full((npx,), -7.0, dtype=torch.float32).cuda()
    ids = torch.full((npx,), -9, dtype=torch.int32).cuda()
    rgb = torch.zeros((3 * npx,), dtype=torch.uint8).cuda() if with_rgb else None
    ctx.render(_dev(states), views, max_hw=(mh, mw), depth=depth, tri_id=ids, rgb=rgb, out_pixels=npx)
    ctx.sync_check()
    return depth.cpu().numpy(), ids.cpu().numpy(), (rgb.cpu().numpy() if with_rgb else None), offs


def _check_agents(scene, states, depth, ids, rgb, offs, hw, hfov=math.pi / 2, label="", far=100.0):
    h, w = hw
    fr = []
    for i in range(states.shape[0]):
        o = offs[i]
        ref = oren.render_view(states[i].astype(np.float64), scene, h, w, hfov)
        px = slice(o, o + h * w)
        rgb_i = None if rgb is None else np.stack([rgb[3 * o + c * h * w: 3 * o + (c + 1) * h * w] for c in range(3)])
        fr.append(compare_render(depth[px], ids[px], rgb_i, ref, far, f"{label} agent {i}"))
    return fr


def test_render_box_room_random_poses(vf):
    sim, ctx = vf
    p = default_params()
    sc = scenes.box_room(seed=1)
    sid = ctx.build_scene(sc["verts"], sc["tris"], sc["rgb"])
    rng = np.random.default_rng(21)
    n = 12
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    states = agents.make_states(rng.uniform([0.5, 0.5, 0.3], [9.5, 9.5, 3.7], size=(n, 3)), p, quat=q)
    header("render: box room, 12 random poses, 64x64")
    depth, ids, rgb, offs = _render(ctx, sim, sid, states)
    fr = _check_agents(sc, states, depth, ids, rgb, offs, (64, 64), label="box room")
    assert np.mean(fr) < 0.01, f"masked fraction {np.mean(fr):.4f}"
    assert (ids >= 0).mean() > 0.99    # the room is closed
    ctx.free_scene(sid)


def test_render_forest_full_frames(vf):
    sim, ctx = vf
    p = default_params()
    sc = scenes.forest(seed=3)
    sid = ctx.build_scene(sc["verts"], sc["tris"], sc["rgb"])
    states = agents.forest_starts(4, 3, sc, p)
    header("render: forest (128,002 triangles), 3 agents, 64x64, brute-force oracle")
    depth, ids, rgb, offs = _render(ctx, sim, sid, states)
    fr = _check_agents(sc, states, depth, ids, rgb, offs, (64, 64), label="forest")
    assert np.mean(fr) < 0.01, f"masked fraction {np.mean(fr):.4f}"
    ctx.free_scene(sid)


def test_render_ragged_sizes_and_fov(vf):
    """Image sizes that are not multiples of the 16x4 packet, non-square, other fields of view."""
    sim, ctx = vf
    p = default_params()
    sc = scenes.box_room(seed=4)
    sid = ctx.build_scene(sc["verts"], sc["tris"], sc["rgb"])
    rng = np.random.default_rng(5)
    for hw, fov in (((13, 29), 1.2), ((60, 44), 2.0), ((1, 1), 0.5), ((96, 96), math.pi / 2)):
        q = rng.normal(size=(3, 4))
        q /= np.linalg.norm(q, axis=1, keepdims=True)
        states = agents.make_states(rng.uniform([1, 1, 0.5], [9, 9, 3.5], size=(3, 3)), p, quat=q)
        header(f"render: ragged {hw} hfov {fov}")
        depth, ids, rgb, offs = _render(ctx, sim, sid, states, hw=hw, hfov=fov)
        fr = _check_agents(sc, states, depth, ids, rgb, offs, hw, hfov=fov, label=f"{hw}")
        assert np.mean(fr) < 0.05
    ctx.free_scene(sid)


def _adversarial_scene():
    """Shared edges, a coplanar duplicate, zero-area triangles, a T-junction, a fan around one vertex."""
    v = []
    t = []

    def quad(a, b, c, d):
        base = len(v)
        v.extend([a, b, c, d])
        t.append((base, base + 1, base + 2))
        t.append((base, base + 2, base + 3))
    quad((4, -2, -2), (4, 2, -2), (4, 2, 2), (4, -2, 2))                    # wall split on a diagonal
    t.append(t[0])                                                          # coplanar duplicate
    base = len(v)
    v.extend([(3, 0, 0), (3, 1, 1), (3, 2, 2)])                             # zero-area (collinear)
    t.append((base, base + 1, base + 2))
    base = len(v)
    v.extend([(3.5, -1, -1), (3.5, -1, -1), (3.5, 0.5, 0.2)])               # zero-area (repeated vertex)
    t.append((base, base + 1, base + 2))
    base = len(v)
    c0 = (2.5, -0.5, 0.5)
    v.append(c0)
    for k in range(7):                                                      # fan: 6 triangles share vertex c0
        ang = 2 * math.pi * k / 6
        v.append((2.5, -0.5 + 0.6 * math.cos(ang), 0.5 + 0.6 * math.sin(ang)))
    for k in range(6):
        t.append((base, base + 1 + k, base + 2 + k))
    base = len(v)
    v.extend([(3.0, 0.0, -1.5), (3.0, 1.5, -1.5), (3.0, 0.75, -0.25)])      # T-junction neighbours
    t.append((base, base + 1, base + 2))
    v.extend([(3.0, 0.75, -0.25), (3.0, 1.5, -1.5), (3.0, 1.5, 0.0)])
    t.append((base + 3, base + 4, base + 5))
    base = len(v)
    v.extend([(1.0, -3.0, 0.0), (6.0, -3.0, 0.0), (6.0, 3.0, 0.0)])          # plane containing the camera
    t.append((base, base + 1, base + 2))
    verts = np.asarray(v, dtype=np.float32)
    tris = np.asarray(t, dtype=np.int32)
    rgb = np.random.default_rng(0).integers(0, 256, size=(len(t), 3)).astype(np.uint8)
    return {"verts": verts, "tris": tris, "rgb": rgb}


def test_render_adversarial_tiny_scene(vf):
    sim, ctx = vf
    p = default_params()
    sc = _adversarial_scene()
    sid = ctx.build_scene(sc["verts"], sc["tris"], sc["rgb"])
    rng = np.random.default_rng(8)
    poses = [agents.make_states([[0.0, 0.0, 0.0]], p)[0],                         # on the plane z = 0
             agents.make_states([[0.0, 0.3, 0.2]], p)[0],
             agents.make_states([[0.5, -0.5, 0.5]], p, quat=agents.yaw_quat([0.1]))[0]]
    for _ in range(5):
        q = np.array([1.0, *rng.normal(scale=0.2, size=3)])
        poses.append(agents.make_states([rng.uniform([-1, -1, -1], [1, 1, 1])], p, quat=q / np.linalg.norm(q))[0])
    states = np.stack(poses)
    header("render: adversarial tiny scene (shared edges, duplicates, degenerate, fan, camera on a plane)")
    depth, ids, rgb, offs = _render(ctx, sim, sid, states, hw=(40, 40), hfov=1.3)
    fr = _check_agents(sc, states, depth, ids, rgb, offs, (40, 40), hfov=1.3, label="adversarial")
    assert np.mean(fr) < 0.2
    ctx.free_scene(sid)


def test_single_triangle_and_single_leaf_scenes(vf):
    sim, ctx = vf
    p = default_params()
    for n_tri in (1, 3, 4, 5):
        base = scenes.icosphere(radius=1.0, subdiv=0, center=(3.0, 0.0, 0.0))
        sc = {"verts": base["verts"], "tris": base["tris"][:n_tri], "rgb": base["rgb"][:n_tri]}
        sid = ctx.build_scene(sc["verts"], sc["tris"], sc["rgb"])
        states = agents.make_states([[0.0, 0.0, 0.0]], p)
        depth, ids, rgb, offs = _render(ctx, sim, sid, states, hw=(24, 24), hfov=1.0)
        _check_agents(sc, states, depth, ids, rgb, offs, (24, 24), hfov=1.0, label=f"{n_tri} tris")
        ctx.free_scene(sid)


# ---------------------------------------------------------------------------
# fused step + render
# ---------------------------------------------------------------------------

def test_fused_step_render_equals_split_and_oracle(vf):
    """vf_step with views == vf_step without views followed by vf_render, bitwise; and parity at step 10."""
    sim, ctx = vf
    p = default_params()
    sc = scenes.forest(seed=3, n_trees=400)
    sid = ctx.build_scene(sc["verts"], sc["tris"], sc["rgb"])
    n = 40
    s0 = agents.forest_starts(4, n, sc, p)
    acts = agents.random_actions(5, 10, n, p)
    views, npx, offs, mh, mw = sim.make_views(n, sid, (64, 64))
    st_f, st_s = _dev(s0), _dev(s0)
    d_f = torch.zeros(npx).cuda()
    d_s = torch.zeros(npx).cuda()
    i_f = torch.zeros(npx, dtype=torch.int32).cuda()
    i_s = torch.zeros(npx, dtype=torch.int32).cuda()
    c_f = torch.zeros(3 * npx, dtype=torch.uint8).cuda()
    c_s = torch.zeros(3 * npx, dtype=torch.uint8).cuda()
    header("fused vs split: 40 agents x 10 steps")
    for k in range(10):
        a = _dev(acts[k])
        ctx.set_launch_mode(True)
        ctx.step(p, st_f, a, views=views, max_hw=(mh, mw), depth=d_f, tri_id=i_f, rgb=c_f, out_pixels=npx)
        ctx.set_launch_mode(False)
        ctx.step(p, st_s, a)
        ctx.render(st_s, views, max_hw=(mh, mw), depth=d_s, tri_id=i_s, rgb=c_s, out_pixels=npx)
        assert torch.equal(st_f, st_s), f"state differs at step {k}"
        assert torch.equal(d_f, d_s) and torch.equal(i_f, i_s) and torch.equal(c_f, c_s), f"image differs at {k}"
    ctx.sync_check()
    ref = odyn.rollout(s0, acts, device_params(p))
    assert state_close(st_f.cpu().numpy(), ref[-1]) <= STATE_TOL
    states = st_f.cpu().numpy()
    fr = _check_agents(sc, states[:6], d_f.cpu().numpy(), i_f.cpu().numpy(), c_f.cpu().numpy(), offs, (64, 64),
                       label="fused")
    assert np.mean(fr) < 0.01
    ctx.free_scene(sid)


def test_fused_in_place_with_env_slots(vf):
    """Resident slots with the fused kernel: rows updated in place once, untouched rows unchanged."""
    sim, ctx = vf
    p = default_params()
    sc = scenes.box_room(seed=1)
    sid = ctx.build_scene(sc["verts"], sc["tris"], sc["rgb"])
    slots = agents.make_states(np.tile([5.0, 5.0, 2.0], (16, 1)) + np.arange(16)[:, None] * 0.05, p)
    st = _dev(slots)
    idx = np.array([3, 11, 0, 7], dtype=np.int32)
    a = agents.random_actions(3, 1, 4, p)[0]
    views, npx, offs, mh, mw = sim.make_views(4, sid, (128, 128))
    depth = torch.zeros(npx).cuda()
    ctx.set_launch_mode(True)
    ctx.step(p, st, _dev(a), views=views, env_idx=torch.as_tensor(idx).cuda(), max_hw=(mh, mw), depth=depth,
             out_pixels=npx)
    ctx.sync_check()
    got = st.cpu().numpy()
    ref = odyn.step(slots[idx], a, device_params(p))
    assert state_close(got[idx], ref) <= 1e-6
    rest = [i for i in range(16) if i not in idx]
    assert np.array_equal(got[rest], slots[rest])
    # a second call from the updated rows (counters were reset by the last arriving workgroup)
    ctx.step(p, st, _dev(a), views=views, env_idx=torch.as_tensor(idx).cuda(), max_hw=(mh, mw), depth=depth,
             out_pixels=npx)
    ctx.sync_check()
    ref2 = odyn.step(ref, a, device_params(p))
    assert state_close(st.cpu().numpy()[idx], ref2) <= 1e-6
    ctx.set_launch_mode(False)
    ctx.step(p, st, _dev(a), views=views, env_idx=torch.as_tensor(idx).cuda(), max_hw=(mh, mw), depth=depth,
             out_pixels=npx)
    ctx.sync_check()
    assert state_close(st.cpu().numpy()[idx], odyn.step(ref2, a, device_params(p))) <= 1e-6
    ctx.free_scene(sid)


# ---------------------------------------------------------------------------
# multi-scene, mixed resolution
# ---------------------------------------------------------------------------

def test_multi_scene_mixed_resolution(vf):
    sim, ctx = vf
    p = default_params()
    scs = [scenes.room_graph(600, 20000), scenes.room_graph(601, 60000), scenes.box_room(seed=2)]
    sids = [ctx.build_scene(s["verts"], s["tris"], s["rgb"]) for s in scs]
    rng = np.random.default_rng(12)
    which = rng.integers(0, 3, size=9)
    states = []
    for j in which:
        if j < 2:
            states.append(agents.room_graph_starts(int(rng.integers(1 << 30)), 1, scs[j], p)[0])
        else:
            states.append(agents.make_states([[5, 5, 2]], p, quat=agents.yaw_quat([rng.uniform(-3, 3)]))[0])
    states = np.stack(states)
    hw = np.array([(64, 64), (128, 128), (96, 96)])[rng.integers(0, 3, size=9)]
    views, npx, offs, mh, mw = sim.make_views(9, np.array(sids)[which], hw)
    depth = torch.zeros(npx).cuda()
    ids = torch.zeros(npx, dtype=torch.int32).cuda()
    header("multi-scene: 3 scenes, 9 agents, 64/96/128")
    ctx.render(_dev(states), views, max_hw=(mh, mw), depth=depth, tri_id=ids, out_pixels=npx)
    ctx.sync_check()
    d, i = depth.cpu().numpy(), ids.cpu().numpy()
    for a in range(9):
        h, w = hw[a]
        ref = oren.render_view(states[a].astype(np.float64), scs[which[a]], h, w, math.pi / 2)
        px = slice(offs[a], offs[a] + h * w)
        compare_render(d[px], i[px], None, ref, 100.0, f"agent {a}")
    for s in sids:
        ctx.free_scene(s)


def test_spatial_order_changes_nothing(vf):
    """The (scene, position) render order of large batches moves work between workgroups only:
    split steps and renders with and without it are bitwise equal, over two scenes, env slots and
    mixed sizes; every output pixel is written."""
    sim, ctx = vf
    p = default_params()
    scs = [scenes.forest(seed=3, n_trees=300), scenes.box_room(seed=1)]
    sids = [ctx.build_scene(s["verts"], s["tris"], s["rgb"]) for s in scs]
    rng = np.random.default_rng(77)
    n, n_slots = 300, 340
    s0 = np.concatenate([agents.forest_starts(9, n_slots - 40, scs[0], p),
                         agents.make_states(rng.uniform([1, 1, 1], [9, 9, 3], (40, 3)), p)])
    env = rng.permutation(n_slots)[:n].astype(np.int32)
    which = (env >= n_slots - 40).astype(np.int64)
    hw = np.array([(64, 64), (40, 24)])[rng.integers(0, 2, n)]
    views, npx, offs, mh, mw = sim.make_views(n, np.array(sids)[which], hw)
    acts = _dev(agents.random_actions(3, 1, n, p)[0])
    env_t = torch.as_tensor(env).cuda()
    outs = []
    header("spatial order on/off: 300 agents, 2 scenes")
    ctx.set_cost_order(False)       # launches put in cost order skip the spatial order
    for on in (True, False):
        ctx.set_spatial_order(on)
        ctx.set_launch_mode(False)
        st = _dev(s0)
        depth = torch.full((npx,), float("nan")).cuda()
        ids = torch.full((npx,), -7, dtype=torch.int32).cuda()
        rgb = torch.zeros(3 * npx, dtype=torch.uint8).cuda()
        ctx.step(p, st, acts, views=views, env_idx=env_t, max_hw=(mh, mw), depth=depth, tri_id=ids, rgb=rgb,
                 out_pixels=npx)
        d2 = torch.full((npx,), float("nan")).cuda()
        ctx.render(st, views, n=n, env_idx=env_t, max_hw=(mh, mw), depth=d2, out_pixels=npx)
        ctx.sync_check()
        outs.append([t.cpu().numpy() for t in (st, depth, ids, rgb, d2)])
    ctx.set_spatial_order(True)
    ctx.set_cost_order(True)
    ctx.set_launch_mode(None)
    for a, b in zip(outs[0], outs[1]):
        assert np.array_equal(a, b, equal_nan=False)
    assert not np.isnan(outs[0][1]).any() and not (outs[0][2] == -7).any()
    # spot-check a few agents against the oracle
    for a in (0, 137, 299):
        h, w = hw[a]
        ref = oren.render_view(outs[0][0][env[a]].astype(np.float64), scs[which[a]], h, w, math.pi / 2)
        px = slice(offs[a], offs[a] + h * w)
        compare_render(outs[0][1][px], outs[0][2][px], None, ref, 100.0, f"agent {a}")
    for sid in sids:
        ctx.free_scene(sid)


def test_step_with_cost_order_changes_nothing(vf):
    """vf_step's split launches run the dynamics and the cost order in one launch (k_step_order): four steps
    of 2,100 agents on permuted env slots of a larger table (the sort runs in two chunks per XCD) give the
    same states, depth and ids with the order on and off."""
    sim, ctx = vf
    p = default_params()
    sc = scenes.forest(seed=3, n_trees=300)
    sid = ctx.build_scene(sc["verts"], sc["tris"], sc["rgb"])
    n, slots, steps = 2100, 2600, 4
    rng = np.random.default_rng(91)
    table = agents.forest_starts(91, slots, sc, p)
    idx = rng.permutation(slots)[:n].astype(np.int32)
    acts = agents.random_actions(92, steps, n, p)
    views, npx, offs, mh, mw = sim.make_views(n, sid, (64, 64))
    header(f"step with cost order on/off: {n} agents on {slots} slots, {steps} steps")
    outs = {}
    try:
        ctx.set_launch_mode(False)
        for on in (True, False):
            ctx.set_cost_order(on)
            st = _dev(table)
            depth = torch.full((npx,), float("nan")).cuda()
            ids = torch.full((npx,), -7, dtype=torch.int32).cuda()
            for k in range(steps):
                ctx.step(p, st, _dev(acts[k]), views=views, env_idx=_dev(idx, torch.int32), max_hw=(mh, mw),
                         depth=depth, tri_id=ids, out_pixels=npx)
            ctx.sync_check()
            outs[on] = (st.cpu().numpy(), depth.cpu().numpy(), ids.cpu().numpy())
    finally:
        ctx.set_cost_order(True)
        ctx.set_launch_mode(None)
    for a, b in zip(outs[True], outs[False]):
        assert np.array_equal(a, b)
    assert not np.isnan(outs[True][1]).any() and not (outs[True][2] == -7).any()
    untouched = np.setdiff1d(np.arange(slots), idx)
    assert np.array_equal(outs[True][0][untouched], table[untouched])
    ctx.free_scene(sid)


def test_cost_order_changes_nothing(vf):
    """Longest-first workgroup order (from the work the previous launch of the same shape reported)
    moves packets between workgroups only: repeated renders with it on and off, with launches of other
    shapes in between, one sorted in two chunks per XCD and one too large for the order kernel (4,100 views
    on a 128 x 128 grid: 1,049,600 workgroups), are bitwise equal and write every pixel."""
    sim, ctx = vf
    p = default_params()
    sc = scenes.forest(seed=3, n_trees=300)
    sid = ctx.build_scene(sc["verts"], sc["tris"], sc["rgb"])
    rng = np.random.default_rng(78)
    outs = {}
    header("cost order on/off: 300, 120, 2,100 and 4,100 agents, mixed sizes")
    for n in (300, 120, 2100, 4100):
        s0 = _dev(agents.forest_starts(10 + n, n, sc, p))
        hw = np.array([(64, 64), (40, 24)])[rng.integers(0, 2, n)]
        hw[0] = (64, 64)
        if n == 4100:
            hw[:] = (40, 24)
            hw[0] = (128, 128)
        views, npx, offs, mh, mw = sim.make_views(n, sid, hw)
        for on in (True, False):
            ctx.set_cost_order(on)
            runs = []
            for rep in range(3):
                depth = torch.full((npx,), float("nan")).cuda()
                ids = torch.full((npx,), -7, dtype=torch.int32).cuda()
                ctx.render(s0, views, n=n, max_hw=(mh, mw), depth=depth, tri_id=ids, out_pixels=npx)
                if n == 300 and rep == 1:
                    # a launch of another shape on the same stream between two of the same shape
                    d_small = torch.empty(20 * 64 * 64, device="cuda")
                    v20, _, _, _, _ = sim.make_views(20, sid, (64, 64))
                    ctx.render(s0, v20, n=20, max_hw=(64, 64), depth=d_small, out_pixels=20 * 64 * 64)
                ctx.sync_check()
                runs.append((depth.cpu().numpy(), ids.cpu().numpy()))
            outs[(n, on)] = runs
        ctx.set_cost_order(True)
        ref_d, ref_i = outs[(n, False)][0]
        assert not np.isnan(ref_d).any() and not (ref_i == -7).any()
        for on in (True, False):
            for d_, i_ in outs[(n, on)]:
                assert np.array_equal(d_, ref_d) and np.array_equal(i_, ref_i), f"n={n} cost order {on}"
        # spot-check against the oracle
        st_np = s0.cpu().numpy()
        for a in (1, n // 2):
            h, w = hw[a]
            ref = oren.render_view(st_np[a].astype(np.float64), sc, h, w, math.pi / 2)
            px = slice(offs[a], offs[a] + h * w)
            compare_render(ref_d[px], ref_i[px], None, ref, 100.0, f"n={n} agent {a}")
    ctx.free_scene(sid)


# ---------------------------------------------------------------------------
# BVH invariants
# ---------------------------------------------------------------------------

def _check_bvh(ctx, sid, sc):
    """Structural invariants of a built scene; returns the exported (nodes, tris)."""
    nodes, tris = ctx.export_scene(sid)
    info = ctx.scene_info(sid)
    T = sc["tris"].shape[0]
    # every triangle appears exactly once, with its own vertices
    assert np.array_equal(np.sort(tris["id"]), np.arange(T))
    v = sc["verts"].astype(np.float64)
    t = sc["tris"]
    assert np.array_equal(tris["v0"], sc["verts"][t[tris["id"], 0]])
    # leaves cover [0, T) exactly once; child boxes lie inside the parent's slot box
    covered = np.zeros(T, dtype=np.int64)
    lo = np.stack([nodes["lo_x"], nodes["lo_y"], nodes["lo_z"]], -1)
    hi = np.stack([nodes["hi_x"], nodes["hi_y"], nodes["hi_z"]], -1)
    width = info["width"]
    assert width in (4, 8) and nodes["child"].shape[1] == width
    empty = -2 ** 31
    for ni in range(len(nodes)):
        for k in range(width):
            c = int(nodes["child"][ni, k])
            if c >= 0:
                assert c > ni
                valid = nodes["child"][c] != empty
                assert np.all(lo[c][valid] >= lo[ni, k]) and np.all(hi[c][valid] <= hi[ni, k])
            elif c != empty:
                f, cnt = (-c - 1) >> 3, ((-c - 1) & 7) + 1
                if width == 4:
                    assert nodes["count"][ni, k] == cnt
                covered[f:f + cnt] += 1
                ids = tris["id"][f:f + cnt]
                tv = v[t[ids]].reshape(-1, 3)
                assert np.all(tv >= lo[ni, k]) and np.all(tv <= hi[ni, k])
            else:                            # an empty slot's box never meets a ray
                assert np.all(lo[ni, k] > 1e37) and np.all(hi[ni, k] > 1e37)
        # every octant's order is a permutation of the slots
        if width == 4:
            words = nodes["order"][ni]
            packed = int(words[0]) | (int(words[1]) << 32)
            perms = [[(packed >> (8 * o + 2 * i)) & 3 for i in range(4)] for o in range(8)]
        else:
            perms = [[(int(nodes["order"][ni, o]) >> (3 * i)) & 7 for i in range(8)] for o in range(8)]
        for perm in perms:
            assert sorted(perm) == list(range(width))
    assert np.all(covered == 1)
    # root bounds contain the scene
    valid0 = nodes["child"][0] != empty
    assert np.all(lo[0][valid0].min(0) <= v.min(0)) and np.all(hi[0][valid0].max(0) >= v.max(0))
    assert info["depth"] >= 2 and info["n_nodes"] == len(nodes)
    return nodes, tris


def test_bvh_invariants_and_deterministic_rebuild(vf):
    sim, ctx = vf
    sc = scenes.forest(seed=3, n_trees=500)
    sid = ctx.build_scene(sc["verts"], sc["tris"], sc["rgb"])
    nodes, tris = _check_bvh(ctx, sid, sc)
    assert ctx.scene_info(sid)["builder"] == "cluster"
    sid2 = ctx.build_scene(sc["verts"], sc["tris"], sc["rgb"])
    nodes2, tris2 = ctx.export_scene(sid2)
    assert nodes.tobytes() == nodes2.tobytes() and tris.tobytes() == tris2.tobytes()
    ctx.free_scene(sid)
    ctx.free_scene(sid2)


def test_bvh_builders_and_leaf_sizes_agree(vf):
    """The clustered and the radix-tree BVH of the same scene, and leaves of 1 to 4 triangles: all valid,
    and the same images bit for bit (the closest hit does not depend on the tree; ties go to the lower id
    either way)."""
    sim, ctx = vf
    p = default_params()
    configs = (("radix", 4), ("cluster", 4), ("cluster", 3), ("cluster", 1), ("radix", 2))
    for name, sc in (("forest", scenes.forest(seed=3, n_trees=500)), ("room graph", scenes.room_graph(7, 20000))):
        if name == "forest":
            states = agents.forest_starts(4, 6, sc, p)
        else:
            states = agents.room_graph_starts(8, 6, sc, p)
        outs = {}
        for builder, leaf in configs:
            ctx.set_bvh_builder(builder)
            ctx.set_bvh_leaf_size(leaf)
            sid = ctx.build_scene(sc["verts"], sc["tris"], sc["rgb"])
            info = ctx.scene_info(sid)
            assert info["builder"] == builder and info["leaf_max"] == leaf
            header(f"BVH builds: {name}, {builder} tree, leaves of <= {leaf}")
            nodes, _ = _check_bvh(ctx, sid, sc)
            c = nodes["child"]
            leaf_c = c[(c < 0) & (c != -2 ** 31)]
            assert (((-leaf_c.astype(np.int64) - 1) & 7) + 1).max() <= leaf
            outs[(builder, leaf)] = _render(ctx, sim, sid, states)
            ctx.free_scene(sid)
        ref = outs[configs[0]]
        for key in configs[1:]:
            for a, b in zip(ref[:3], outs[key][:3]):
                assert np.array_equal(a, b), f"{name}: images differ between {configs[0]} and {key}"
        fr = _check_agents(sc, states[:2], *outs[("cluster", 4)], (64, 64), label=f"{name} cluster")
        assert np.mean(fr) < 0.02
    ctx.set_bvh_builder("cluster")
    ctx.set_bvh_leaf_size(4)
    with pytest.raises(Exception):
        ctx.set_bvh_leaf_size(5)
    with pytest.raises(Exception):
        ctx.set_bvh_leaf_size(0)


def test_duplicate_geometry_builds_balanced(vf):
    """Thousands of identical triangles (duplicated geometry): the clustering pairs identical boxes off in a
    logarithmic number of passes (no fallback, shallow tree, fast build), and the duplicates resolve to the
    lowest caller id on every pixel that sees them."""
    sim, ctx = vf
    p = default_params()
    floor = scenes.floor_quad(half=20.0, z=-1.0)
    one = scenes.plane_quad((4.0, -1.0, -0.5), (0.0, 2.0, 0.0), (0.0, 0.0, 2.0))
    n_dup = 20000
    verts = np.concatenate([floor["verts"], one["verts"]]).astype(np.float32)
    tris = np.concatenate([floor["tris"], np.tile(one["tris"][:1] + 4, (n_dup, 1))]).astype(np.int32)
    rgb = np.concatenate([floor["rgb"], np.tile(one["rgb"][:1], (n_dup, 1))]).astype(np.uint8)
    sc = {"verts": verts, "tris": tris, "rgb": rgb}
    sid = ctx.build_scene(verts, tris, rgb)
    info = ctx.scene_info(sid)
    header(f"duplicate geometry: {n_dup} identical triangles, build {info['build_ms']:.2f} ms, depth {info['depth']}")
    assert info["builder"] == "cluster" and info["depth"] <= 16
    assert info["build_ms"] < 50.0
    _check_bvh(ctx, sid, sc)
    states = agents.make_states([[0.0, 0.0, 0.0]], p)
    depth, ids, rgb_out, offs = _render(ctx, sim, sid, states, hw=(32, 32), hfov=1.2)
    ref = oren.render_view(states[0].astype(np.float64), sc, 32, 32, 1.2)
    # every duplicate pixel is an exact tie (masked by the oracle); the GPU must resolve all of them to the
    # lowest id, 2, and see the duplicated triangle on about as many pixels
    dup_ref = int((ref["id"].reshape(-1) >= 2).sum())
    dup_gpu = ids >= 2
    assert dup_ref > 50 and np.all(ids[dup_gpu] == 2)
    assert abs(int(dup_gpu.sum()) - dup_ref) <= 0.1 * dup_ref
    compare_render(depth, ids, None, ref, 100.0, "duplicates")      # everything off the mask
    ctx.free_scene(sid)


def _chain_scene(n, ratio=2.2, half=0.5, seed=12):
    """n equal triangles facing a camera at the origin, centred on its axis at x = ratio^k.  For ratio > 2
    the cheapest merge of triangle k is with the cluster of all nearer ones, and of that cluster with k,
    so the clustering merges one pair per pass: a chain, as deep as a BVH of n leaves can be.  A ray
    along the axis enters every box of it."""
    verts, tris = [], []
    for k in range(n):
        x = ratio ** k
        verts += [(x, -half, -half), (x, half, -half), (x, 0.0, half)]
        tris.append((3 * k, 3 * k + 1, 3 * k + 2))
    rgb = np.random.default_rng(seed).integers(0, 256, (n, 3))
    return {"verts": np.asarray(verts, dtype=np.float32), "tris": np.asarray(tris, dtype=np.int32),
            "rgb": rgb.astype(np.uint8)}


SHALLOW_DEPTH = 21    # deepest 4-wide BVH whose walk fits one 64-lane stack register: 3 (d - 1) + 4 <= 64


def test_deep_bvh_takes_the_two_register_stack(vf):
    """A BVH deeper than one stack register holds is rendered right (against the oracle), and while it is
    resident every launch takes the two-register stack: another scene renders to the same bits as with
    only shallow scenes resident, before and after the deep scene is freed."""
    sim, ctx = vf
    p = default_params()
    room = scenes.box_room(seed=1)
    sid_room = ctx.build_scene(room["verts"], room["tris"], room["rgb"])
    rng = np.random.default_rng(21)
    q = rng.normal(size=(6, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    poses = agents.make_states(rng.uniform([2, 2, 1], [8, 8, 3], (6, 3)), p, quat=q)
    shallow = _render(ctx, sim, sid_room, poses)
    ctx.set_bvh_leaf_size(1)
    sid = None
    try:
        for n in (75, 90, 105):
            sc = _chain_scene(n)
            sid = ctx.build_scene(sc["verts"], sc["tris"], sc["rgb"])
            depth_n = ctx.scene_info(sid)["depth"]
            if depth_n > SHALLOW_DEPTH:
                break
            ctx.free_scene(sid)
            sid = None
        header(f"deep BVH: {n} chained triangles, depth {depth_n}")
        assert sid is not None, f"no chain scene built deeper than {SHALLOW_DEPTH} levels (last: {depth_n})"
        # the far plane beyond the chain's last triangle, so the packet walks the whole chain
        far = 1e30
        cam = agents.make_states([[0.0, 0.0, 0.0]], p)
        views, npx, offs, mh, mw = sim.make_views(1, sid, (48, 48), far=far)
        depth_t = torch.full((npx,), -7.0, dtype=torch.float32).cuda()
        ids_t = torch.full((npx,), -9, dtype=torch.int32).cuda()
        ctx.render(_dev(cam), views, max_hw=(mh, mw), depth=depth_t, tri_id=ids_t, out_pixels=npx)
        ctx.sync_check()
        ref = oren.render_view(cam[0].astype(np.float64), sc, 48, 48, math.pi / 2, far=far)
        ids = ids_t.cpu().numpy()
        assert (ids >= 0).sum() > 200
        compare_render(depth_t.cpu().numpy(), ids, None, ref, far, "deep chain")
        deep = _render(ctx, sim, sid_room, poses)
        for a, b in zip(shallow[:3], deep[:3]):
            assert np.array_equal(a, b), "the two stack forms give different images"
        ctx.free_scene(sid)
        sid = None
        after = _render(ctx, sim, sid_room, poses)
        for a, b in zip(shallow[:3], after[:3]):
            assert np.array_equal(a, b)
        record("deep_bvh", depth=int(depth_n), triangles=int(n))
    finally:
        if sid is not None:
            ctx.free_scene(sid)
        ctx.set_bvh_leaf_size(4)
        ctx.free_scene(sid_room)


def _look_quat(f):
    """Attitude whose body x axis (the camera axis) points along f, with no roll."""
    f = np.asarray(f, dtype=np.float64) / np.linalg.norm(f)
    yaw, el = math.atan2(f[1], f[0]), math.asin(f[2])
    qz = np.array([math.cos(yaw / 2), 0.0, 0.0, math.sin(yaw / 2)])
    qy = np.array([math.cos(-el / 2), 0.0, math.sin(-el / 2), 0.0])
    w1, x1, y1, z1 = qz
    w2, x2, y2, z2 = qy
    q = np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                  w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])
    assert np.allclose(oren.quat_to_rot(q)[:, 0], f, atol=1e-12)
    return q


def test_octant_packets_all_eight_and_mixed(vf):
    """Narrow views along the eight octant diagonals put every ray of every packet in one octant (the
    traversal with fixed slab planes); wide views across the horizon mix octants in a packet.  Both kinds
    against the oracle, and the counting variant shows which traversal ran."""
    sim, ctx = vf
    p = default_params()
    sc = scenes.box_room(seed=1)
    sid = ctx.build_scene(sc["verts"], sc["tris"], sc["rgb"])
    dirs = [(sx, sy, sz) for sz in (1, -1) for sy in (1, -1) for sx in (1, -1)]
    q = np.stack([_look_quat(f) for f in dirs])
    states = agents.make_states(np.tile([5.0, 5.0, 2.0], (8, 1)), p, quat=q)
    header("octant packets: 8 narrow views along the octant diagonals, 32x32")
    ctx.read_stats(reset=True)
    ctx.set_stats(True)
    depth, ids, rgb, offs = _render(ctx, sim, sid, states, hw=(32, 32), hfov=0.3)
    ctx.set_stats(False)
    st = ctx.read_stats(reset=True)
    assert st["box_lane"] > 0 and st["box_ops"] == 11 * st["box_lane"]     # every box test at 11 ops
    fr = _check_agents(sc, states, depth, ids, rgb, offs, (32, 32), hfov=0.3, label="octant view")
    assert np.mean(fr) < 0.02
    # wide views level with the horizon: the rows of tiles across it hold rays of both vertical signs
    q2 = np.stack([_look_quat(f) for f in ((1, 0.3, 0), (-0.4, -1, 0), (0.2, 1, 0.05))])
    states2 = agents.make_states(np.tile([5.0, 5.0, 2.0], (3, 1)), p, quat=q2)
    header("octant packets: 3 wide views across the horizon, 64x64 (mixed packets)")
    ctx.set_stats(True)
    depth, ids, rgb, offs = _render(ctx, sim, sid, states2, hw=(64, 64), hfov=2.0)
    ctx.set_stats(False)
    st = ctx.read_stats(reset=True)
    assert 11 * st["box_lane"] < st["box_ops"] < 18 * st["box_lane"]
    fr = _check_agents(sc, states2, depth, ids, rgb, offs, (64, 64), hfov=2.0, label="mixed view")
    assert np.mean(fr) < 0.02
    ctx.free_scene(sid)


# ---------------------------------------------------------------------------
# error handling
# ---------------------------------------------------------------------------

def test_errors_are_reported_not_faults(vf):
    sim, ctx = vf
    from paper_2407_14783_amd import capi
    p = default_params()
    sc = scenes.box_room(seed=1)
    sid = ctx.build_scene(sc["verts"], sc["tris"], sc["rgb"])
    st = _dev(agents.box_room_start(p))
    # unknown scene id -> agent skipped, sticky device error
    views, npx, offs, mh, mw = sim.make_views(1, sid + 17, (16, 16))
    depth = torch.full((npx,), 3.0).cuda()
    ctx.render(st, views, max_hw=(mh, mw), depth=depth, out_pixels=npx)
    with pytest.raises(capi.VfError) as e:
        ctx.sync_check()
    assert e.value.status == capi.VF_EDEVICE and "scene" in str(e.value)
    assert torch.all(depth == 3.0)
    # clip ranges the renderer cannot order hits in (near <= 0, far <= near) -> bad view, nothing written
    for near, far in ((0.0, 100.0), (-1.0, 100.0), (2.0, 2.0)):
        views, npx, offs, mh, mw = sim.make_views(1, sid, (16, 16), near=near, far=far)
        depth = torch.full((npx,), 3.0).cuda()
        ctx.render(st, views, max_hw=(mh, mw), depth=depth, out_pixels=npx)
        with pytest.raises(capi.VfError) as e:
            ctx.sync_check()
        assert e.value.status == capi.VF_EDEVICE and "clip" in str(e.value)
        assert torch.all(depth == 3.0)
    # output capacity too small -> rejected on the device, nothing written
    views, npx, offs, mh, mw = sim.make_views(1, sid, (16, 16))
    ctx.render(st, views, max_hw=(mh, mw), depth=depth, out_pixels=npx - 1)
    with pytest.raises(capi.VfError):
        ctx.sync_check()
    assert torch.all(depth == 3.0)
    # env slot out of range
    ctx.step(p, st, _dev(np.zeros((1, 4))), env_idx=torch.tensor([5], dtype=torch.int32).cuda())
    with pytest.raises(capi.VfError):
        ctx.sync_check()
    # host-side validation
    bad = dict(p)
    bad["n_sub"] = 0
    with pytest.raises(capi.VfError) as e:
        ctx.step(bad, st, _dev(np.zeros((1, 4))))
    assert e.value.status == capi.VF_EINVAL
    with pytest.raises(capi.VfError) as e:
        ctx.build_scene(sc["verts"], np.array([[0, 1, 10_000]], dtype=np.int32))
    assert e.value.status == capi.VF_EINVAL
    # a non-finite vertex used by a triangle is rejected before the build works on it; the error does
    # not stick to later calls
    for bad_value in (float("nan"), float("inf")):
        vbad = sc["verts"].copy()
        vbad[sc["tris"][5, 1], 2] = bad_value
        with pytest.raises(capi.VfError) as e:
            ctx.build_scene(vbad, sc["tris"], sc["rgb"])
        assert e.value.status == capi.VF_EINVAL and "finite" in str(e.value)
    ctx.sync_check()
    with pytest.raises(capi.VfError) as e:
        ctx.free_scene(999)
    assert e.value.status == capi.VF_ENOSCENE
    ctx.sync_check()
    ctx.free_scene(sid)


def test_budget_is_enforced():
    from paper_2407_14783_amd import capi, sim
    small = sim.Context(0, budget_bytes=200_000)
    sc = scenes.forest(seed=3, n_trees=200)
    with pytest.raises(capi.VfError) as e:
        small.build_scene(sc["verts"], sc["tris"], sc["rgb"])
    assert e.value.status == capi.VF_ENOMEM
    used, budget = small.mem_usage()
    assert used <= budget
    small.close()


@pytest.mark.parametrize("mode", ["split", "fused"])
def test_nan_action_is_isolated(vf, mode):
    """A NaN action reaches only its own agent: every other agent's state, depth and ids are bitwise those
    of the same batch without it, over three steps.  (The poisoned agent's rate command turns into zero
    thrust on the rotors it reaches -- the thrust clamp's min / max return the non-NaN operand -- so its
    own state changes but stays finite.)"""
    sim, ctx = vf
    p = default_params()
    sc = scenes.forest(seed=3, n_trees=300)
    sid = ctx.build_scene(sc["verts"], sc["tris"], sc["rgb"])
    n, bad = 48 if mode == "split" else 6, 3
    s0 = agents.forest_starts(4, n, sc, p)
    acts = agents.random_actions(5, 3, n, p)
    poisoned = acts.copy()
    poisoned[0, bad, 1] = np.nan
    views, npx, offs, mh, mw = sim.make_views(n, sid, (64, 64))
    ctx.set_launch_mode(mode == "fused")
    header(f"NaN action isolation: {n} agents, {mode} launch, agent {bad} poisoned")
    res = []
    try:
        for a in (acts, poisoned):
            st = _dev(s0)
            depth = torch.zeros(npx, device="cuda")
            ids = torch.zeros(npx, dtype=torch.int32, device="cuda")
            for k in range(3):
                ctx.step(p, st, _dev(a[k]), views=views, max_hw=(mh, mw), depth=depth, tri_id=ids, out_pixels=npx)
            ctx.sync_check()
            res.append((st.cpu().numpy(), depth.cpu().numpy(), ids.cpu().numpy()))
    finally:
        ctx.set_launch_mode(None)
    (s_a, d_a, i_a), (s_b, d_b, i_b) = res
    others = np.arange(n) != bad
    assert np.array_equal(s_a[others], s_b[others])
    px = np.ones(npx, dtype=bool)
    px[offs[bad]:offs[bad] + 4096] = False
    assert np.array_equal(d_a[px], d_b[px]) and np.array_equal(i_a[px], i_b[px])
    assert not np.array_equal(s_a[bad], s_b[bad])
    ctx.free_scene(sid)
