"""Table II noise on the device against the FP64 oracle: Poisson noise of the three image sensors, all four
models on segmentation labels, and the render kernel's epilogue form against the separate pass.

Both sides draw the same Philox4x32-10 words.  A discrete outcome (a Poisson count, a rounded label or
level, a salt-and-pepper choice) must match exactly wherever the oracle's decision margin -- how far a
compared quantity was from its threshold -- is clear of what the two sides' rounding can move: 1e-9 for
the FP64 Poisson draws (transcendentals one unit in the last place apart), 1e-3 for labels whose value
comes through the device's float32 Box-Muller normal.  The pixels set aside are counted and must stay
under 1%.  Poisson depth is compared as the float32 the device writes (the FP64 value rounded once).
"""
import math

import numpy as np
import pytest
import torch

from oracle import noise as onoise
from workloads import agents, default_params, scenes
from tests.gpu_util import header, record

pytestmark = pytest.mark.gpu

POISSON_MARGIN = 1e-9
LABEL_MARGIN = 1e-3


@pytest.fixture(scope="module")
def vf():
    from paper_2407_14783_amd import capi, sim
    ctx = sim.Context(0)
    yield sim, capi, ctx
    ctx.close()


def _rendered(sim, ctx, n=5, hw=(33, 47), keys=None, seed=11):
    sc = scenes.box_room(seed=1)
    sid = ctx.build_scene(sc["verts"], sc["tris"], sc["rgb"])
    rng = np.random.default_rng(seed)
    pos = rng.uniform([2, 2, 1], [8, 8, 3], (n, 3))
    st = torch.as_tensor(agents.make_states(pos, default_params(),
                                            quat=agents.yaw_quat(rng.uniform(-np.pi, np.pi, n)))).cuda()
    views, npx, offs, mh, mw = sim.make_views(n, sid, hw, noise_keys=keys)
    depth = torch.empty(npx).cuda()
    ids = torch.empty(npx, dtype=torch.int32).cuda()
    rgb = torch.empty(3 * npx, dtype=torch.uint8).cuda()
    ctx.render(st, views, max_hw=(mh, mw), depth=depth, tri_id=ids, rgb=rgb, out_pixels=npx)
    ctx.sync_check()
    return sc, sid, st, views, npx, offs, (mh, mw), depth, ids, rgb


@pytest.mark.parametrize("scale", [1.5, 40.0])
def test_depth_poisson_matches_oracle(vf, scale):
    """P(D c) / c with rates D c of about 2-15 (inversion and rejection both) and 40-600 (rejection)."""
    sim, capi, ctx = vf
    keys = [4, 1, 99, 123456, 7]
    sc, sid, st, views, npx, offs, hw, depth, ids, rgb = _rendered(sim, ctx, keys=keys)
    clean = depth.cpu().numpy().astype(np.float64)
    hit = ids.cpu().numpy() >= 0
    seed = 0xDEADBEEF1234
    header(f"noise: depth Poisson, {scale} counts per metre")
    ctx.sensor_noise(views, 5, hw, npx, depth=depth, tri_id=ids, depth_model=capi.VF_NOISE_POISSON,
                     depth_scale=scale, seed=seed)
    ctx.sync_check()
    got = depth.cpu().numpy()
    P = hw[0] * hw[1]
    compared = set_aside = 0
    for a in range(5):
        s = slice(offs[a], offs[a] + P)
        ref, margin = onoise.noisy_depth(clean[s], hit[s], onoise.NOISE_POISSON, 0.0, 0.0, seed, keys[a], 0.01, 100.0,
                                         scale=scale, with_margin=True)
        ok = margin > POISSON_MARGIN
        assert np.array_equal(got[s][ok], ref[ok].astype(np.float32)), f"agent {a}"
        compared += int((ok & hit[s]).sum())
        set_aside += int((~ok).sum())
        assert np.array_equal(got[s][~hit[s]], clean[s][~hit[s]].astype(np.float32))
    record(f"noise[depth poisson c={scale}]", compared=compared, set_aside=set_aside)
    assert compared > 0.9 * hit.sum() and set_aside <= 0.01 * hit.sum()
    ctx.free_scene(sid)


@pytest.mark.parametrize("scale", [0.05, 1.0])
def test_rgb_poisson_matches_oracle(vf, scale):
    """Per-channel P(v c) / c rounded half up: rates 0-13 (inversion) and 0-255 (both methods)."""
    sim, capi, ctx = vf
    sc, sid, st, views, npx, offs, hw, depth, ids, rgb = _rendered(sim, ctx)
    clean = rgb.cpu().numpy().copy()
    header(f"noise: colour Poisson, {scale} counts per level")
    ctx.sensor_noise(views, 5, hw, npx, rgb=rgb, rgb_model=capi.VF_NOISE_POISSON, rgb_scale=scale, seed=77)
    ctx.sync_check()
    got = rgb.cpu().numpy()
    P = hw[0] * hw[1]
    compared = set_aside = 0
    for a in range(5):
        planes = np.stack([clean[3 * offs[a] + c * P: 3 * offs[a] + (c + 1) * P] for c in range(3)])
        gp = np.stack([got[3 * offs[a] + c * P: 3 * offs[a] + (c + 1) * P] for c in range(3)])
        ref, margin = onoise.noisy_rgb(planes, onoise.NOISE_POISSON, 0.0, 0.0, 77, a, scale=scale, with_margin=True)
        ok = margin > POISSON_MARGIN
        assert np.array_equal(gp[:, ok], ref[:, ok]), f"agent {a}"
        compared += int(ok.sum())
        set_aside += int((~ok).sum())
    record(f"noise[rgb poisson c={scale}]", compared=compared, set_aside=set_aside)
    assert set_aside <= 0.01 * (compared + set_aside)
    ctx.free_scene(sid)


@pytest.mark.parametrize("model,sigma,p,scale", [(1, 2.5, 0.0, 1.0), (2, 0.1, 0.0, 1.0), (3, 0.0, 0.2, 1.0),
                                                 (4, 0.0, 0.0, 1.0), (4, 0.0, 0.0, 0.05)])
def test_label_noise_matches_oracle(vf, model, sigma, p, scale):
    """Segmentation labels (0..180 by triangle) under Normal, speckle, salt & pepper and Poisson noise."""
    sim, capi, ctx = vf
    keys = [11, 12, 13, 14, 15]
    sc, sid, st, views, npx, offs, hw, depth, ids, rgb = _rendered(sim, ctx, keys=keys)
    labels = (np.arange(sc["tris"].shape[0]) * 37 % 181).astype(np.int32)
    ctx.set_labels(sid, labels)
    seg = ctx.segmentation(views, 5, hw, ids, npx)
    ctx.sync_check()
    clean = seg.cpu().numpy().copy()
    header(f"noise: labels, model {model}, sigma {sigma}, p {p}, scale {scale}")
    ctx.sensor_noise(views, 5, hw, npx, seg=seg, seg_model=model, seg_sigma=sigma, seg_p=p, seg_scale=scale,
                     seg_salt_label=500, seed=2024)
    ctx.sync_check()
    got = seg.cpu().numpy()
    P = hw[0] * hw[1]
    compared = set_aside = 0
    thr = POISSON_MARGIN if model == 4 else LABEL_MARGIN
    for a in range(5):
        s = slice(offs[a], offs[a] + P)
        ref, margin = onoise.noisy_segmentation(clean[s], model, sigma, p, 2024, keys[a], scale=scale, salt_label=500,
                                                with_margin=True)
        ok = margin > thr
        assert np.array_equal(got[s][ok], ref[ok]), f"agent {a}: {np.nonzero(got[s][ok] != ref[ok])[0][:5]}"
        compared += int(ok.sum())
        set_aside += int((~ok).sum())
        assert np.array_equal(got[s][clean[s] < 0], clean[s][clean[s] < 0])   # unlabelled pixels stay
    record(f"noise[labels model={model} c={scale}]", compared=compared, set_aside=set_aside)
    assert set_aside <= 0.01 * (compared + set_aside)
    if model in (1, 2, 4):
        assert np.any(got != clean)
    ctx.free_scene(sid)


CFGS = {
    "normal": dict(depth_model=1, depth_sigma=0.05, rgb_model=1, rgb_sigma=6.0),
    "speckle": dict(depth_model=2, depth_sigma=0.02, rgb_model=2, rgb_sigma=0.1),
    "salt_pepper": dict(depth_model=3, depth_p=0.1, rgb_model=3, rgb_p=0.2),
    "poisson": dict(depth_model=4, depth_scale=20.0, rgb_model=4, rgb_scale=0.5),
}


@pytest.mark.parametrize("name", list(CFGS))
def test_render_epilogue_equals_separate_pass(vf, name):
    """vf_render / vf_step with the render-noise epilogue give the bits of a plain render followed by
    vf_sensor_noise (with the ids) of the same configuration: split and fused launches, ragged tiles."""
    sim, capi, ctx = vf
    cfg = dict(CFGS[name], seed=0xABCDEF)
    keys = [5, 6, 7, 8, 9]
    sc, sid, st, views, npx, offs, hw, depth, ids, rgb = _rendered(sim, ctx, keys=keys)
    header(f"noise: render epilogue vs separate pass, {name}")
    ctx.sensor_noise(views, 5, hw, npx, depth=depth, rgb=rgb, tri_id=ids, **cfg)
    ctx.sync_check()
    d2 = torch.empty_like(depth)
    i2 = torch.empty_like(ids)
    c2 = torch.empty_like(rgb)
    ctx.set_render_noise(**cfg)
    try:
        ctx.render(st, views, max_hw=hw, depth=d2, tri_id=i2, rgb=c2, out_pixels=npx)
        ctx.sync_check()
    finally:
        ctx.set_render_noise()
    assert torch.equal(i2, ids)
    assert torch.equal(d2, depth)
    assert torch.equal(c2, rgb)
    # a step: fused (small batch) and split launches against step + render + separate pass
    p = default_params()
    act = torch.as_tensor(agents.random_actions(3, 1, 5, p)[0]).cuda()
    outs = []
    for mode in (True, False):
        ctx.set_launch_mode(mode)
        for noise_on in (False, True):
            s1 = st.clone()
            dd, ii, cc = torch.empty_like(depth), torch.empty_like(ids), torch.empty_like(rgb)
            if noise_on:
                ctx.set_render_noise(**cfg)
            try:
                ctx.step(p, s1, act, views=views, max_hw=hw, depth=dd, tri_id=ii, rgb=cc, out_pixels=npx)
                ctx.sync_check()
            finally:
                ctx.set_render_noise()
            if not noise_on:
                ctx.sensor_noise(views, 5, hw, npx, depth=dd, rgb=cc, tri_id=ii, **cfg)
                ctx.sync_check()
            outs.append((s1, dd, ii, cc))
    ctx.set_launch_mode(None)
    for j in (1, 2, 3):
        for x, y in zip(outs[0], outs[j]):
            assert torch.equal(x, y), f"{name}: launch {j}"
    ctx.free_scene(sid)


def test_noise_parameter_errors(vf):
    sim, capi, ctx = vf
    sc, sid, st, views, npx, offs, hw, depth, ids, rgb = _rendered(sim, ctx, n=2)
    for bad in (dict(depth_model=4, depth_scale=0.0), dict(rgb_model=4, rgb_scale=-1.0),
                dict(seg_model=4, seg_scale=float("nan")), dict(seg_model=5), dict(seg_model=1, seg_sigma=-0.5),
                dict(seg_model=3, seg_p=2.0)):
        with pytest.raises(capi.VfError):
            ctx.sensor_noise(views, 2, hw, npx, depth=depth, **bad)
        with pytest.raises(capi.VfError):
            ctx.set_render_noise(**bad)
    ctx.free_scene(sid)
