"""Benchmark of the batched quadrotor step + ray-cast render on one MI355X.

A step is one vf_step call over the whole batch: CTBR controller, rotor lag,
RK4 (Sec. III-A) and the 64x64 depth / triangle id / colour render of every
agent at its new pose (Sec. III-B), on synthetic inputs resident in HBM.  The
library picks the launch form (one fused kernel for small batches, else the
dynamics kernel, an ordering kernel -- longest packets first by the previous
step's traversal work, or agents in spatial order -- and the render kernel).

Default workload ("forest-256"): 256 agents in a seeded procedural forest of
2,000 open 32-segment cylinders on a 40 x 40 m ground quad (128,002 triangles),
64x64 depth + tri id + RGB, dt = 0.02 s, 200 seeded CTBR action steps (cycled).

Printed: one JSON line with frames/s, ms/step, the roofline of the render kernel
(ALU-bound: VALU lane-operations of the ray-box and ray-triangle tests it
performs, counted by a replay with the counting kernel variant, over its
HIP-event time), HBM traffic if supplied from rocprofv3 counters, the serving
latency of the continuous-batching loop, and the FP64 oracle timed on the host.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "64x64 depth frames/s per MI355X + % of HBM roofline; serving p50/p99 latency"
# Work per test, in VALU lane-operations.  The roofline prices each test at the algorithmic figure of a
# ray-box slab test (14) and a Moller-Trumbore ray-triangle test (28).  Beside it, the prices of what the
# kernel issues: box tests from the counting variant (11 VALU ops in a one-octant packet: 6 fused slab
# distances with the exit growth folded in, 4 min/max, 1 compare; 14 with one mixed axis; 18 in general:
# 6 fused slab distances, 10 min/max, 1 multiply for the exit growth, 1 compare) and triangle tests at 40
# (as compiled: 28 mul/FMA for 2 cross, 4 dot, 3 scalings by 1/det and u+v, 3 subs, 1 reciprocal,
# 5 compares -- the last a 64-bit (depth, id) compare --, 2 selects, 1 move).
OPS_PER_BOX, OPS_PER_TRI = 14, 28
ISSUED_OPS_PER_TRI = 40
NODE_BYTES, TRI_BYTES = 128, 48   # one 4-wide node; one leaf triangle record
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12      # 256 CUs x 64 lanes/clk x 2.4 GHz = 39.3 T lane-ops/s
ALU_UNIT = "T lane-ops/s"
HBM_PEAK_GBPS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--agents", type=int, default=256)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-stats", action="store_true", help="skip the counting replay (profiling runs)")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the box-room latency, multi-scene and differentiable measurements")
    ap.add_argument("--traffic-kib", type=str, default=None,
                    help="FETCH,WRITE KiB per dispatch of the render kernel from rocprofv3, already scaled "
                         "(default: the committed profiles/render_forest256_pmc.md figures if the kernel is unchanged)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of known size (for counter scaling)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--multi-scene-only", action="store_true",
                    help="run only the multi-scene batch and print its record (for counter runs)")
    ap.add_argument("--differentiable-only", action="store_true",
                    help="run only the differentiable rollout and print its record (for kernel traces)")
    ap.add_argument("--no-cost-order", action="store_true",
                    help="plain workgroup order (no longest-first order from the previous launch's work)")
    ap.add_argument("--no-spatial-order", action="store_true",
                    help="render agents in the given order instead of (scene, position) order")
    return ap.parse_args()


def copy_calibration():
    import torch
    n = 256 * 1024 * 1024 // 4
    a = torch.ones(n, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": a.numel() * 4, "copy_bytes_written": b.numel() * 4, "launches": 5}))


TRAFFIC_SOURCES = ("render.hip", "vf_internal.h", "dynamics.h", "noise.h", "swarm.h", "bvh_build.hip")


def traffic_source_hash():
    """Hash of the code (comments and whitespace removed) of the sources the counter records depend on."""
    import hashlib
    import re
    csrc = os.path.join(ROOT, "paper_2407_14783_amd", "csrc")
    parts = []
    for f in TRAFFIC_SOURCES:
        text = open(os.path.join(csrc, f), encoding="utf-8").read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        parts.append(" ".join(text.split()))
    return hashlib.sha256("\n".join(parts).encode()).hexdigest()[:16]


def committed_traffic(name="render_forest256_pmc.md"):
    """(fetch_kib, write_kib) per dispatch from a profiles/ counter summary if the render kernel's
    sources and the BVH build (which lays out what it reads) still hash as when the counters were taken,
    else None."""
    import hashlib
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    line = [l for l in open(path) if l.startswith("traffic_kib_per_dispatch:")]
    if not line:
        return None
    kv = dict(tok.split("=") for tok in line[0].split(":", 1)[1].split())
    h = traffic_source_hash()
    if h != kv.get("source_sha256_16"):
        return None
    return float(kv["fetch"]), float(kv["write"])


def cpu_baseline(sc, s0, acts, params, budget_s):
    """The oracle (FP64 dynamics + brute-force render, as it stands) on a bounded sample."""
    from oracle import dynamics as odyn
    from oracle import render as oren
    n_agents = min(4, s0.shape[0])
    s = s0[:n_agents].astype(np.float64)
    frames = 0
    threads = 1
    t0 = time.perf_counter()
    k = 0
    while True:
        s = odyn.step(s, acts[k % acts.shape[0]][:n_agents], params)
        for i in range(n_agents):
            r = oren.render_view(s[i], sc, 64, 64, math.pi / 2, with_mask=False)
            threads = r["threads"]
            frames += 1
        k += 1
        if time.perf_counter() - t0 > budget_s or k >= 50:
            break
    dt = time.perf_counter() - t0
    return {"value": frames / dt, "unit": "frames/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(), "os_cpu_count": os.cpu_count(),
            "sample": f"{n_agents} agents x {k} steps of the forest-256 workload (FP64 RK4 + brute-force "
                      f"all-triangle ray casting, {frames} frames, {dt:.1f} s)"}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline_extra(params):
    """The oracle on the other workloads' samples: the full box-room run (1 agent, 100 steps) and one
    64x64 frame in the smallest and in the largest room graph (20k and 2M triangles)."""
    from oracle import dynamics as odyn
    from oracle import render as oren
    from workloads import agents, scenes
    out = {}
    sc = scenes.box_room(seed=1)
    s = agents.box_room_start(params).astype(np.float64)
    acts = agents.random_actions(2, 100, 1, params)
    t0 = time.perf_counter()
    for k in range(100):
        s = odyn.step(s, acts[k], params)
        oren.render_view(s[0], sc, 64, 64, math.pi / 2, with_mask=False)
    dt = time.perf_counter() - t0
    out["box_room"] = {"frames_per_s": 100 / dt, "sample": "1 agent x 100 steps, 192 triangles",
                       "ray_tri_tests_per_s": 100 * 4096 * 192 / dt}
    scs = scenes.multi_scene_set(seed=6)
    for j in (0, 7):
        st = agents.room_graph_starts(60 + j, 1, scs[j], params).astype(np.float64)
        st = odyn.step(st, agents.random_actions(6, 1, 1, params)[0], params)
        t0 = time.perf_counter()
        oren.render_view(st[0], scs[j], 64, 64, math.pi / 2, with_mask=False)
        dt = time.perf_counter() - t0
        nt = int(scs[j]["tris"].shape[0])
        out[f"room_graph_{nt}"] = {"frames_per_s": 1 / dt, "sample": f"1 agent x 1 step, {nt} triangles",
                                   "ray_tri_tests_per_s_brute_force_equivalent": 4096 * nt / dt}
    return out


def serving_summary(ctx, sim, params):
    from paper_2407_14783_amd import serving
    return serving.bench_summary(ctx, params, n_requests=10000)


def hover_biased_throughput(ctx, sim, sid, sc, params, n=256, steps=100):
    """The forest-256 batch under hover-biased actions (c ~ U(0.9, 1.1) g, body rates ~ U(-1, 1)^3), so the
    agents stay among the trees instead of leaving the forest."""
    import torch
    from workloads import agents
    s0 = agents.forest_starts(4, n, sc, params)
    acts = torch.as_tensor(agents.random_actions(5, steps, n, params, c_range=(0.9, 1.1), rate=1.0)).cuda()
    views, npx, offs, mh, mw = sim.make_views(n, sid, (64, 64))
    state = torch.as_tensor(s0).cuda()
    depth = torch.empty(npx, device="cuda")
    ids = torch.empty(npx, dtype=torch.int32, device="cuda")
    p = sim.capi.params_struct(params)
    for k in range(10):
        ctx.step(p, state, acts[k], views=views, max_hw=(mh, mw), depth=depth, tri_id=ids, out_pixels=npx)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for k in range(steps):
        ctx.step(p, state, acts[k], views=views, max_hw=(mh, mw), depth=depth, tri_id=ids, out_pixels=npx)
    e1.record()
    torch.cuda.synchronize()
    ctx.sync_check()
    ms = e0.elapsed_time(e1) / steps
    return {"workload": "forest-256, hover-biased actions", "ms_per_step": ms, "frames_per_s": n / (ms / 1e3),
            "hit_fraction": float((ids >= 0).float().mean().item())}


def box_room_latency(ctx, sim, params, steps=100):
    """Single agent in the 192-triangle box room: latency-bound step + render (us per step)."""
    import torch
    from workloads import agents, scenes
    sc = scenes.box_room(seed=1)
    sid = ctx.build_scene(sc["verts"], sc["tris"], sc["rgb"])
    s = torch.as_tensor(agents.box_room_start(params)).cuda()
    acts = torch.as_tensor(agents.random_actions(2, steps, 1, params)).cuda()
    views, npx, offs, mh, mw = sim.make_views(1, sid, (64, 64))
    depth = torch.empty(npx, device="cuda")
    p = sim.capi.params_struct(params)
    out = {}
    for mode, fused in (("split", False), ("fused", True)):
        ctx.set_launch_mode(fused)
        for k in range(10):
            ctx.step(p, s, acts[k], views=views, max_hw=(mh, mw), depth=depth, out_pixels=npx)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for k in range(steps):
            ctx.step(p, s, acts[k], views=views, max_hw=(mh, mw), depth=depth, out_pixels=npx)
        e1.record()
        torch.cuda.synchronize()
        out[f"{mode}_us_per_step"] = e0.elapsed_time(e1) / steps * 1e3
    ctx.set_launch_mode(None)
    ctx.sync_check()
    ctx.free_scene(sid)
    return {"workload": "box-room: 1 agent, 192 triangles, 64x64 depth, 100 steps", **out,
            "frames_per_s": 1e6 / min(out["split_us_per_step"], out["fused_us_per_step"])}


def multi_scene_throughput(ctx, sim, params, steps=20, count=True):
    """4,096 agents over the 8 room-graph scenes (Dirichlet split), half 64x64 and half 128x128 depth."""
    import torch
    from workloads import agents, scenes
    from paper_2407_14783_amd.serving import ROOM_LEAF_SIZE
    scs = scenes.multi_scene_set(seed=6)
    ctx.set_bvh_leaf_size(ROOM_LEAF_SIZE)      # room graphs: leaves of at most 3 triangles
    t0 = time.perf_counter()
    sids = [ctx.build_scene(s["verts"], s["tris"], s["rgb"]) for s in scs]
    build_s = time.perf_counter() - t0
    ctx.set_bvh_leaf_size(4)
    counts = agents.multi_scene_split(6, 4096, 8)
    st = np.concatenate([agents.room_graph_starts(60 + j, int(c), scs[j], params) for j, c in enumerate(counts)])
    scene_of = np.repeat(np.arange(8), counts)
    rng = np.random.default_rng(6)
    big = rng.permutation(4096) < 2048
    hw = np.where(big, 128, 64)
    views, npx, offs, mh, mw = sim.make_views(4096, np.asarray(sids)[scene_of], np.stack([hw, hw], 1))
    state = torch.as_tensor(st).cuda()
    acts = torch.as_tensor(agents.random_actions(6, steps, 4096, params)).cuda()
    depth = torch.empty(npx, device="cuda")
    p = sim.capi.params_struct(params)
    for k in range(3):
        ctx.step(p, state, acts[k], views=views, max_hw=(mh, mw), depth=depth, out_pixels=npx)
    state_at_start = state.clone()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for k in range(steps):
        ctx.step(p, state, acts[k], views=views, max_hw=(mh, mw), depth=depth, out_pixels=npx)
    e1.record()
    torch.cuda.synchronize()
    ctx.sync_check()
    ms = e0.elapsed_time(e1) / steps
    # the render kernel's launch time: HIP events around every render launch in a replay of the same steps
    state.copy_(state_at_start)
    torch.cuda.synchronize()
    ctx.set_timing(True)
    for k in range(steps):
        ctx.step(p, state, acts[k], views=views, max_hw=(mh, mw), depth=depth, out_pixels=npx)
    torch.cuda.synchronize()
    ctx.sync_check()
    render_ms, render_launches = ctx.timing_read(reset=True)
    ctx.set_timing(False)
    render_s = render_ms / 1e3 / max(render_launches, 1)
    roof = rates = None
    if count:
        # the same steps from the same states with the counting kernel variant (not timed)
        state.copy_(state_at_start)
        ctx.read_stats(reset=True)
        ctx.set_stats(True)
        for k in range(steps):
            ctx.step(p, state, acts[k], views=views, max_hw=(mh, mw), depth=depth, out_pixels=npx)
        ctx.set_stats(False)
        roof, rates = alu_roofline(ctx.read_stats(reset=True), steps, render_s)
    infos = [ctx.scene_info(s) for s in sids]
    for s in sids:
        ctx.free_scene(s)
    out = {"workload": "multi-scene: 4,096 agents over 8 room graphs (20k-2M triangles), half 64x64 half 128x128",
           "ms_per_step": ms, "frames_per_s": 4096 / (ms / 1e3), "rays_per_s": npx / (ms / 1e3),
           "frames_64x64_equivalent_per_s": npx / 4096 / (ms / 1e3),
           "render_kernel_avg_us": render_s * 1e6,
           "scene_triangles": [int(i["n_tris"]) for i in infos],
           "scene_bytes": [int(i["bytes"]) for i in infos],
           "scene_build_device_ms": [round(float(i["build_ms"]), 2) for i in infos],
           "bvh_leaf_size": int(infos[0]["leaf_max"]),
           "scene_build_wall_s_incl_upload": build_s}
    if roof:
        out["alu_roofline"] = roof
        out["test_rates"] = rates
    tk = committed_traffic("render_multiscene4096_pmc.md")
    if tk:
        traffic = (tk[0] + tk[1]) * 1024.0
        out["hbm"] = {"bytes_per_launch": traffic, "achieved_GBps": traffic / render_s / 1e9,
                      "peak_GBps": HBM_PEAK_GBPS, "frac": traffic / render_s / 1e9 / HBM_PEAK_GBPS,
                      "source": "profiles/render_multiscene4096_pmc.md"}
    return out


def alu_roofline(st, launches, render_s):
    """ALU roofline of the render kernel from the counting replay's counters over `launches` launches and
    the average launch time render_s (HIP events around the render launches of the timed steps, or of their
    replay from the same start state).  achieved = the algorithmic work of
    the launch over render_s: the ray-box and ray-triangle tests each ray's own traversal needs (the visits
    of nodes and leaves whose box that ray entered), priced at OPS_PER_BOX / OPS_PER_TRI.  Beside it the
    tests the packets issue (every valid lane at every node and leaf its packet visits), at the same prices
    and at the kernel's issued prices: their excess over the need is the packets' waste."""
    rays = st["rays"] / launches
    box, tri = st["box_lane"] / launches, st["tri_lane"] / launches
    nbox, ntri = st["need_box"] / launches, st["need_tri"] / launches
    ops = box * OPS_PER_BOX + tri * OPS_PER_TRI
    issued_ops = st["box_ops"] / launches + tri * ISSUED_OPS_PER_TRI
    need_ops = nbox * OPS_PER_BOX + ntri * OPS_PER_TRI
    achieved = need_ops / render_s / 1e12
    logical = st["node_wave"] / launches * NODE_BYTES + st["tri_wave"] / launches * TRI_BYTES
    roof = {"bound": "alu", "achieved": achieved, "peak": ALU_PEAK_TOPS, "unit": ALU_UNIT,
            "frac": achieved / ALU_PEAK_TOPS, "traffic": None,
            "work": "the tests each ray's own traversal needs, at the prices below",
            "prices": {"box_test": OPS_PER_BOX, "tri_test": OPS_PER_TRI},
            "frac_issued_tests": ops / render_s / 1e12 / ALU_PEAK_TOPS,
            "frac_issued_tests_at_issued_prices": issued_ops / render_s / 1e12 / ALU_PEAK_TOPS,
            "render_kernel_us": render_s * 1e6,
            "per_launch": {"rays": rays, "ray_box_tests": box, "ray_tri_tests": tri,
                           "wave_node_visits": st["node_wave"] / launches,
                           "box_tests_per_ray": box / max(rays, 1), "tri_tests_per_ray": tri / max(rays, 1),
                           "needed_box_tests_per_ray": nbox / max(rays, 1),
                           "needed_tri_tests_per_ray": ntri / max(rays, 1),
                           "packet_efficiency_box": nbox / max(box, 1), "packet_efficiency_tri": ntri / max(tri, 1),
                           "issued_valu_ops_per_box_test": st["box_ops"] / max(st["box_lane"], 1),
                           "valu_ops_needed": need_ops, "valu_ops_issued_tests": ops,
                           "valu_ops_at_issued_prices": issued_ops, "logical_scene_bytes": logical}}
    rates = {"ray_box_tests_per_s": box / render_s, "ray_tri_tests_per_s": tri / render_s,
             "needed_ray_box_tests_per_s": nbox / render_s, "needed_ray_tri_tests_per_s": ntri / render_s,
             "valu_ceiling_box_tests_per_s": ALU_PEAK_TOPS * 1e12 / OPS_PER_BOX,
             "valu_ceiling_tri_tests_per_s": ALU_PEAK_TOPS * 1e12 / OPS_PER_TRI,
             "logical_scene_GBps": logical / render_s / 1e9,
             "basis": "per second of render-kernel time; ceilings = VALU peak / algorithmic ops per test"}
    return roof, rates


def copy_ceiling_gbps(reps=5):
    """Measured HBM ceiling: a plain 1 GiB device-to-device copy (read + write bytes per second)."""
    import torch
    a = torch.empty(256 * 2 ** 20, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    gbps = 2 * a.numel() * 4 * reps / (e0.elapsed_time(e1) / 1e3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return gbps


def bptt_throughput(ctx, sim, params, n=1024, horizon=64, k=8):
    """Differentiable rollout: 1,024 agents in the forest, horizon 64, checkpoints every 8, depth loss."""
    import torch
    from paper_2407_14783_amd import autograd as vag
    from workloads import agents, scenes
    sc = scenes.forest(seed=3)
    sid = ctx.build_scene(sc["verts"], sc["tris"], sc["rgb"])
    s0 = torch.as_tensor(agents.forest_starts(8, n, sc, params)).cuda().requires_grad_(True)
    rng = np.random.default_rng(8)
    a = np.concatenate([rng.uniform(0.9, 1.15, (horizon, n, 1)) * params["g"],
                        rng.uniform(-0.6, 0.6, (horizon, n, 3))], axis=2).astype(np.float32)
    acts = torch.as_tensor(a).cuda().requires_grad_(True)
    goals = s0.detach()[:, 0:3] + 10.0
    views, npx, offs, mh, mw = sim.make_views(n, sid, (64, 64))

    def once():
        states, depths = vag.rollout(ctx, params, s0, acts, views, (mh, mw), npx, checkpoint_every=k)
        loss = torch.exp(-depths).view(horizon, n, -1).mean(2).sum() + 0.01 * ((states[:, :, 0:3] - goals) ** 2).sum()
        loss.backward()
        return loss
    once()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = 2
    for _ in range(reps):
        s0.grad = None
        acts.grad = None
        once()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    ctx.free_scene(sid)
    return {"workload": "differentiable: 1,024 agents, forest, horizon 64, checkpoints every 8, 64x64 depth loss",
            "s_per_rollout_fwd_bwd": dt, "agent_steps_per_s": n * horizon / dt}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: there is no multi-GPU path here "
              "(agents would shard by scene with no exchange)", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    import torch
    from paper_2407_14783_amd import sim
    if args.multi_scene_only:
        from workloads import default_params
        ctx = sim.Context(0)
        print(json.dumps({"multi_scene": multi_scene_throughput(ctx, sim, default_params(), count=not args.no_stats)}))
        ctx.close()
        return
    if args.differentiable_only:
        from workloads import default_params
        ctx = sim.Context(0)
        print(json.dumps({"differentiable": bptt_throughput(ctx, sim, default_params())}))
        ctx.close()
        return
    from workloads import agents, default_params, scenes

    params = default_params()
    n = args.agents
    sc = scenes.forest(seed=3)
    s0 = agents.forest_starts(4, n, sc, params)
    acts_np = agents.random_actions(5, 200, n, params)
    ctx = sim.Context(0)
    ctx.set_spatial_order(not args.no_spatial_order)
    ctx.set_cost_order(not args.no_cost_order)
    # the latency-bound single-agent case first, on an idle device
    box_room = None if args.no_extra else box_room_latency(ctx, sim, params)
    sid = ctx.build_scene(sc["verts"], sc["tris"], sc["rgb"])
    info = ctx.scene_info(sid)
    views, npx, offs, mh, mw = sim.make_views(n, sid, (64, 64))
    state = torch.as_tensor(s0).cuda()
    acts = torch.as_tensor(acts_np).cuda()
    depth = torch.empty(npx, device="cuda")
    tri_id = torch.empty(npx, dtype=torch.int32, device="cuda")
    rgb = torch.empty(3 * npx, dtype=torch.uint8, device="cuda")
    pstruct = sim.capi.params_struct(params)
    stream = torch.cuda.current_stream()

    def run(k0, k1):
        for k in range(k0, k1):
            ctx.step(pstruct, state, acts[k % 200], views=views, max_hw=(mh, mw), depth=depth, tri_id=tri_id,
                     rgb=rgb, out_pixels=npx, stream=stream)

    run(0, args.warmup)
    torch.cuda.synchronize()
    ctx.sync_check()
    state_at_start = state.clone()      # the timed region starts here; the repeats restart from it
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    run(args.warmup, args.warmup + args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.sync_check()
    repeats = [gpu_ms_first := e0.elapsed_time(e1)]
    hit_frac = float((tri_id >= 0).float().mean().item())
    # the same K steps again from the same start state with HIP events around every render-kernel launch
    # (vf_set_timing), for the render kernel's average launch duration.  The events add a few microseconds
    # to every step, so the timed run above carries none.
    state.copy_(state_at_start)
    torch.cuda.synchronize()
    ctx.set_timing(True)
    e0.record(stream)
    run(args.warmup, args.warmup + args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ctx.sync_check()
    render_ms, render_launches = ctx.timing_read(reset=True)
    ctx.set_timing(False)
    events_ms = e0.elapsed_time(e1)
    # four more runs of the same K steps from the same states, for the run-to-run spread
    for _ in range(4):
        state.copy_(state_at_start)
        torch.cuda.synchronize()
        e0.record(stream)
        run(args.warmup, args.warmup + args.steps)
        e1.record(stream)
        torch.cuda.synchronize()
        repeats.append(e0.elapsed_time(e1))
    render_s = render_ms / 1e3 / max(render_launches, 1)     # average render-kernel duration
    gpu_ms = gpu_ms_first
    ms_per_step = gpu_ms / args.steps
    frames_per_s = n * args.steps / (gpu_ms / 1e3)

    out = {"metric": METRIC, "value": frames_per_s, "unit": "frames/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "forest-256", "agents": n, "scene_triangles": int(info["n_tris"]),
                      "image": "64x64", "outputs": "depth f32 + tri id i32 + RGB u8", "controller": "CTBR",
                      "integrator": "RK4", "dt": params["dt"], "bvh_nodes": int(info["n_nodes"]),
                      "bvh_depth": int(info["depth"]), "scene_build_ms": round(float(info["build_ms"]), 3)},
           "wall_s": wall, "hit_fraction": hit_frac,
           "ms_per_step_5_runs": {"runs": [r / args.steps for r in repeats],
                                  "median": float(np.median(repeats)) / args.steps},
           "render_kernel": {"avg_us": render_s * 1e6, "launches": render_launches,
                             "timing": "HIP events around each render launch on its stream, in a replay of "
                                       "the timed steps from the same start state",
                             "ms_per_step_with_events": events_ms / args.steps}}

    if not args.no_stats:
        # replay the same steps with the counting kernel variant (not timed)
        state.copy_(torch.as_tensor(s0).cuda())
        run(0, args.warmup)
        torch.cuda.synchronize()
        ctx.read_stats(reset=True)
        ctx.set_stats(True)
        run(args.warmup, args.warmup + args.steps)
        ctx.set_stats(False)
        st = ctx.read_stats(reset=True)
        out["roofline"], out["test_rates"] = alu_roofline(st, args.steps, render_s)
        out["ray_tri_tests_per_s"] = out["roofline"]["per_launch"]["ray_tri_tests"] / (ms_per_step / 1e3)
        out["rays_per_s"] = out["roofline"]["per_launch"]["rays"] / (ms_per_step / 1e3)
    tk = tuple(float(x) for x in args.traffic_kib.split(",")) if args.traffic_kib else committed_traffic()
    if tk:
        fetch_kib, write_kib = tk
        traffic = (fetch_kib + write_kib) * 1024.0
        if "roofline" in out:
            out["roofline"]["traffic"] = traffic
        out["hbm"] = {"bytes_per_launch": traffic, "achieved_GBps": traffic / render_s / 1e9,
                      "peak_GBps": HBM_PEAK_GBPS, "frac": traffic / render_s / 1e9 / HBM_PEAK_GBPS}
        if not args.no_extra:
            cc = copy_ceiling_gbps()
            out["hbm"]["copy_ceiling_GBps"] = cc
            out["hbm"]["frac_of_copy"] = traffic / render_s / 1e9 / cc
    if not args.no_serving:
        out["serving"] = serving_summary(ctx, sim, params)
    if not args.no_extra:
        out["box_room_latency"] = box_room
        out["forest256_hover_biased"] = hover_biased_throughput(ctx, sim, sid, sc, params)
        out["multi_scene"] = multi_scene_throughput(ctx, sim, params)
        out["differentiable"] = bptt_throughput(ctx, sim, params)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(sc, s0, acts_np, params, args.cpu_seconds)
        out["cpu_baseline_other_workloads"] = cpu_baseline_extra(params)
    ctx.free_scene(sid)
    ctx.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
