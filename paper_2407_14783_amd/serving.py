"""Serving form: thin binding of the library's continuous-batching server, plus the
Poisson load generator used to measure p50/p99 latency next to frames/s.

The scheduler itself (admission by HBM budget, env-slot ordering, multi-stream
overlap) is native code in the library (csrc/serve.cpp); this module only
marshals requests and results.
"""
import ctypes
import math
import threading
import time

import numpy as np
import torch

from . import capi
from .capi import check, lib


class ServerConfig(ctypes.Structure):
    _fields_ = [("params", capi.DynParams), ("n_streams", ctypes.c_int32), ("max_batch_agents", ctypes.c_int32),
                ("max_h", ctypes.c_int32), ("max_w", ctypes.c_int32), ("want_tri_id", ctypes.c_int32),
                ("want_rgb", ctypes.c_int32), ("hbm_budget_bytes", ctypes.c_int64)]


class RequestDesc(ctypes.Structure):
    _fields_ = [("scene_id", ctypes.c_int32), ("H", ctypes.c_int32), ("W", ctypes.c_int32), ("n_env", ctypes.c_int32),
                ("hfov", ctypes.c_float), ("near_clip", ctypes.c_float), ("far_clip", ctypes.c_float),
                ("miss_depth", ctypes.c_float)]


class RequestOut(ctypes.Structure):
    _fields_ = [("depth", ctypes.c_void_p), ("tri_id", ctypes.c_void_p), ("rgb", ctypes.c_void_p),
                ("state", ctypes.c_void_p), ("host_results", ctypes.c_int32), ("pad", ctypes.c_int32)]


class ServerStats(ctypes.Structure):
    _fields_ = [("batches", ctypes.c_int64), ("agents", ctypes.c_int64), ("requests", ctypes.c_int64),
                ("max_batch_agents", ctypes.c_int64), ("pending", ctypes.c_int64),
                ("in_flight_batches", ctypes.c_int64), ("requeued", ctypes.c_int64),
                ("failed_batches", ctypes.c_int64)]


_P, _I64 = ctypes.c_void_p, ctypes.c_int64
lib.vf_server_create.argtypes = [_P, ctypes.POINTER(ServerConfig), _P, _I64, ctypes.POINTER(_P)]
lib.vf_server_submit.argtypes = [_P, ctypes.POINTER(RequestDesc), _P, _P, ctypes.POINTER(RequestOut),
                                 ctypes.POINTER(_I64)]
lib.vf_server_poll.argtypes = [_P, _I64, ctypes.POINTER(ctypes.c_int32)]
lib.vf_server_wait.argtypes = [_P, _I64, _P, _P, _P, _P, ctypes.POINTER(ctypes.c_double)]
lib.vf_server_stats_get.argtypes = [_P, ctypes.POINTER(ServerStats)]
lib.vf_server_destroy.argtypes = [_P]
lib.vf_server_inject_faults.argtypes = [_P, _I64]
for _f in ("vf_server_create", "vf_server_submit", "vf_server_poll", "vf_server_wait", "vf_server_stats_get",
           "vf_server_destroy", "vf_server_inject_faults"):
    getattr(lib, _f).restype = ctypes.c_int32


class Server:
    """Continuous-batching step + render server over a resident state table [S, 17] (device)."""

    def __init__(self, sim_ctx, params, state_table, n_streams=3, max_batch_agents=8192, max_hw=(128, 128),
                 want_tri_id=False, want_rgb=False, budget_bytes=2 << 30):
        if not (state_table.is_cuda and state_table.is_contiguous() and state_table.shape[1] == 17):
            raise ValueError("state_table must be a contiguous device tensor [S, 17]")
        cfg = ServerConfig()
        cfg.params = params if isinstance(params, capi.DynParams) else capi.params_struct(params)
        cfg.n_streams = n_streams
        cfg.max_batch_agents = max_batch_agents
        cfg.max_h, cfg.max_w = max_hw
        cfg.want_tri_id = int(want_tri_id)
        cfg.want_rgb = int(want_rgb)
        cfg.hbm_budget_bytes = int(budget_bytes)
        self.want_tri_id, self.want_rgb = want_tri_id, want_rgb
        self.state_table = state_table
        self._meta = {}
        self._keep = {}
        h = ctypes.c_void_p()
        check(lib.vf_server_create(sim_ctx.h, ctypes.byref(cfg), ctypes.c_void_p(state_table.data_ptr()),
                                   state_table.shape[0], ctypes.byref(h)), "vf_server_create")
        self.h = h

    def prepare(self, scene_id, hw, env_slots, actions, hfov=math.pi / 2, near=0.01, far=100.0, miss_depth=None,
                out=None, host_results=True):
        """Marshal one request (validation, ctypes descriptors, contiguous host arrays) without submitting it.
        out: optional dict of device tensors {'depth', 'tri_id', 'rgb', 'state'} receiving the results."""
        slots = np.ascontiguousarray(env_slots, dtype=np.int32)
        acts = np.ascontiguousarray(actions, dtype=np.float32).reshape(slots.shape[0], 4)
        d = RequestDesc(scene_id, hw[0], hw[1], slots.shape[0], hfov, near, far, far if miss_depth is None else miss_depth)
        o = RequestOut()
        n_px = slots.shape[0] * hw[0] * hw[1]
        sizes = {"depth": n_px, "tri_id": n_px, "rgb": 3 * n_px, "state": 17 * slots.shape[0]}
        for k, tns in (out or {}).items():
            if tns is None:
                continue
            if not (tns.is_cuda and tns.is_contiguous() and tns.numel() >= sizes[k]):
                raise ValueError(f"out[{k!r}] must be a contiguous device tensor of >= {sizes[k]} elements")
            setattr(o, k, tns.data_ptr())
        o.host_results = 1 if host_results else 0
        return (d, slots, acts, o, slots.ctypes.data_as(ctypes.c_void_p), acts.ctypes.data_as(ctypes.c_void_p),
                (slots.shape[0], hw[0], hw[1]), out)

    def submit_prepared(self, prep):
        """Submit a request marshalled by prepare(); returns its ticket."""
        d, slots, acts, o, p_slots, p_acts, meta, out = prep
        t = ctypes.c_int64()
        check(lib.vf_server_submit(self.h, ctypes.byref(d), p_slots, p_acts, ctypes.byref(o), ctypes.byref(t)),
              "vf_server_submit")
        self._keep[t.value] = out
        self._meta[t.value] = meta
        return t.value

    def submit(self, scene_id, hw, env_slots, actions, hfov=math.pi / 2, near=0.01, far=100.0, miss_depth=None,
               out=None, host_results=True):
        """out: optional dict of device tensors {'depth', 'tri_id', 'rgb', 'state'} receiving the results."""
        return self.submit_prepared(self.prepare(scene_id, hw, env_slots, actions, hfov, near, far, miss_depth,
                                                 out, host_results))

    def poll(self, ticket):
        done = ctypes.c_int32()
        check(lib.vf_server_poll(self.h, ticket, ctypes.byref(done)), "vf_server_poll")
        return bool(done.value)

    def wait(self, ticket, fetch=True):
        n, hh, ww = self._meta.pop(ticket)
        self._keep.pop(ticket, None)
        px = n * hh * ww
        depth = np.empty(px, dtype=np.float32) if fetch else None
        ids = np.empty(px, dtype=np.int32) if fetch and self.want_tri_id else None
        rgb = np.empty(3 * px, dtype=np.uint8) if fetch and self.want_rgb else None
        st = np.empty((n, 17), dtype=np.float32) if fetch else None
        lat = ctypes.c_double()

        def p(a):
            return None if a is None else a.ctypes.data_as(ctypes.c_void_p)
        check(lib.vf_server_wait(self.h, ticket, p(depth), p(ids), p(rgb), p(st), ctypes.byref(lat)), "vf_server_wait")
        return {"depth": depth, "tri_id": ids, "rgb": rgb, "state": st, "latency_s": lat.value}

    def inject_faults(self, n):
        """Treat the next n batches that finish as failed (restored and run again)."""
        check(lib.vf_server_inject_faults(self.h, int(n)), "vf_server_inject_faults")

    def stats(self):
        s = ServerStats()
        check(lib.vf_server_stats_get(self.h, ctypes.byref(s)), "vf_server_stats_get")
        return {k: getattr(s, k) for k, _ in ServerStats._fields_}

    def close(self):
        if self.h:
            check(lib.vf_server_destroy(self.h), "vf_server_destroy")
            self.h = None


# ---------------------------------------------------------------------------
# load generation
# ---------------------------------------------------------------------------

def make_requests(seed, n_requests, n_scenes, slots_per_scene, params, sizes=((64, 64), (96, 96)), slots="window"):
    """Seeded request mix: n_env = floor(exp(U(0, ln 1025))) in [1, 1024], uniform scene and size, CTBR
    actions as in the batched workloads.  slots: "window" gives each scene's requests the next n_env of its
    env slots in turn (wrapping), as clients that each own their environments would: requests in flight
    together touch distinct slots until a scene's 4,096 slots wrap.  "random" draws distinct random slots
    of the scene for every request, so two requests of one scene almost always share a slot and are
    stepped one after the other."""
    rng = np.random.default_rng(seed)
    reqs = []
    cursor = [0] * n_scenes
    for _ in range(n_requests):
        n_env = int(min(1024, slots_per_scene, max(1, math.floor(math.exp(rng.uniform(0.0, math.log(1025.0)))))))
        sc = int(rng.integers(0, n_scenes))
        hw = sizes[int(rng.integers(0, len(sizes)))]
        if slots == "window":
            local = (cursor[sc] + np.arange(n_env)) % slots_per_scene
            cursor[sc] = (cursor[sc] + n_env) % slots_per_scene
        else:
            local = rng.choice(slots_per_scene, size=n_env, replace=False)
        slots_ = sc * slots_per_scene + local
        acts = np.empty((n_env, 4), dtype=np.float32)
        acts[:, 0] = rng.uniform(0.5, 2.0, n_env) * params["g"]
        acts[:, 1:] = rng.uniform(-3.0, 3.0, (n_env, 3))
        reqs.append((sc, hw, slots_.astype(np.int32), acts))
    return reqs


def run_load(server, scene_ids, reqs, rate=None, seed=0, device_out=None):
    """Submit requests (Poisson arrivals at `rate` per second, or all at once if rate is None);
    a collector thread waits for them in order.  Returns latencies (s), wall time, frames.
    device_out: a device float tensor the depth images go to (each request gets its own
    slice of a ring); otherwise results come back to host memory."""
    rng = np.random.default_rng(seed)
    tickets = []
    lock = threading.Condition()
    lat = []
    done_flag = [False]

    def collector():
        k = 0
        while True:
            with lock:
                while k >= len(tickets) and not done_flag[0]:
                    lock.wait()
                if k >= len(tickets):
                    return
                t = tickets[k]
            r = server.wait(t, fetch=False)
            lat.append(r["latency_s"])
            k += 1

    # all marshalling before the clock starts: the timed loop only paces and submits
    preps = []
    ring = 0
    for sc, hw, slots, acts in reqs:
        if device_out is not None:
            n_px = slots.shape[0] * hw[0] * hw[1]
            if ring + n_px > device_out.numel():
                ring = 0
            preps.append(server.prepare(scene_ids[sc], hw, slots, acts, out={"depth": device_out[ring:ring + n_px]},
                                        host_results=False))
            ring += n_px
        else:
            preps.append(server.prepare(scene_ids[sc], hw, slots, acts))
    th = threading.Thread(target=collector)
    th.start()
    t0 = time.perf_counter()
    next_t = t0
    frames = 0
    for (sc, hw, slots, acts), prep in zip(reqs, preps):
        if rate is not None:
            next_t += rng.exponential(1.0 / rate)
            gap = next_t - time.perf_counter()
            if gap > 3e-4:
                time.sleep(gap - 2e-4)
            while time.perf_counter() < next_t:
                pass
        t = server.submit_prepared(prep)
        frames += slots.shape[0]
        with lock:
            tickets.append(t)
            lock.notify()
    with lock:
        done_flag[0] = True
        lock.notify()
    th.join()
    wall = time.perf_counter() - t0
    return np.asarray(lat), wall, frames


# the room graphs are built with leaves of at most 3 triangles: their large flat faces traverse faster so
# (measured on the multi-scene batch; the forest prefers 4)
ROOM_LEAF_SIZE = 3


def bench_summary(sim_ctx, params, n_requests=4000, seed=7, n_streams=3):
    """Serving measurement over the eight multi-scene room graphs (see the module docstring)."""
    from workloads import agents, scenes
    from . import sim
    scs = scenes.multi_scene_set(seed=6)
    sim_ctx.set_bvh_leaf_size(ROOM_LEAF_SIZE)
    sids = [sim_ctx.build_scene(s["verts"], s["tris"], s["rgb"]) for s in scs]
    sim_ctx.set_bvh_leaf_size(4)
    per = 4096
    table = np.concatenate([agents.room_graph_starts(seed * 100 + j, per, scs[j], params) for j in range(8)])
    state = torch.as_tensor(table).cuda()
    # plain batched step on the same mix: 4096 agents, 8 scenes, half 64x64 half 96x96
    rng = np.random.default_rng(seed)
    n_plain = 4096
    slot_idx = rng.choice(state.shape[0], n_plain, replace=False).astype(np.int32)
    scene_of = slot_idx // per
    hw = np.where(rng.random(n_plain) < 0.5, 64, 96)
    views, npx, offs, mh, mw = sim.make_views(n_plain, np.asarray(sids)[scene_of], np.stack([hw, hw], 1))
    depth = torch.empty(npx, device="cuda")
    idx_t = torch.as_tensor(slot_idx).cuda()
    acts = torch.as_tensor(agents.random_actions(seed, 1, n_plain, params)[0]).cuda()
    p = capi.params_struct(params)
    for _ in range(3):
        sim_ctx.step(p, state, acts, views=views, env_idx=idx_t, max_hw=(mh, mw), depth=depth, out_pixels=npx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = 10
    for _ in range(reps):
        sim_ctx.step(p, state, acts, views=views, env_idx=idx_t, max_hw=(mh, mw), depth=depth, out_pixels=npx)
    torch.cuda.synchronize()
    plain_fps = n_plain * reps / (time.perf_counter() - t0)
    server = Server(sim_ctx, params, state, n_streams=n_streams, max_batch_agents=8192, max_hw=(96, 96),
                    budget_bytes=3 * (1 << 30))
    reqs = make_requests(seed, n_requests, 8, per, params)
    mean_env = float(np.mean([r[2].shape[0] for r in reqs]))
    ring = torch.empty(256 << 20 >> 2, dtype=torch.float32, device="cuda")     # 256 MiB of depth outputs
    lat, wall, frames = run_load(server, sids, reqs[:min(2000, n_requests)], rate=None, device_out=ring)
    sat_fps = frames / wall
    lam_server = sat_fps / mean_env
    lam_plain = plain_fps / mean_env        # the plain batched step's rate in requests of the mix
    out = {"workload": "8 room-graph scenes (20k-2M triangles), 4,096 resident env slots each, requests of "
                       "1-1,024 envs (log-uniform), 64x64 or 96x96, one step + render each, each scene's requests "
                       "on the scene's next env slots in turn, depth delivered to a device buffer",
           "requests_per_rate": n_requests, "mean_envs_per_request": mean_env,
           "plain_batched_frames_per_s": plain_fps, "saturated_frames_per_s": sat_fps,
           "saturated_fraction_of_plain": sat_fps / plain_fps,
           "lambda_sat_plain_requests_per_s": lam_plain, "saturated_requests_per_s": lam_server,
           "rates": [], "rates_of_server_saturation": []}
    for key, lam in (("rates", lam_plain), ("rates_of_server_saturation", lam_server)):
        for frac in (0.25, 0.5, 0.9):
            lat, wall, frames = run_load(server, sids, reqs, rate=frac * lam, seed=int(frac * 100), device_out=ring)
            out[key].append({"load": frac, "requests_per_s": frac * lam, "p50_ms": float(np.percentile(lat, 50) * 1e3),
                             "p99_ms": float(np.percentile(lat, 99) * 1e3), "frames_per_s": frames / wall,
                             "offered_frames_per_s": frac * lam * mean_env})
    out["server_stats"] = server.stats()
    server.close()
    for s in sids:
        sim_ctx.free_scene(s)
    return out
