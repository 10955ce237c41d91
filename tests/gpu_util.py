"""Shared helpers of the GPU parity tests (device side through the C ABI, oracle on the host)."""
import math

import numpy as np

DEPTH_RTOL = 1e-4     # depth tolerance off the edge/tie mask
STATE_TOL = 1e-5      # |s_gpu - s_oracle| <= STATE_TOL * max(1, |s_oracle|) per component


RECORDS = []          # (test, fields) of measured errors and bounds, printed in the terminal summary


def header(msg):
    print(f"[gpu-test] {msg}", flush=True)


def record(name, **fields):
    """Keep a measured figure (an error and its bound, a count) for the end-of-run summary, which pytest
    prints even under -q; also echoed at once."""
    RECORDS.append((name, fields))
    print(f"[gpu-record] {name} " + " ".join(f"{k}={_fmt(v)}" for k, v in fields.items()), flush=True)


def _fmt(v):
    return f"{v:.3e}" if isinstance(v, float) else str(v)


def format_records():
    return [f"{name} " + " ".join(f"{k}={_fmt(v)}" for k, v in fields.items()) for name, fields in RECORDS]


def compare_render(depth, tri_id, rgb, ref, miss_depth, label=""):
    """Element-wise comparison of one agent's image against the oracle's render_view() result.

    Off the oracle's edge/tie mask: ids bit-exact, colours bit-exact, depth within
    DEPTH_RTOL relative (misses: the miss depth exactly).  Returns the masked fraction.
    """
    mask = np.asarray(ref["mask"]).reshape(-1)
    ok = ~mask
    d_o = np.asarray(ref["depth"]).reshape(-1)
    id_o = np.asarray(ref["id"]).reshape(-1)
    depth = np.asarray(depth).reshape(-1)
    tri_id = np.asarray(tri_id).reshape(-1)
    bad_id = ok & (tri_id != id_o)
    assert not bad_id.any(), f"{label}: {bad_id.sum()} ids differ off-mask, e.g. pixel {np.nonzero(bad_id)[0][:5]}"
    hit = ok & (id_o >= 0)
    rel = np.abs(depth[hit] - d_o[hit]) / np.maximum(np.abs(d_o[hit]), 1e-30)
    assert rel.size == 0 or rel.max() <= DEPTH_RTOL, f"{label}: depth rel err {rel.max():.3e}"
    miss = ok & (id_o < 0)
    assert np.all(depth[miss] == np.float32(miss_depth)), f"{label}: miss depth differs"
    if rgb is not None:
        rgb = np.asarray(rgb).reshape(3, -1)
        rgb_o = np.asarray(ref["rgb"]).reshape(3, -1)
        assert np.array_equal(rgb[:, ok], rgb_o[:, ok]), f"{label}: colours differ off-mask"
    return float(mask.mean())


def state_close(s_gpu, s_ref, tol=STATE_TOL):
    s_gpu = np.asarray(s_gpu, dtype=np.float64)
    s_ref = np.asarray(s_ref, dtype=np.float64)
    err = np.abs(s_gpu - s_ref) / np.maximum(1.0, np.abs(s_ref))
    return float(err.max())


def hfov90():
    return math.pi / 2
