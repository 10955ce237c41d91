"""Writes the oracle regression fixtures in this folder.  Calls only ``oracle/`` and ``workloads/``.

box_room_oracle.json: the single-agent box-room workload (Sec. III-A Eqs. 1-4
dynamics with RK4, Sec. III-B depth render): states after 10, 50 and 100 steps
and depth/id at 16 fixed pixels of the frame after step 100.  A later change of
the oracle's arithmetic that moves these numbers must name the passage that
justifies it.
"""
import json
import math
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import dynamics, render  # noqa: E402
from workloads import default_params, scenes, agents  # noqa: E402

PIXELS = [0, 63, 2016, 2080, 4032, 4095, 1000, 1234, 2345, 3456, 777, 3030, 64, 640, 2600, 3999]


def main():
    p = default_params()
    sc = scenes.box_room(seed=1)
    s0 = agents.box_room_start(p)
    acts = agents.random_actions(2, 100, 1, p)
    traj = dynamics.rollout(s0, acts, p)
    r = render.render_view(traj[100, 0], sc, 64, 64, math.pi / 2, pixels=np.array(PIXELS))
    out = {
        "citation": "Sec. III-A Eqs. (1)-(4) RK4 step; Sec. III-B depth render; box-room workload, seeds 1 (scene) and 2 (actions)",
        "writer": "tests/golden/make_golden.py (oracle only)",
        "states": {str(k): traj[k, 0].tolist() for k in (10, 50, 100)},
        "pixels": PIXELS,
        "depth": r["depth"].tolist(),
        "id": r["id"].tolist(),
        "mask": r["mask"].astype(int).tolist(),
    }
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "box_room_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
