"""Seeded procedural triangle scenes (stand-ins for the scan datasets of Sec. III-B).

Every generator returns a dict with
  ``verts``  float32 [V, 3]   world metres, z up
  ``tris``   int32   [T, 3]   vertex indices (winding is irrelevant: the
                              renderer is double-sided)
  ``rgb``    uint8   [T, 3]   flat per-triangle colour
plus generator metadata used only to place agents in free space.

Recipes (all values drawn from ``numpy.random.default_rng(seed)``):
  box_room   10 x 10 x 4 m room (faces split 2 x 2, 48 triangles) holding 12
             axis-aligned boxes with sides U(0.3, 2) m resting on the floor,
             192 triangles in total.
  forest     40 x 40 m ground quad plus open 32-segment cylinders ("trees")
             with radius U(0.1, 0.4) m and height U(3, 8) m; 2,000 trees give
             128,002 triangles.
  room_graph grid of 6 x 6 x 3 m rooms whose shared walls carry doorways on a
             random spanning tree plus about 20 % extra edges, filled with
             boxes and 16-segment floor-to-ceiling pillars until the triangle
             count is within 2 % of the target.
The paper trains in cluttered procedural scenes and scan datasets (Sec. III-B,
Sec. IV-A); those datasets are not available, so these recipes stand in.
"""
import math

import numpy as np

# ---------------------------------------------------------------------------
# mesh primitives (vectorised over K objects)
# ---------------------------------------------------------------------------

_BOX_TRIS = np.array([
    [0, 2, 6], [0, 6, 4],   # x = lo
    [1, 5, 7], [1, 7, 3],   # x = hi
    [0, 1, 5], [0, 5, 4],   # y = lo
    [2, 6, 7], [2, 7, 3],   # y = hi
    [0, 2, 3], [0, 3, 1],   # z = lo
    [4, 5, 7], [4, 7, 6],   # z = hi
], dtype=np.int64)


def boxes_mesh(lo, hi):
    """Closed axis-aligned boxes: lo, hi float [K,3] -> verts [8K,3], tris [12K,3]."""
    lo = np.asarray(lo, dtype=np.float64).reshape(-1, 3)
    hi = np.asarray(hi, dtype=np.float64).reshape(-1, 3)
    k = lo.shape[0]
    bits = np.array([[(i >> 0) & 1, (i >> 1) & 1, (i >> 2) & 1] for i in range(8)], dtype=bool)
    verts = np.where(bits[None, :, :], hi[:, None, :], lo[:, None, :]).reshape(k * 8, 3)
    tris = (_BOX_TRIS[None, :, :] + 8 * np.arange(k)[:, None, None]).reshape(k * 12, 3)
    return verts, tris


def cylinders_mesh(cx, cy, r, z0, z1, nseg):
    """Open vertical cylinders (side walls only): K cylinders -> 2*nseg*K verts and tris."""
    cx, cy, r, z0, z1 = (np.asarray(a, dtype=np.float64).reshape(-1) for a in (cx, cy, r, z0, z1))
    k = cx.shape[0]
    ang = 2.0 * np.pi * np.arange(nseg) / nseg
    ca, sa = np.cos(ang), np.sin(ang)
    bx = cx[:, None] + r[:, None] * ca[None, :]
    by = cy[:, None] + r[:, None] * sa[None, :]
    bottom = np.stack([bx, by, np.broadcast_to(z0[:, None], bx.shape)], axis=-1)
    top = np.stack([bx, by, np.broadcast_to(z1[:, None], bx.shape)], axis=-1)
    verts = np.concatenate([bottom, top], axis=1).reshape(k * 2 * nseg, 3)
    j = np.arange(nseg)
    jn = (j + 1) % nseg
    b0, b1, t0, t1 = j, jn, nseg + j, nseg + jn
    one = np.concatenate([np.stack([b0, b1, t1], -1), np.stack([b0, t1, t0], -1)], axis=0)
    tris = (one[None, :, :] + 2 * nseg * np.arange(k)[:, None, None]).reshape(k * 2 * nseg, 3)
    return verts, tris


def quads_mesh(corners):
    """Planar quads given as [K,4,3] corner arrays (in cyclic order) -> 2K triangles."""
    corners = np.asarray(corners, dtype=np.float64).reshape(-1, 4, 3)
    k = corners.shape[0]
    verts = corners.reshape(k * 4, 3)
    one = np.array([[0, 1, 2], [0, 2, 3]], dtype=np.int64)
    tris = (one[None] + 4 * np.arange(k)[:, None, None]).reshape(k * 2, 3)
    return verts, tris


def _axis_quad(axis, level, a0, a1, b0, b1):
    """Quad on the plane x_axis = level spanning [a0,a1] x [b0,b1] on the other two axes."""
    u, w = [i for i in range(3) if i != axis]
    c = np.zeros((4, 3))
    c[:, axis] = level
    c[:, u] = [a0, a1, a1, a0]
    c[:, w] = [b0, b0, b1, b1]
    return c


def _concat(parts):
    """Merge (verts, tris, rgb) parts into one mesh with re-based indices."""
    vs, ts, cs = [], [], []
    base = 0
    for v, t, c in parts:
        vs.append(v)
        ts.append(t + base)
        cs.append(np.broadcast_to(np.asarray(c, dtype=np.uint8).reshape(-1, 3), (t.shape[0], 3)))
        base += v.shape[0]
    return (np.concatenate(vs).astype(np.float32),
            np.concatenate(ts).astype(np.int32),
            np.ascontiguousarray(np.concatenate(cs)).astype(np.uint8))


def _scene(verts, tris, rgb, **meta):
    d = {"verts": verts, "tris": tris, "rgb": rgb}
    d.update(meta)
    return d


# ---------------------------------------------------------------------------
# small analytic test scenes
# ---------------------------------------------------------------------------

def floor_quad(half=50.0, z=0.0, rgb=(10, 20, 30)):
    """Square quad on the plane z = const, two triangles."""
    v, t = quads_mesh(_axis_quad(2, z, -half, half, -half, half)[None])
    return _scene(*_concat([(v, t, rgb)]))


def plane_quad(origin, e_u, e_v, rgb=(200, 100, 50)):
    """Parallelogram origin + s e_u + t e_v, s,t in [0,1], two triangles."""
    o, a, b = (np.asarray(x, dtype=np.float64) for x in (origin, e_u, e_v))
    v, t = quads_mesh(np.stack([o, o + a, o + a + b, o + b])[None])
    return _scene(*_concat([(v, t, rgb)]))


def box_interior(lo=(0.0, 0.0, 0.0), hi=(10.0, 10.0, 4.0), split=2):
    """Six inward faces of an axis-aligned box, each split split x split quads."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    quads, colours = [], []
    shade = {(0, 0): (150, 60, 60), (0, 1): (60, 150, 60), (1, 0): (60, 60, 150),
             (1, 1): (150, 150, 60), (2, 0): (120, 120, 120), (2, 1): (230, 230, 230)}
    for axis in range(3):
        u, w = [i for i in range(3) if i != axis]
        au = np.linspace(lo[u], hi[u], split + 1)
        aw = np.linspace(lo[w], hi[w], split + 1)
        for side, level in ((0, lo[axis]), (1, hi[axis])):
            for i in range(split):
                for j in range(split):
                    quads.append(_axis_quad(axis, level, au[i], au[i + 1], aw[j], aw[j + 1]))
                    colours.append(shade[(axis, side)])
    v, t = quads_mesh(np.stack(quads))
    rgb = np.repeat(np.asarray(colours, dtype=np.uint8), 2, axis=0)
    return _scene(v.astype(np.float32), t.astype(np.int32), rgb, lo=lo, hi=hi)


def icosphere(radius=1.0, subdiv=2, center=(0.0, 0.0, 0.0), rgb=(80, 160, 240)):
    """Subdivided icosahedron with every vertex on the sphere of the given radius."""
    p = (1.0 + math.sqrt(5.0)) / 2.0
    v = [(-1, p, 0), (1, p, 0), (-1, -p, 0), (1, -p, 0), (0, -1, p), (0, 1, p),
         (0, -1, -p), (0, 1, -p), (p, 0, -1), (p, 0, 1), (-p, 0, -1), (-p, 0, 1)]
    f = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4),
         (11, 10, 2), (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8),
         (3, 8, 9), (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    verts = [np.asarray(x, dtype=np.float64) / np.linalg.norm(x) for x in v]
    faces = list(f)
    for _ in range(subdiv):
        cache = {}

        def mid(a, b):
            key = (min(a, b), max(a, b))
            if key not in cache:
                m = verts[a] + verts[b]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]
        nf = []
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    vv = np.stack(verts) * radius + np.asarray(center, dtype=np.float64)
    tt = np.asarray(faces, dtype=np.int64)
    return _scene(*_concat([(vv, tt, rgb)]), radius=radius, center=np.asarray(center, dtype=np.float64))


# ---------------------------------------------------------------------------
# benchmark scenes
# ---------------------------------------------------------------------------

def box_room(seed=1, n_boxes=12, room=(10.0, 10.0, 4.0), start=(5.0, 5.0, 2.0), clearance=0.5):
    """10 x 10 x 4 m room with 12 boxes (192 triangles)."""
    rng = np.random.default_rng(seed)
    room_m = box_interior((0.0, 0.0, 0.0), room, split=2)
    start = np.asarray(start, dtype=np.float64)
    los, his = [], []
    while len(los) < n_boxes:
        size = rng.uniform(0.3, 2.0, size=3)
        cx = rng.uniform(size[0] / 2, room[0] - size[0] / 2)
        cy = rng.uniform(size[1] / 2, room[1] - size[1] / 2)
        lo = np.array([cx - size[0] / 2, cy - size[1] / 2, 0.0])
        hi = np.array([cx + size[0] / 2, cy + size[1] / 2, size[2]])
        gap = np.maximum(np.maximum(lo - start, start - hi), 0.0)
        if np.linalg.norm(gap) < clearance:
            continue
        los.append(lo)
        his.append(hi)
    bv, bt = boxes_mesh(np.stack(los), np.stack(his))
    box_rgb = np.repeat(rng.integers(0, 256, size=(n_boxes, 3)), 12, axis=0)
    verts, tris, rgb = _concat([(room_m["verts"].astype(np.float64), room_m["tris"].astype(np.int64), room_m["rgb"]),
                                (bv, bt, box_rgb)])
    return _scene(verts, tris, rgb, boxes=(np.stack(los), np.stack(his)), room=np.asarray(room), start=start)


def forest(seed=3, n_trees=2000, half=20.0, nseg=32):
    """Ground quad plus n_trees open cylinders (2 + 2*nseg*n_trees triangles)."""
    rng = np.random.default_rng(seed)
    cx = rng.uniform(-half, half, n_trees)
    cy = rng.uniform(-half, half, n_trees)
    r = rng.uniform(0.1, 0.4, n_trees)
    h = rng.uniform(3.0, 8.0, n_trees)
    col = rng.integers(0, 256, size=(n_trees, 3))
    gv, gt = quads_mesh(_axis_quad(2, 0.0, -half, half, -half, half)[None])
    tv, tt = cylinders_mesh(cx, cy, r, np.zeros(n_trees), h, nseg)
    verts, tris, rgb = _concat([(gv, gt, (96, 96, 96)), (tv, tt, np.repeat(col, 2 * nseg, axis=0))])
    return _scene(verts, tris, rgb, trees=np.stack([cx, cy, r, h], axis=1), half=half)


def room_graph_target(j):
    """Triangle target of the j-th multi-scene scene: round(2e4 * 100**(j/7)), j = 0..7."""
    return int(round(2.0e4 * 100.0 ** (j / 7.0)))


def room_graph(seed, target_tris, room=6.0, height=3.0, door_w=1.0, door_h=2.2, extra_door_p=0.2,
               tris_per_room=400, pillar_seg=16):
    """Grid of rooms joined by doorways, filled with boxes and pillars to ~target_tris triangles."""
    rng = np.random.default_rng(seed)
    g = max(2, int(round(math.sqrt(target_tris / tris_per_room))))
    # random spanning tree over the g x g room grid (randomised Kruskal) + extra doors
    edges = [((i, j), (i + 1, j)) for i in range(g - 1) for j in range(g)] + \
            [((i, j), (i, j + 1)) for i in range(g) for j in range(g - 1)]
    order = rng.permutation(len(edges))
    parent = list(range(g * g))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a
    door = np.zeros(len(edges), dtype=bool)
    for e in order:
        (i0, j0), (i1, j1) = edges[e]
        ra, rb = find(i0 * g + j0), find(i1 * g + j1)
        if ra != rb:
            parent[ra] = rb
            door[e] = True
    door |= rng.random(len(edges)) < extra_door_p
    quads = []
    for i in range(g):
        for j in range(g):
            x0, y0 = i * room, j * room
            quads.append(_axis_quad(2, 0.0, x0, x0 + room, y0, y0 + room))
            quads.append(_axis_quad(2, height, x0, x0 + room, y0, y0 + room))
    for e, ((i0, j0), (i1, j1)) in enumerate(edges):
        if i1 != i0:   # wall on plane x = const, spanning y
            axis, level, a0 = 0, (i0 + 1) * room, j0 * room
        else:          # wall on plane y = const, spanning x
            axis, level, a0 = 1, (j0 + 1) * room, i0 * room
        if door[e]:
            d0 = a0 + (room - door_w) / 2.0
            quads.append(_axis_quad(axis, level, a0, d0, 0.0, height))
            quads.append(_axis_quad(axis, level, d0 + door_w, a0 + room, 0.0, height))
            quads.append(_axis_quad(axis, level, d0, d0 + door_w, door_h, height))
        else:
            quads.append(_axis_quad(axis, level, a0, a0 + room, 0.0, height))
    ext = g * room
    for k in range(g):
        quads.append(_axis_quad(0, 0.0, k * room, (k + 1) * room, 0.0, height))
        quads.append(_axis_quad(0, ext, k * room, (k + 1) * room, 0.0, height))
        quads.append(_axis_quad(1, 0.0, k * room, (k + 1) * room, 0.0, height))
        quads.append(_axis_quad(1, ext, k * room, (k + 1) * room, 0.0, height))
    sv, st = quads_mesh(np.stack(quads))
    n_struct = st.shape[0]
    # objects: half boxes (12 triangles), half pillars (2*pillar_seg triangles)
    per_pair = 12 + 2 * pillar_seg
    n_pairs = max(0, int(round((target_tris - n_struct) / per_pair)))
    n_box = n_pairs
    n_pil = n_pairs
    rem = target_tris - (n_struct + n_pairs * per_pair)
    n_box += max(0, int(round(rem / 12)))
    room_of_box = rng.integers(0, g * g, n_box)
    room_of_pil = rng.integers(0, g * g, n_pil)
    size = rng.uniform(0.3, 2.0, size=(n_box, 3))
    bx = (room_of_box // g) * room + rng.uniform(size[:, 0] / 2, room - size[:, 0] / 2)
    by = (room_of_box % g) * room + rng.uniform(size[:, 1] / 2, room - size[:, 1] / 2)
    blo = np.stack([bx - size[:, 0] / 2, by - size[:, 1] / 2, np.zeros(n_box)], 1)
    bhi = np.stack([bx + size[:, 0] / 2, by + size[:, 1] / 2, size[:, 2]], 1)
    pr = rng.uniform(0.1, 0.4, n_pil)
    px = (room_of_pil // g) * room + rng.uniform(pr + 0.05, room - pr - 0.05)
    py = (room_of_pil % g) * room + rng.uniform(pr + 0.05, room - pr - 0.05)
    bv, bt = boxes_mesh(blo, bhi)
    pv, pt = cylinders_mesh(px, py, pr, np.zeros(n_pil), np.full(n_pil, height), pillar_seg)
    col_b = np.repeat(rng.integers(0, 256, size=(n_box, 3)), 12, axis=0)
    col_p = np.repeat(rng.integers(0, 256, size=(n_pil, 3)), 2 * pillar_seg, axis=0)
    wall_rgb = np.full((n_struct, 3), 180, dtype=np.uint8)
    verts, tris, rgb = _concat([(sv, st, wall_rgb), (bv, bt, col_b), (pv, pt, col_p)])
    return _scene(verts, tris, rgb, grid=g, room=room, height=height,
                  box_lo=blo, box_hi=bhi, pillars=np.stack([px, py, pr], 1))


def multi_scene_set(seed=6):
    """The eight room-graph scenes of the multi-scene workload (~20k ... ~2M triangles)."""
    return [room_graph(seed * 100 + j, room_graph_target(j)) for j in range(8)]
