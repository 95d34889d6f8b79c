"""Pins of the oracle's obstacle extraction from the mesh and its free-space
test (Sec. 4 "Agent embodiment and action space": a 0.2 m-diameter, 1.5 m
cylinder; "Collision dynamics": the agent slides along the scene's own walls
and obstacles).

Obstacles are the mesh's horizontal cross-sections at given heights across
the agent's body; a disc is free when every cross-section segment is at
least its radius away.  Closed forms: a wall quad cut at height h gives two
collinear pieces meeting where its diagonal crosses h and spanning the wall
exactly; a pillar gives its footprint's four edges; a doorway leaves its gap
open below the lintel; floors, ceilings and low boxes give nothing; a tilted
triangle's cut lands on the interpolated edge points.  The free-space test
is pinned by exact distances to a wall, an endpoint and a point obstacle,
and, on a generated apartment, against the generator's own description of
its walls and boxes (independent code and data).
"""
import numpy as np
import pytest

from scenegen import make_apartment, nav_segments
from tests.geom import merge, quad

H = 2.8


def wall(x0, x1, z, y0=0.0, y1=H):
    """Vertical quad along x at depth z, split along its (x0, y0)-(x1, y1)
    diagonal."""
    return quad([x0, y0, z], [x1, y0, z], [x1, y1, z], [x0, y1, z])


def union_x(segs):
    """Sorted x intervals of collinear segments along x."""
    iv = sorted((min(s[0], s[2]), max(s[0], s[2])) for s in segs)
    out = []
    for a, b in iv:
        if out and a <= out[-1][1]:
            out[-1][1] = max(out[-1][1], b)
        else:
            out.append([a, b])
    return out


def test_wall_cut_closed_form(oracle_lib):
    """Wall from x = 1 to 5 at z = -2.  Triangle (a, b, c) = ((1,0), (5,0),
    (5,2.8)) is cut at height h on edges b->c (x = 5) and c->a (the
    diagonal, x = 1 + 4 h / 2.8); the other triangle (a, c, d) on the
    diagonal and on d->a (x = 1).  Both pieces lie on z = -2 and together
    span [1, 5] exactly."""
    pos, idx = wall(1.0, 5.0, -2.0)
    for h in (0.1, 0.75, 1.5):
        s = oracle_lib.nav_slice(pos, idx, [h])
        xd = np.float32(1.0 + 4.0 * (h / H))
        assert s.shape == (2, 4)
        assert (s[:, 1] == -2.0).all() and (s[:, 3] == -2.0).all()
        assert {tuple(sorted((a, b))) for a, b in s[:, [0, 2]]} == {(xd, 5.0), (1.0, xd)}, (h, s)
        assert union_x(s) == [[1.0, 5.0]]


def test_heights_multiply_and_order(oracle_lib):
    """One segment per (triangle, height) that cuts it, in triangle-major
    order: K heights over the wall give 2 K segments, triangle 0's first."""
    pos, idx = wall(0.0, 2.0, 0.0)
    hs = [0.1, 0.5, 1.0, 1.5]
    s = oracle_lib.nav_slice(pos, idx, hs)
    assert s.shape == (8, 4)
    # triangle 0 = ((0,0),(2,0),(2,2.8)): its cuts end at x = 2 on edge b->c
    assert (np.maximum(s[:4, 0], s[:4, 2]) == 2.0).all()
    assert (np.minimum(s[4:, 0], s[4:, 2]) == 0.0).all()
    diag = np.float32(np.array(hs) * (2.0 / H))
    assert np.array_equal(np.minimum(s[:4, 0], s[:4, 2]), diag)


def test_pillar_footprint(oracle_lib):
    """A closed box x in [1, 1.4], z in [2, 2.4], y in [0, 2.8]: every cut
    strictly between floor and top is its footprint's four edges (two
    pieces each); the horizontal top and bottom faces give nothing."""
    from tests.geom import unit_cube
    pos, idx = unit_cube(1.0, 1.4, 0.0, H, 2.0, 2.4)
    s = oracle_lib.nav_slice(pos, idx, [0.1, 1.5])
    assert s.shape == (16, 4)          # 4 side faces x 2 triangles x 2 heights
    pts = {(round(float(x), 6), round(float(z), 6)) for x, z in s.reshape(-1, 2)}
    corners = {(1.0, 2.0), (1.4, 2.0), (1.0, 2.4), (1.4, 2.4)}
    assert corners <= pts
    xs, zs = s.reshape(-1, 2)[:, 0], s.reshape(-1, 2)[:, 1]
    on_edge = (np.isclose(xs, 1.0) | np.isclose(xs, 1.4)) | (np.isclose(zs, 2.0) | np.isclose(zs, 2.4))
    assert on_edge.all()
    assert xs.min() == np.float32(1.0) and xs.max() == np.float32(1.4)


def test_doorway_gap_and_lintel(oracle_lib):
    """A wall at z = 0 from x = 0 to 4 with a 0.9 x 2.1 m doorway at
    x in [1.5, 2.4], built as left, right and lintel rectangles: below 2.1 m
    the gap is open, above it the lintel closes it."""
    m = merge(wall(0.0, 1.5, 0.0), wall(2.4, 4.0, 0.0), wall(1.5, 2.4, 0.0, 2.1, H))
    s = oracle_lib.nav_slice(m[0], m[1], [0.1, 1.5])
    assert union_x(s) == [[0.0, 1.5], [np.float32(2.4), 4.0]]
    s = oracle_lib.nav_slice(m[0], m[1], [2.5])
    assert union_x(s) == [[0.0, 4.0]]


def test_floor_ceiling_and_low_boxes(oracle_lib):
    """Horizontal floor (y = 0) and ceiling (y = 2.8) quads give nothing at
    body heights; a 0.05 m box gives nothing at 0.1 m; a 0.3 m box gives its
    footprint at 0.1 m only."""
    from tests.geom import unit_cube
    floor = quad([0, 0, 0], [5, 0, 0], [5, 0, 5], [0, 0, 5])
    ceil = quad([0, H, 0], [5, H, 0], [5, H, 5], [0, H, 5])
    low = unit_cube(1.0, 1.5, 0.0, 0.05, 1.0, 1.5)
    mid = unit_cube(3.0, 3.5, 0.0, 0.3, 3.0, 3.5)
    hs = [0.1, 0.5, 1.0, 1.5]
    assert oracle_lib.nav_slice(*merge(floor, ceil, low)[:2], hs).shape[0] == 0
    s = oracle_lib.nav_slice(mid[0], mid[1], hs)
    assert s.shape == (8, 4)
    xs, zs = s[:, [0, 2]].ravel(), s[:, [1, 3]].ravel()
    assert xs.min() == 3.0 and xs.max() == 3.5 and zs.min() == 3.0 and zs.max() == 3.5
    assert ((xs == 3.0) | (xs == 3.5) | (zs == 3.0) | (zs == 3.5)).all()   # on the footprint's edges


def test_tilted_triangle_and_vertex_on_plane(oracle_lib):
    """Vertices (0,0,0), (2,2,0), (0,2,2) cut at y = 1: edge v0->v1 at
    (1, 0), edge v2->v0 (interpolated from v0 upwards) at (0, 1).  A vertex
    exactly at the height counts as above: cut at y = 2 the triangle has
    v0 below and v1, v2 above, so the segment joins v1 and v2 themselves."""
    pos = np.array([[0, 0, 0], [2, 2, 0], [0, 2, 2]], np.float32)
    idx = np.array([[0, 1, 2]], np.uint32)
    s = oracle_lib.nav_slice(pos, idx, [1.0])
    assert s.tolist() == [[1.0, 0.0, 0.0, 1.0]]
    s = oracle_lib.nav_slice(pos, idx, [2.0])
    assert s.tolist() == [[2.0, 0.0, 0.0, 2.0]]
    assert oracle_lib.nav_slice(pos, idx, [2.5, -0.5]).shape[0] == 0


def test_free_space_exact_distances(oracle_lib):
    """Wall (0,0)-(4,0), r = 0.25: a point at distance 0.25 is
    free (the disc touches), at 0.25 - 2^-20 it is blocked; beyond the end
    the distance is to the endpoint (3-4-5 triangle scaled: (4.15, 0.2) is
    0.25 from (4, 0)); a zero-length segment is a point obstacle; no
    segments: free."""
    w = np.array([[0.0, 0.0, 4.0, 0.0]], np.float32)
    r = 0.25
    f = lambda pts, seg=w: oracle_lib.nav_free(seg, pts, r).tolist()
    assert f([[2.0, 0.25], [2.0, -0.25]]) == [True, True]
    assert f([[2.0, 0.25 - 2 ** -20], [0.0, -0.25 + 2 ** -20]]) == [False, False]
    assert f([[4.15, 0.2], [4.15, 0.2 - 2 ** -20], [-0.15, -0.2]]) == [True, False, True]
    pt = np.array([[1.0, 1.0, 1.0, 1.0]], np.float32)
    assert f([[1.25, 1.0], [1.0, 1.0 + 0.25 - 2 ** -20]], pt) == [True, False]
    assert oracle_lib.nav_free(np.zeros((0, 4), np.float32), [[0, 0]], r).tolist() == [True]


def test_apartment_free_space_matches_the_generator(oracle_lib):
    """On an unjittered generated apartment the walls are vertical quads on
    the generator's wall segments and the boxes' sides stand on their
    footprints, so the mesh's cross-section at 0.1 m (plus one at 1.5 m)
    blocks a 0.1 m disc exactly where the generator's own wall and box
    description puts an obstacle within 0.1 m (points within 1e-6 m of that
    threshold skipped); the doorways stay passable."""
    sc = make_apartment(seed=5, target_T=20_000)
    segs = oracle_lib.nav_slice(sc.positions, sc.indices, [0.1, 1.5])
    meta = nav_segments(sc).astype(np.float64)
    rng = np.random.default_rng(1)
    b = sc.bounds
    pts = np.stack([rng.uniform(b[0] + 0.01, b[2] - 0.01, 3000), rng.uniform(b[1] + 0.01, b[3] - 0.01, 3000)], 1)
    # distance to the generator's segments, computed here independently
    ax, az, bx, bz = (meta[:, k][None, :] for k in range(4))
    ex, ez = bx - ax, bz - az
    L2 = np.maximum(ex * ex + ez * ez, 1e-300)
    t = np.clip(((pts[:, :1] - ax) * ex + (pts[:, 1:] - az) * ez) / L2, 0, 1)
    d = np.hypot(ax + t * ex - pts[:, :1], az + t * ez - pts[:, 1:]).min(axis=1)
    keep = np.abs(d - 0.1) > 1e-6
    got = oracle_lib.nav_free(segs, pts[keep], 0.1)
    assert np.array_equal(got, d[keep] >= 0.1), int((got != (d[keep] >= 0.1)).sum())
    assert 0.05 < (~got).mean() < 0.95
