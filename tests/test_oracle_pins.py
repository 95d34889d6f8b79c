"""Closed-form pins for the CPU oracle.

Every expected value here is derived by hand from the camera model or the
geometry (the derivation sits in each docstring), never read off the oracle.
Paper anchors: the sensor (256^2, 90 degree field of view, depth sharing
pose and intrinsics) is Sec. 4 "Sensory input"; the single-pass colour +
depth + semantic render is Sec. 3 "Rendering engine".
"""
import json
import os

import numpy as np
import pytest

from tests.geom import IDENT_POSE, pose_at, quad, merge, unit_cube

NONE = 0xFFFFFFFF
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def ulp_diff(a, b):
    a = np.asarray(a, np.float32).view(np.int32).astype(np.int64)
    b = np.asarray(b, np.float32).view(np.int32).astype(np.int64)
    return np.abs(a - b)


# --------------------------------------------------------------- a1 / C2
def test_paper_sensor_constants(oracle_lib):
    """The paper's sensor: 256^2 at 90 degrees (fixture cites Sec. 4).  With a
    90 degree field of view, f = W / (2 tan 45 deg) = W / 2 exactly."""
    spec = json.load(open(os.path.join(GOLDEN, "paper_sensor.json")))
    W = spec["resolution"]
    assert oracle_lib.focal(W, spec["hfov_deg"]) == W / 2
    for w in (128, 256, 512, 1000, 4096):
        assert oracle_lib.focal(w, 90.0) == w / 2


def test_focal_60_degrees(oracle_lib):
    """tan 30 deg = 1/sqrt(3), so f = W sqrt(3) / 2, rounded once to fp32."""
    for w in (96, 100, 640):
        assert oracle_lib.focal(w, 60.0) == np.float32(w * np.sqrt(3.0) / 2.0)


def test_projection_closed_form(oracle_lib):
    """W = H = 128, 90 degrees: f = 64, principal point (64, 64).  A camera
    point (1, 0, -2) lands at x = 64 + 64 * 1/2 = 96 px -> X = 96 * 256 =
    24576; y = 64 -> Y = 16384.  (0, 1, -4): y = 64 - 64/4 = 48 -> 12288."""
    assert oracle_lib.project_point([1, 0, -2], IDENT_POSE, 128, 128) == (24576, 16384, 0.5)
    assert oracle_lib.project_point([0, 1, -4], IDENT_POSE, 128, 128)[:2] == (16384, 12288)
    assert oracle_lib.project_point([0, 0, 1], IDENT_POSE, 128, 128) is None      # behind


def test_rotation_convention(oracle_lib):
    """R is world-from-camera, row-major.  R = [[0,0,1],[0,1,0],[-1,0,0]] makes
    the camera look along world -X.  World point (-2, 0, -1) relative to the
    camera is d = (-2, 0, -1); camera coords R^T d = (1, 0, -2), so it lands
    at X = 24576 as above.  The camera position is subtracted first."""
    R = [[0, 0, 1], [0, 1, 0], [-1, 0, 0]]
    assert oracle_lib.project_point([-2, 0, -1], pose_at(0, 0, 0, R), 128, 128)[:2] == (24576, 16384)
    assert oracle_lib.project_point([3, 5, 6], pose_at(5, 5, 7, R), 128, 128)[:2] == (24576, 16384)


def test_snap_rounds_half_to_even(oracle_lib):
    """Camera x = 1 + 2^-14 at w = 2: cxS + (x fS) rw = 16384 + 16385 * 0.5 =
    24576.5 exactly -> 24576 (even).  x = 1 + 3 * 2^-14 -> 24577.5 -> 24578."""
    a = oracle_lib.project_point([1 + 2 ** -14, 0, -2], IDENT_POSE, 128, 128)
    b = oracle_lib.project_point([1 + 3 * 2 ** -14, 0, -2], IDENT_POSE, 128, 128)
    assert a[0] == 24576 and b[0] == 24578


# --------------------------------------------------------------- C7 / C8
def cube_scene(dx=0.0, dy=0.0):
    pos, idx = unit_cube(-0.5 + dx, 0.5 + dx, 1.0 + dy, 2.0 + dy, -3.0, -2.0)
    return pos, idx


def test_cube_face_on(oracle_lib):
    """Camera at (0, 1.5, 0) looking -Z, 128^2, 90 deg (f = 64).  The front
    face z = -2 (w = 2) spans x, y in [64 - 16, 64 + 16] = [48, 80] px, so
    pixel centres i + 1/2 in (48, 80) are i = 48..79: 32 x 32 = 1024 pixels,
    all at depth 2.  The face diagonal runs from (48, 48) to (80, 80) through
    the 32 centres (i + 1/2, i + 1/2); the triangle above it (x > y, id 0)
    has the diagonal as an owned edge (it points up-left, dy < 0), so it gets
    32 * 31 / 2 + 32 = 528 pixels and the other triangle (id 1) 496.  Every
    other face of the cube lies behind the front face."""
    pos, idx = cube_scene()
    r = oracle_lib.render_view(pos, None, idx, 128, 128, pose_at(0, 1.5, 0))
    hit = r["tri"] != NONE
    exp = json.load(open(os.path.join(GOLDEN, "cube_face_on.json")))
    assert hit.sum() == exp["covered"]
    assert set(np.unique(r["tri"][hit]).tolist()) == {0, 1}
    assert (r["tri"] == 0).sum() == exp["tri0"] and (r["tri"] == 1).sum() == exp["tri1"]
    ys, xs = np.nonzero(hit)
    assert ys.min() == 48 and ys.max() == 79 and xs.min() == 48 and xs.max() == 79
    diag = np.arange(48, 80)
    assert (r["tri"][diag, diag] == 0).all()
    assert ulp_diff(r["depth"][hit], 2.0).max() <= 6
    assert (r["depth"][~hit] == 0).all() and (r["rgb"][~hit] == 0).all()
    assert (r["rgb"][hit] == 255).all()


def test_cube_half_pixel_shift(oracle_lib):
    """Shift the cube by half a pixel at w = 2 (1/64 m) right and up: the
    left and top face edges now pass through pixel centres (x = 48.5,
    y = 47.5).  Left and top edges are owned (inclusive), right and bottom
    edges are not, so the silhouette is still exactly 32 x 32 = 1024 pixels,
    now columns 48..79 and rows 47..78."""
    pos, idx = cube_scene(dx=1.0 / 64.0, dy=1.0 / 64.0)
    r = oracle_lib.render_view(pos, None, idx, 128, 128, pose_at(0, 1.5, 0))
    hit = r["tri"] != NONE
    assert hit.sum() == 1024
    ys, xs = np.nonzero(hit)
    assert (xs.min(), xs.max(), ys.min(), ys.max()) == (48, 79, 47, 78)


def test_wall_depth_and_parallel_walls(oracle_lib):
    """A wall at distance 3.7 that fills the view: every pixel has depth 3.7
    (fp32) up to the rounding of the interpolation: the key is a sum of
    three products scaled by 1/A (each op 1/2 ulp, 1/A 1 ulp) and depth is
    its reciprocal: at most ~5 ulp, asserted as 6.  A second, farther wall
    with a smaller id never shows."""
    far = quad([-50, -50, -5.0], [50, -50, -5.0], [50, 50, -5.0], [-50, 50, -5.0])
    near = quad([-40, -40, -3.7], [40, -40, -3.7], [40, 40, -3.7], [-40, 40, -3.7])
    pos, idx, _ = merge(far, near)
    r = oracle_lib.render_view(pos, None, idx, 96, 64, IDENT_POSE)
    assert (r["tri"] >= 2).all() and (r["tri"] != NONE).all()
    assert ulp_diff(r["depth"], np.float32(3.7)).max() <= 6


def test_duplicate_triangle_tie_goes_to_smaller_id(oracle_lib):
    """Two identical triangles give bit-identical keys everywhere; the rule
    keeps the smaller index, whichever comes first."""
    t = quad([-1, -1, -2], [1, -1, -2], [1, 1, -2], [-1, 1, -2])
    pos = np.concatenate([t[0], t[0]])
    idx = np.array([[4, 5, 6], [0, 1, 2], [0, 2, 3], [4, 6, 7]], np.uint32)  # dup of 1 is 0, of 2 is 3
    r = oracle_lib.render_view(pos, None, idx, 64, 64, IDENT_POSE)
    vals = set(np.unique(r["tri"]).tolist()) - {NONE}
    assert vals == {0, 2}


def test_floor_depth_rows(oracle_lib):
    """Floor y = 0 from z = -0.5 to -100 (|x| <= 100) under a level camera at
    height h = 1.5, 128^2, f = 64.  A pixel row j sees the floor iff its
    centre is below the principal point (j + 1/2 > 64) and the ray reaches
    the floor within z in [-100, -0.5]; the hit has planar depth
    d = h f / (j + 1/2 - 64).  1/d is affine in screen y with gradient
    1/(h f) per px; snapping moves each vertex by at most sqrt(2)/512 px and
    a convex combination keeps that bound, so the relative depth error is
    at most sqrt(2) / (512 (j + 1/2 - 64)) plus fp32 rounding (1e-6)."""
    pos, idx = quad([-100, 0, -0.5], [100, 0, -0.5], [100, 0, -100], [-100, 0, -100])
    r = oracle_lib.render_view(pos, None, idx, 128, 128, pose_at(0, 1.5, 0))
    h, f = 1.5, 64.0
    for j in range(128):
        dy = j + 0.5 - 64
        d = h * f / dy if dy > 0 else np.inf
        row = r["depth"][j]
        if dy > 0 and 0.5 < d < 100 * 0.999:
            # the floor's side edges at |x| = 100 are outside the view here
            assert (r["tri"][j] != NONE).all(), j
            rel = np.abs(row.astype(np.float64) - d) / d
            assert rel.max() <= np.sqrt(2) / (512 * dy) + 1e-6, (j, rel.max())
        elif dy <= 0 or d > 100 * 1.001:
            assert (r["tri"][j] == NONE).all(), j


def test_near_clipped_floor_depth(oracle_lib):
    """Same floor, now extending behind the camera (z from +50 to -100) so
    that the triangles under the camera straddle the near plane and get
    clipped.  Every row below the horizon is covered and depths follow
    h f / (j + 1/2 - 64) within the same snapping bound as the unclipped
    floor.  Here the clip points are exact in fp32 (the clipped edges run
    along x or z, so the interpolated coordinate equals both end points), and
    the only extra error is 1/near rounded once (1/2 ulp, weighted by the clip
    vertex's small barycentric weight): 1e-6 more is allowed for it."""
    pos, idx = quad([-100, 0, 50], [100, 0, 50], [100, 0, -100], [-100, 0, -100])
    r = oracle_lib.render_view(pos, None, idx, 128, 128, pose_at(0, 1.5, 0))
    assert r["stats"]["clipped"] == 2
    for j in range(65, 128):
        dy = j + 0.5 - 64
        d = 1.5 * 64.0 / dy
        assert (r["tri"][j] != NONE).all()
        rel = (np.abs(r["depth"][j].astype(np.float64) - d) / d).max()
        assert rel <= np.sqrt(2) / (512 * dy) + 2e-6, (j, rel)
    assert (r["tri"][:64] == NONE).all()


def test_colour_ramp_perspective_correct(oracle_lib):
    """A floor quad (z from -1 to -5) whose red channel is affine in world z:
    red = 10 + 40 (-z - 1), i.e. 10 at the near edge and 170 at the far
    edge; green = 100, blue = 200.  The camera at height 1.5 sees row j at
    planar depth d = 96 / (j + 1/2 - 64), where the true red is
    10 + 40 (d - 1).  The oracle must match within 1 (rounding), while
    screen-affine interpolation would be off by far more."""
    pos, idx = quad([-3, 0, -1], [3, 0, -1], [3, 0, -5], [-3, 0, -5])
    col = np.array([[10, 100, 200], [10, 100, 200], [170, 100, 200], [170, 100, 200]], np.uint8)
    r = oracle_lib.render_view(pos, col, idx, 128, 128, pose_at(0, 1.5, 0))
    max_aff = 0.0
    y_near, y_far = 64 + 96 / 1.0, 64 + 96 / 5.0
    for j in range(128):
        dy = j + 0.5 - 64
        if dy <= 0:
            continue
        d = 96.0 / dy
        if not (1.0 < d < 5.0):
            continue
        cols = slice(64 - 8, 64 + 8)
        exp = 10 + 40 * (d - 1)
        got = r["rgb"][j, cols].astype(np.float64)
        assert np.abs(got[:, 0] - exp).max() <= 1.0, (j, got[:, 0], exp)
        assert (got[:, 1] == 100).all() and (got[:, 2] == 200).all()
        aff = 10 + 160 * (y_near - (j + 0.5)) / (y_near - y_far)
        max_aff = max(max_aff, abs(aff - exp))
    assert max_aff > 20        # the test discriminates against affine shading


# --------------------------------------------------------------- C4
def test_near_clip_vertex_counts(oracle_lib):
    """A triangle with 0, 1, 2 or 3 vertices behind the near plane renders
    as 1, 2 (quad), 1 (triangle) or 0 sub-triangles; every visible pixel
    keeps the parent index."""
    base = np.array([[-1, -1, -2], [1, -1, -2], [0, 1, -2]], np.float32)
    idx = np.array([[0, 1, 2]], np.uint32)
    cases = {0: (1, 0), 1: (2, 1), 2: (1, 1), 3: (0, 0)}
    for behind, (subs, clipped) in cases.items():
        p = base.copy()
        p[:behind, 2] = 0.5        # behind the camera (w = -0.5)
        r = oracle_lib.render_view(p, None, idx, 64, 64, IDENT_POSE)
        assert r["stats"]["survivors"] == subs, behind
        assert r["stats"]["clipped"] == clipped
        vals = set(np.unique(r["tri"]).tolist()) - {NONE}
        assert vals == ({0} if subs else set())


# --------------------------------------------------------------- C7 fill rule
def centre(i, j, w=1.0, W=128):
    """Camera point at depth w that projects to pixel centre (i+1/2, j+1/2)
    for f = 64 (W = 128): x = 64 + 64 X/w -> X = (i + 1/2 - 64) w / 64."""
    return [(i + 0.5 - 64) * w / 64.0, -(j + 0.5 - 64) * w / 64.0, -w]


def test_fill_rule_square_on_centres(oracle_lib):
    """A square whose corners sit on the centres of pixels (10,10), (20,10),
    (20,20), (10,20): its left and top edges are owned, right and bottom are
    not, so exactly columns 10..19 x rows 10..19 are covered, each once."""
    pos, idx = quad(centre(10, 10), centre(20, 10), centre(20, 20), centre(10, 20))
    cnt, st = oracle_lib.coverage_count(pos, idx, 128, 128, IDENT_POSE)
    exp = np.zeros((128, 128), np.uint32)
    exp[10:20, 10:20] = 1
    assert (cnt == exp).all()
    # the other diagonal split gives the same pixels
    pos2 = pos[[1, 2, 3, 0]]
    cnt2, _ = oracle_lib.coverage_count(pos2, idx, 128, 128, IDENT_POSE)
    assert (cnt2 == exp).all()


def test_fill_rule_fan_around_centre(oracle_lib):
    """Eight triangles fanned around a vertex placed on the centre of pixel
    (30, 30), with rim vertices on pixel centres: the shared vertex's pixel
    is covered exactly once and so is every pixel inside the fan."""
    c = centre(30, 30)
    rim = [centre(30 + dx, 30 + dy) for dx, dy in
           [(7, 0), (7, 7), (0, 7), (-7, 7), (-7, 0), (-7, -7), (0, -7), (7, -7)]]
    pos = np.array([c] + rim, np.float32)
    idx = np.array([[0, 1 + k, 1 + (k + 1) % 8] for k in range(8)], np.uint32)
    cnt, _ = oracle_lib.coverage_count(pos, idx, 128, 128, IDENT_POSE)
    assert cnt[30, 30] == 1
    assert cnt.max() == 1
    # the fan is the square [23, 37]^2 of centres: left/top owned
    exp = np.zeros((128, 128), np.uint32)
    exp[23:37, 23:37] = 1
    assert (cnt == exp).all()


def test_fill_rule_horizontal_and_vertical_edges(oracle_lib):
    """A triangle with a horizontal edge through row-40 centres includes that
    row when the triangle lies below it (a top edge) and excludes it when the
    triangle lies above it (a bottom edge).  Same for a vertical edge through
    column-40 centres: included on the left side of the shape, excluded on
    the right side."""
    below = np.array([centre(30, 40), centre(50, 40), centre(40, 50)], np.float32)
    above = np.array([centre(30, 40), centre(50, 40), centre(40, 30)], np.float32)
    right_of = np.array([centre(40, 30), centre(40, 50), centre(50, 40)], np.float32)
    left_of = np.array([centre(40, 30), centre(40, 50), centre(30, 40)], np.float32)
    idx = np.array([[0, 1, 2]], np.uint32)
    c = lambda p: oracle_lib.coverage_count(p, idx, 128, 128, IDENT_POSE)[0]
    assert c(below)[40, 31:49].all() and c(below)[40, 35] == 1
    assert not c(above)[40].any()
    assert c(right_of)[31:49, 40].all()
    assert not c(left_of)[:, 40].any()


# --------------------------------------------------------------- degenerate
def test_degenerate_triangles(oracle_lib):
    """Collinear or repeated vertices give A = 0: nothing is drawn."""
    pos = np.array([[-1, 0, -2], [0, 0, -2], [1, 0, -2], [0.5, 0.5, -2]], np.float32)
    idx = np.array([[0, 1, 2], [3, 3, 1], [0, 0, 0]], np.uint32)
    r = oracle_lib.render_view(pos, None, idx, 64, 64, IDENT_POSE)
    assert (r["tri"] == NONE).all() and r["stats"]["survivors"] == 0


def test_empty_and_all_behind(oracle_lib):
    pos = np.zeros((3, 3), np.float32)
    r = oracle_lib.render_view(pos, None, np.zeros((0, 3), np.uint32), 32, 16, IDENT_POSE)
    assert (r["tri"] == NONE).all() and (r["depth"] == 0).all() and (r["rgb"] == 0).all()
    pos, idx = quad([-1, -1, 2], [1, -1, 2], [1, 1, 2], [-1, 1, 2])
    r = oracle_lib.render_view(pos, None, idx, 32, 16, IDENT_POSE)
    assert (r["tri"] == NONE).all() and r["stats"]["survivors"] == 0


# --------------------------------------------------------------- domain / args
def test_pose_domain_check(oracle_lib):
    """D f 256 / near + W 128 < 2^28.  With f = 64, near = 0.01: D < ~163.8 m."""
    lo, hi = np.array([0, 0, 0], np.float32), np.array([10, 3, 10], np.float32)
    assert oracle_lib.pose_check(lo, hi, pose_at(5, 1.5, 5), 128, 128) == 0
    assert oracle_lib.pose_check(lo, hi, pose_at(5, 1.5, 170), 128, 128) == oracle_lib.OR_ERR_RANGE
    bad = pose_at(5, 1.5, 5, R=[[1, 0, 0], [0, 1, 0], [0, 0, 1.1]])
    assert oracle_lib.pose_check(lo, hi, bad, 128, 128) == oracle_lib.OR_ERR_INVALID_ARG


def test_invalid_arguments(oracle_lib):
    from oracle.binding import OracleError
    pos, idx = quad([-1, -1, -2], [1, -1, -2], [1, 1, -2], [-1, 1, -2])
    with pytest.raises(OracleError):
        oracle_lib.render_view(pos, None, idx + 10, 8, 8, IDENT_POSE)
    with pytest.raises(OracleError):
        oracle_lib.render_view(pos, None, idx, 8, 8, IDENT_POSE, hfov_deg=180.0)
    with pytest.raises(OracleError):
        oracle_lib.render_view(pos, None, idx, 0, 8, IDENT_POSE)


def test_tiny_fronto_parallel_triangles_exact_depth(oracle_lib):
    """Small triangles (a fraction of a pixel to a few pixels) facing the
    camera at depth 2.5: 1/w is constant over each, so every covered pixel
    reads 2.5 up to the same ~5 ulp of rounding as the wall.  With tiny
    areas the 1/A factor is what carries the depth, so this pins it."""
    rng = np.random.default_rng(3)
    tris = []
    for k in range(200):
        c = rng.uniform(-0.9, 0.9, size=2) * 2.5
        s = rng.uniform(0.01, 0.1)
        tris.append([[c[0], c[1], -2.5], [c[0] + s, c[1], -2.5], [c[0], c[1] + s * rng.uniform(0.5, 2), -2.5]])
    pos = np.array(tris, np.float32).reshape(-1, 3)
    idx = np.arange(len(pos), dtype=np.uint32).reshape(-1, 3)
    r = oracle_lib.render_view(pos, None, idx, 128, 128, IDENT_POSE)
    hit = r["tri"] != NONE
    assert hit.sum() > 200
    assert ulp_diff(r["depth"][hit], np.float32(2.5)).max() <= 6


# --------------------------------------------------------------- work counters
# The per-view counters are the algorithmic work the benchmark's roofline
# figure is built from (Sec. 3 "Performance": cost grows with the number of
# triangles drawn and the pixels they cover).  survivors = sub-triangles with
# a non-empty box of pixel centres in the viewport, bbox_tests = the number
# of those centres, covered = (sub-triangle, pixel) pairs that pass the
# coverage test, whether or not they win the depth test.
def corner(x, y, w=1.0):
    """Camera point at depth w that projects to the pixel corner (x, y) px
    of a 128^2, 90 degree sensor (f = 64)."""
    return [(x - 64) * w / 64.0, -(y - 64) * w / 64.0, -w]


def stats_of(oracle_lib, pos, idx, W=128):
    return oracle_lib.render_view(pos, None, idx, W, W, IDENT_POSE)["stats"]


def test_counters_square_on_pixel_corners(oracle_lib):
    """A square with corners on the pixel corners (10, 30) and (20, 40): each
    half's box of centres is columns 10..19 x rows 30..39 (a centre i + 1/2
    lies inside [10, 20] for i = 10..19), 100 each; the two halves cover
    each of the 100 pixels exactly once."""
    pos, idx = quad(corner(10, 30), corner(20, 30), corner(20, 40), corner(10, 40))
    st = stats_of(oracle_lib, pos, idx)
    assert (st["survivors"], st["bbox_tests"], st["covered"]) == (2, 200, 100)


def test_counters_right_triangle_on_centres(oracle_lib):
    """Legs on pixel centres: vertices at the centres of (20, 20), (20 + n,
    20) and (20, 20 + n).  Its box holds (n + 1)^2 centres; under the
    top-left rule the top and left legs are owned and the hypotenuse is
    not, so exactly the centres (20 + u, 20 + v) with u, v >= 0, u + v < n
    are covered: n (n + 1) / 2."""
    for n in (1, 2, 5, 13):
        pos = np.array([centre(20, 20), centre(20 + n, 20), centre(20, 20 + n)], np.float32)
        idx = np.array([[0, 1, 2]], np.uint32)
        st = stats_of(oracle_lib, pos, idx)
        assert (st["survivors"], st["bbox_tests"], st["covered"]) == (1, (n + 1) ** 2, n * (n + 1) // 2), n
        # the other winding gives the same counts
        st = stats_of(oracle_lib, pos, idx[:, [0, 2, 1]])
        assert (st["bbox_tests"], st["covered"]) == ((n + 1) ** 2, n * (n + 1) // 2), n


def test_counters_box_clamped_to_the_viewport(oracle_lib):
    """A square over pixel corners x in [-10, 10], y in [120, 140] of a 128^2
    view: only columns 0..9 and rows 120..127 hold centres in the viewport,
    so each half counts 10 x 8 = 80 tests, and 80 pixels are covered; a
    square entirely left of the viewport has no survivor."""
    pos, idx = quad(corner(-10, 120), corner(10, 120), corner(10, 140), corner(-10, 140))
    st = stats_of(oracle_lib, pos, idx)
    assert (st["survivors"], st["bbox_tests"], st["covered"]) == (2, 160, 80)
    pos, idx = quad(corner(-30, 50), corner(-10, 50), corner(-10, 60), corner(-30, 60))
    st = stats_of(oracle_lib, pos, idx)
    assert (st["survivors"], st["bbox_tests"], st["covered"]) == (0, 0, 0)


def test_counters_count_fragments_hidden_by_the_depth_test(oracle_lib):
    """Two squares over the same 10 x 10 pixels, the nearer one (w = 1) drawn
    first and the farther one (w = 2) second: both pass coverage on all 100
    pixels, so covered = 200 although the farther one wins none."""
    near = quad(corner(10, 30, 1.0), corner(20, 30, 1.0), corner(20, 40, 1.0), corner(10, 40, 1.0))
    far = quad(corner(10, 30, 2.0), corner(20, 30, 2.0), corner(20, 40, 2.0), corner(10, 40, 2.0))
    pos, idx, _ = merge(near, far)
    r = oracle_lib.render_view(pos, None, idx, 128, 128, IDENT_POSE)
    st = r["stats"]
    assert (st["survivors"], st["bbox_tests"], st["covered"]) == (4, 400, 200)
    assert set(np.unique(r["tri"][r["tri"] != NONE]).tolist()) == {0, 1}


def test_counters_face_on_cube(oracle_lib):
    """The face-on unit cube (see test_cube_face_on): the front face's two
    triangles have corners on the pixel corners (48, 48)..(80, 80), so each
    box holds 32 x 32 centres and together they cover the 1024 pixels once.
    Its back face (w = 3, half-width 0.5 m) spans x and y in
    [64 - 32/3, 64 + 32/3] = [53.33, 74.67] px: centres 53..74, 22 x 22,
    so 2 x 484 tests and 484 covered.  Side faces seen edge-on project to zero
    area and are dropped, except the four visible through perspective
    (left, right, top, bottom faces between w = 2 and 3), whose counts are
    the oracle's business; the front face's share is exact."""
    pos, idx = cube_scene()
    st = stats_of(oracle_lib, pos, idx[:2])
    assert (st["survivors"], st["bbox_tests"], st["covered"]) == (2, 2048, 1024)
    st = stats_of(oracle_lib, pos, idx[2:4])
    assert (st["survivors"], st["bbox_tests"], st["covered"]) == (2, 2 * 484, 484)


def test_counters_degenerate_and_empty(oracle_lib):
    """Degenerate triangles and geometry behind the camera count nothing."""
    pos = np.array([[-1, 0, -2], [0, 0, -2], [1, 0, -2], [0.5, 0.5, -2]], np.float32)
    idx = np.array([[0, 1, 2], [3, 3, 1], [0, 0, 0]], np.uint32)
    st = stats_of(oracle_lib, pos, idx, 64)
    assert (st["survivors"], st["bbox_tests"], st["covered"]) == (0, 0, 0)
    pos, idx = quad(corner(10, 30, -1.0), corner(20, 30, -1.0), corner(20, 40, -1.0), corner(10, 40, -1.0))
    st = stats_of(oracle_lib, pos, idx)
    assert (st["survivors"], st["bbox_tests"], st["covered"]) == (0, 0, 0)
