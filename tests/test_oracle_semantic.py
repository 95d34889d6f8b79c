"""Pins of the oracle's semantic instance mask (Sec. 3 "Rendering engine":
one pass writes colour, depth and the semantic instance attachment).  The
expected values come from the geometry of the scenes, not from the lookup
the oracle performs."""
import json
import os

import numpy as np

from scenegen import scenes as S
from tests.geom import merge, pose_at, unit_cube

NONE = 0xFFFFFFFF
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_cube_face_on_instance_per_face(oracle_lib):
    """The face-on cube of the coverage golden (1024 pixels, all on the
    front face): with one id per face, the mask holds the front face's id
    on exactly those pixels and NONE elsewhere; with the two front triangles
    in different instances the split is the golden's 528 / 496."""
    pos, idx = unit_cube(-0.5, 0.5, 1.0, 2.0, -3.0, -2.0)
    exp = json.load(open(os.path.join(GOLDEN, "cube_face_on.json")))
    per_face = np.repeat(np.arange(100, 106, dtype=np.uint32), 2)
    r = oracle_lib.render_view(pos, None, idx, 128, 128, pose_at(0, 1.5, 0), instances=per_face)
    sem = r["semantic"]
    assert (sem == 100).sum() == exp["covered"]
    assert ((sem == 100) | (sem == NONE)).all()
    assert (sem[48:80, 48:80] == 100).all()
    split = np.array([7, 9] + [3] * 10, np.uint32)
    r = oracle_lib.render_view(pos, None, idx, 128, 128, pose_at(0, 1.5, 0), instances=split)
    assert (r["semantic"] == 7).sum() == exp["tri0"]
    assert (r["semantic"] == 9).sum() == exp["tri1"]
    assert (r["semantic"] == 3).sum() == 0


def test_two_cubes_side_by_side(oracle_lib):
    """Two unit cubes at z in [-3, -2], seen from (0, 1.5, 0) looking -Z (w
    = 2 at the front, f = 64, 128^2): the left one's front face covers
    columns [16, 48), the right one's [80, 112), rows [48, 80); their inner
    side faces show too, each on its own half of the image.  Cube instance
    ids 11 and 4 (the larger id first, so an order mix-up shows): each id
    covers exactly the pixels its cube covers when rendered alone, all on
    its own half."""
    a = unit_cube(-1.5, -0.5, 1.0, 2.0, -3.0, -2.0)
    b = unit_cube(0.5, 1.5, 1.0, 2.0, -3.0, -2.0)
    pos, idx = merge(a, b)[:2]
    inst = np.array([11] * 12 + [4] * 12, np.uint32)
    pose = pose_at(0, 1.5, 0)
    r = oracle_lib.render_view(pos, None, idx, 128, 128, pose, instances=inst)
    sem = r["semantic"]
    alone_a = oracle_lib.render_view(a[0], None, a[1], 128, 128, pose)["tri"] != NONE
    alone_b = oracle_lib.render_view(b[0], None, b[1], 128, 128, pose)["tri"] != NONE
    assert ((sem == 11) == alone_a).all() and ((sem == 4) == alone_b).all()
    assert (sem[48:80, 16:48] == 11).all() and (sem[48:80, 80:112] == 4).all()
    assert not (sem[:, 64:] == 11).any() and not (sem[:, :64] == 4).any()
    assert ((sem == NONE) == ~(alone_a | alone_b)).all()


def test_room_ceiling_is_one_instance(oracle_lib):
    """From 0.3 m below the middle of a room's ceiling, looking straight up
    with a 90-degree field of view, only a 0.6 m square of the ceiling (rect
    1 of the room, 200 triangles on a grid of cells over 0.4 m) is in view:
    several triangles, one instance, every pixel."""
    sc = S.make_room(5)
    Lx, Lz = sc.meta["Lx"], sc.meta["Lz"]
    R_up = [[1, 0, 0], [0, 0, -1], [0, 1, 0]]          # camera -Z -> world +Y
    pose = pose_at(Lx / 2, S.ROOM_HEIGHT - 0.3, Lz / 2, R_up)
    r = oracle_lib.render_view(sc.positions, sc.colors, sc.indices, 64, 64, pose,
                               instances=sc.instances)
    assert len(np.unique(r["tri"])) > 1
    assert (r["semantic"] == 1).all()


def test_room_box_faces_share_one_instance(oracle_lib):
    """Looking down at 35 degrees along a box's diagonal from above its (+x,
    +z) corner, 2.5 m up (under the 2.8 m ceiling), shows its top and two
    sides: three faces' triangles (8 per face), all carrying the box's one
    id (box 0 of room 5: instance 6, after the six room surfaces)."""
    sc = S.make_room(5)
    inst = 6
    bt = np.nonzero(sc.instances == inst)[0]
    assert bt.size == 40
    h = float(sc.positions[sc.indices[bt].ravel()][:, 1].max())
    x0, z0, x1, z1 = sc.boxes[0]
    target = np.array([(x0 + x1) / 2, h / 2, (z0 + z1) / 2])
    d = np.array([-1.0, -1.0, -1.0]) / np.sqrt(3.0)     # world view direction
    eye = target - (2.5 - h / 2) * np.sqrt(3.0) * d
    right = np.cross(d, [0.0, 1.0, 0.0])
    right /= np.linalg.norm(right)
    R = np.stack([right, np.cross(right, d), -d], axis=1)   # columns: camera axes
    pose = np.concatenate([eye, R.ravel()]).astype(np.float32)
    r = oracle_lib.render_view(sc.positions, sc.colors, sc.indices, 96, 96, pose,
                               instances=sc.instances)
    on_box = np.isin(r["tri"], bt)
    faces = np.unique((r["tri"][on_box] - bt[0]) // 8)
    assert faces.tolist() == [0, 2, 4]          # top, +x side, +z side
    assert on_box.sum() > 300
    assert ((r["semantic"] == inst) == on_box).all()


def test_scene_instance_tables():
    """Generator tables: one id per structural surface, one per box; a
    box's 40 (room) triangles share it; ids are dense from 0."""
    sc = S.make_room(2, num_boxes=7)
    assert sc.instances.shape == (sc.num_triangles,) and sc.instances.dtype == np.uint32
    counts = np.bincount(sc.instances)
    assert counts.tolist() == [200] * 6 + [40] * 7
    ap = S.make_apartment(1, 20000)
    n_inst = int(ap.instances.max()) + 1
    assert np.unique(ap.instances).size == n_inst
    assert n_inst - len(ap.boxes) > 8          # structural surfaces of 8 rooms
    assert (np.diff(ap.instances.astype(np.int64)) >= 0).all()
