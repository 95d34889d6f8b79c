"""Edge cases of the render path on the GPU, against the oracle: the
largest sensor (4096^2: 262,144 tiles, binned through the global-atomic
path for views beyond the LDS tile budget), one-row / one-column / one-pixel
sensors, a scene without triangles, a view with nothing in front of it, and
an empty batch."""
import numpy as np
import pytest

import oracle
from scenegen import configs
from tests.geom import pose_at
from tests.gpu_common import NONE, compare, gpu_ctx, note, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = gpu_ctx()
    yield c
    c.close()


def aabb_of(sc):
    return sc.positions.min(axis=0), sc.positions.max(axis=0)


def render_one(ctx, h, sn, pose):
    import torch
    o = ctx.alloc(sn, 1, tri=True)
    ctx.render_batch([(h, sn, pose, o.get("rgb"), o.get("depth"), o["tri"])])
    torch.cuda.synchronize()
    return {k: v[0] for k, v in to_np(o).items()}


def test_largest_sensor(ctx):
    """f = 2048 px: with the default 1 cm near plane a room-sized scene can
    snap outside the fixed-point domain (D f 256 / near > 2^28), which the
    library refuses before rendering; at 5 cm it fits."""
    import paper_1904_01201_amd as P
    note("edges: 4096^2 room view")
    w = configs.room_2k_128()
    sc = w.scenes[0]
    h = ctx.upload_scene(sc)
    pose = w.poses[3, 0]
    with pytest.raises(P.HabError) as e:
        render_one(ctx, h, ctx.sensor(4096, 4096), pose)
    assert e.value.status == P.HAB_ERR_RANGE
    assert oracle.pose_check(*aabb_of(sc), pose, 4096, 4096) == oracle.OR_ERR_RANGE
    sn = ctx.sensor(4096, 4096, 90.0, 0.05)
    g = render_one(ctx, h, sn, pose)
    o = oracle.render_view(sc.positions, sc.colors, sc.indices, 4096, 4096, pose, near_m=0.05)
    compare(g, o, "4096^2")
    assert (g["tri"] != NONE).mean() > 0.5
    ctx.release(h)


@pytest.mark.parametrize("W,H", [(4096, 1), (1, 4096), (1, 1), (3, 517)])
def test_thin_and_tiny_sensors(ctx, W, H):
    note(f"edges: {W}x{H}")
    w = configs.room_2k_128()
    sc = w.scenes[0]
    h = ctx.upload_scene(sc)
    sn = ctx.sensor(W, H, 70.0, 0.05)
    for k in (0, 7):
        g = render_one(ctx, h, sn, w.poses[k, 0])
        o = oracle.render_view(sc.positions, sc.colors, sc.indices, W, H, w.poses[k, 0], hfov_deg=70.0,
                               near_m=0.05)
        compare(g, o, f"{W}x{H} view {k}")
    ctx.release(h)


def test_scene_without_triangles_and_view_of_nothing(ctx):
    note("edges: empty scene, nothing in view")
    pos = np.array([[0, 0, -2], [1, 0, -2], [0, 1, -2]], np.float32)
    empty = ctx.upload(pos, None, np.zeros((0, 3), np.uint32))
    sn = ctx.sensor(64, 48)
    g = render_one(ctx, empty, sn, pose_at(0, 0, 0))
    assert (g["tri"] == NONE).all() and (g["depth"] == 0).all() and (g["rgb"] == 0).all()
    one = ctx.upload(pos, None, np.array([[0, 1, 2]], np.uint32))
    g = render_one(ctx, one, sn, pose_at(0, 0, 0, [[-1, 0, 0], [0, 1, 0], [0, 0, -1]]))  # facing away
    assert (g["tri"] == NONE).all() and (g["depth"] == 0).all()
    g = render_one(ctx, one, sn, pose_at(0, 0, 0))
    o = oracle.render_view(pos, None, np.array([[0, 1, 2]], np.uint32), 64, 48, pose_at(0, 0, 0))
    compare(g, o, "one triangle")
    assert (g["tri"] == 0).sum() > 100
    ctx.render_batch([])                     # an empty batch is a no-op
    assert ctx.get_error() == 0
    ctx.release(empty)
    ctx.release(one)


def test_largest_batch(ctx):
    """4,096 views in one launch sequence (the most one sequence holds: the
    per-view prefix in setup's and binning's LDS is at its largest), 16 x 12
    depth views: a sample against the oracle; 4,097 views are split into two
    sequences, the last view checked too."""
    import torch
    import paper_1904_01201_amd as P
    note("edges: 4096-view batch")
    w = configs.room_2k_128()
    sc = w.scenes[0]
    h = ctx.upload_scene(sc)
    sn = ctx.sensor(16, 12, 90.0, 0.01, P.OUT_DEPTH)
    n = 4096
    poses = w.poses[np.arange(n) % w.poses.shape[0], np.arange(n) % w.poses.shape[1]]
    out = ctx.alloc(sn, n, tri=True)
    items = [(h, sn, poses[k], None, out["depth"][k], out["tri"][k]) for k in range(n)]
    ctx.render_batch(items)
    torch.cuda.synchronize()
    g = to_np(out)
    for k in range(0, n, 257):
        o = oracle.render_view(sc.positions, sc.colors, sc.indices, 16, 12, poses[k])
        compare({"depth": g["depth"][k], "tri": g["tri"][k]}, o, f"view {k}")
    extra = ctx.alloc(sn, 1, tri=True)
    ctx.render_batch(items + [(h, sn, poses[5], None, extra["depth"], extra["tri"])])
    torch.cuda.synchronize()
    o = oracle.render_view(sc.positions, sc.colors, sc.indices, 16, 12, poses[5])
    compare({k: v[0] for k, v in to_np(extra).items()}, o, "view 4096 (second sequence)")
    assert ctx.get_error() == 0
    ctx.release(h)
