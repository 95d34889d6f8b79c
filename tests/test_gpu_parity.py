"""Parity of the HIP renderer (through the C ABI) with the CPU oracle.

Bar: visible-triangle ids bit-exact, depth within 1e-5 relative, colour
within 1/255; per-view work counters (survivors, bbox pixel tests, covered
fragments) exactly equal to the oracle's.  Systems forms (tile size, bin
capacity with forced overflow, batching, graph replay) must reproduce the
plain per-view output bit for bit.
"""
import numpy as np
import pytest

import oracle
from scenegen import configs, make_apartment, random_walks
from tests.geom import IDENT_POSE, pose_at, quad, merge, unit_cube
from tests.gpu_common import NONE, compare, gpu_ctx, note, to_np
from tests.test_oracle_vs_raycast import random_scene

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = gpu_ctx()
    yield c
    c.close()


def render_gpu(ctx, pos, col, idx, W, H, poses, hfov=90.0, near=0.01, **kw):
    import paper_1904_01201_amd as P
    sc = ctx.upload(pos, col, idx)
    s = ctx.sensor(W, H, hfov, near, P.OUT_RGB | P.OUT_DEPTH)
    poses = np.asarray(poses, np.float32).reshape(-1, 12)
    out = ctx.alloc(s, poses.shape[0], tri=True)
    out = ctx.render(sc, s, poses, out=out, **kw)
    import torch
    torch.cuda.synchronize()
    res = [{k: v[i] for k, v in to_np(out).items()} for i in range(poses.shape[0])]
    stats = out.get("stats")
    ctx.release(sc)
    return res, stats


def check_views(ctx, pos, col, idx, W, H, poses, hfov=90.0, near=0.01, what="", stats=True):
    g, st = render_gpu(ctx, pos, col, idx, W, H, poses, hfov, near, stats=stats)
    nb = 0
    for k, p in enumerate(np.asarray(poses, np.float32).reshape(-1, 12)):
        o = oracle.render_view(pos, col, idx, W, H, p, hfov_deg=hfov, near_m=near)
        nb += compare(g[k], o, f"{what} view {k}")
        if stats:
            ost = o["stats"]
            assert st[k]["survivors"] == ost["survivors"], (what, k, st[k], ost)
            assert st[k]["bbox_tests"] == ost["bbox_tests"], (what, k, st[k], ost)
            assert st[k]["covered"] == ost["covered"], (what, k, st[k], ost)
    return nb


def test_closed_form_scenes(ctx):
    note("closed_form_scenes")
    pos, idx = unit_cube(-0.5, 0.5, 1.0, 2.0, -3.0, -2.0)
    check_views(ctx, pos, None, idx, 128, 128, pose_at(0, 1.5, 0), what="cube")
    pos2, idx2 = unit_cube(-0.5 + 1 / 64, 0.5 + 1 / 64, 1.0 + 1 / 64, 2.0 + 1 / 64, -3.0, -2.0)
    check_views(ctx, pos2, None, idx2, 128, 128, pose_at(0, 1.5, 0), what="cube shifted")
    f, fi = quad([-100, 0, 50], [100, 0, 50], [100, 0, -100], [-100, 0, -100])
    check_views(ctx, f, None, fi, 128, 128, pose_at(0, 1.5, 0), what="clipped floor")
    fl, fli = quad([-3, 0, -1], [3, 0, -1], [3, 0, -5], [-3, 0, -5])
    col = np.array([[10, 100, 200], [10, 100, 200], [170, 100, 200], [170, 100, 200]], np.uint8)
    check_views(ctx, fl, col, fli, 128, 128, pose_at(0, 1.5, 0), what="colour ramp")


def test_cube_counts_on_gpu(ctx):
    """The closed-form cube pin, read off the GPU output directly."""
    note("cube_counts")
    pos, idx = unit_cube(-0.5, 0.5, 1.0, 2.0, -3.0, -2.0)
    g, _ = render_gpu(ctx, pos, None, idx, 128, 128, pose_at(0, 1.5, 0))
    tri = g[0]["tri"]
    assert (tri != NONE).sum() == 1024 and (tri == 0).sum() == 528 and (tri == 1).sum() == 496


def test_room_all_poses(ctx):
    """room_2k_128: every one of the 100 poses."""
    note("room_2k_128 x100")
    w = configs.room_2k_128()
    sc = w.scenes[0]
    nb = check_views(ctx, sc.positions, sc.colors, sc.indices, 128, 128, w.poses[:, 0], what="room")
    note(f"room depth values not bit-identical: {nb}")


@pytest.mark.parametrize("seed", range(40))
def test_random_tiny_scenes(ctx, seed):
    """Random tiny scenes with near-plane crossings, coplanar duplicates,
    odd sizes and fields of view (the FP64 ray-caster scenes)."""
    pos, col, idx, W, H, hfov, pose = random_scene(1000 + seed)
    note(f"random scene {seed} T={idx.shape[0]} {W}x{H} hfov={hfov:.1f}")
    check_views(ctx, pos, col, idx, W, H, pose, hfov=hfov, what=f"random {seed}")


def test_apartment_sampled_walk(ctx):
    """apartment_200k_256: every 10th pose of the 1,000-step walk."""
    note("apartment_200k_256 sample")
    w = configs.apartment_200k_256()
    sc = w.scenes[0]
    poses = w.poses[::10, 0]
    check_views(ctx, sc.positions, sc.colors, sc.indices, 256, 256, poses, what="apartment")


def test_tile_size_and_capacity_invariance(ctx):
    """Tile size 8/16/32, a tiny bin capacity and a per-tile cap of 1 (every
    busy tile takes the overflow path) give bit-identical outputs."""
    note("tiling invariance")
    w = configs.room_2k_128()
    sc = w.scenes[0]
    poses = w.poses[:6, 0]
    ref, _ = render_gpu(ctx, sc.positions, sc.colors, sc.indices, 128, 128, poses, tile_size=16)
    for kw in ({"tile_size": 8}, {"tile_size": 32}, {"tile_size": 16, "tile_cap": 1},
               {"tile_size": 8, "bin_factor": 0.01}, {"tile_size": 32, "tile_cap": 3}):
        note(f"tiling {kw}")
        g, _ = render_gpu(ctx, sc.positions, sc.colors, sc.indices, 128, 128, poses, **kw)
        for a, b in zip(ref, g):
            for k in a:
                assert np.array_equal(a[k], b[k]), (kw, k)


def test_batch_equals_alone(ctx):
    """A heterogeneous batch (two scenes, 64/96/128 px, RGB-only, depth-only,
    RGB+D) reproduces each view rendered alone, bit for bit."""
    import torch
    import paper_1904_01201_amd as P
    note("batch vs alone")
    room = configs.room_2k_128().scenes[0]
    apt = make_apartment(seed=77, target_T=30_000)
    s_room, s_apt = ctx.upload_scene(room), ctx.upload_scene(apt)
    sensors = [ctx.sensor(128, 128), ctx.sensor(96, 64, 75.0, 0.05, P.OUT_DEPTH),
               ctx.sensor(64, 64, 100.0, 0.01, P.OUT_RGB)]
    poses_room = configs.room_2k_128().poses[:6, 0]
    poses_apt = random_walks(apt, 6, 3, seed=5)[-1]
    items, alone = [], []
    for k in range(12):
        scene = s_room if k % 2 == 0 else s_apt
        pose = poses_room[k // 2] if k % 2 == 0 else poses_apt[k // 2]
        sn = sensors[k % 3]
        o = ctx.alloc(sn, 1, tri=True)
        items.append((scene, sn, pose, o.get("rgb"), o.get("depth"), o.get("tri")))
        a = ctx.render(scene, sn, pose, out=ctx.alloc(sn, 1, tri=True))
        alone.append(a)
    ctx.render_batch(items)
    torch.cuda.synchronize()
    for k, (it, a) in enumerate(zip(items, alone)):
        for j, name in ((3, "rgb"), (4, "depth"), (5, "tri")):
            if it[j] is not None:
                assert torch.equal(it[j], a[name]), (k, name)
    ctx.release(s_room)
    ctx.release(s_apt)


def test_split_batch_equals_alone(ctx):
    """Batches of 32 views or more render as two halves side by side (eager
    batch, plain entry point, graph stepper): every view's output and work
    counters equal those of the view rendered alone, and so do the outputs
    at 31 views and with HAB_RENDER_ONE_SEQUENCE (one launch sequence)."""
    import torch
    note("split batch vs alone")
    room = configs.room_2k_128()
    apt = make_apartment(seed=78, target_T=20_000)
    s_room, s_apt = ctx.upload_scene(room.scenes[0]), ctx.upload_scene(apt)
    sn = ctx.sensor(64, 64)
    poses_room = room.poses[:20, 0]
    poses_apt = random_walks(apt, 20, 2, seed=6)[-1]
    for n in (41, 31):
        items, alone, alone_stats = [], [], []
        for k in range(n):
            scene, pose = ((s_room, poses_room[(k // 2) % 20]) if k % 2 == 0
                           else (s_apt, poses_apt[(k // 2) % 20]))
            o = ctx.alloc(sn, 1, tri=True)
            items.append((scene, sn, pose, o["rgb"], o["depth"], o["tri"]))
            a = ctx.render(scene, sn, pose, out=ctx.alloc(sn, 1, tri=True), stats=True)
            alone.append(a)
            alone_stats.append(a["stats"][0])
        for one in (False, True):
            for it in items:
                for j in (3, 4, 5):
                    it[j].zero_()
            stats = ctx.render_batch(items, stats=True, one_sequence=one)
            torch.cuda.synchronize()
            for k, (it, a) in enumerate(zip(items, alone)):
                for j, name in ((3, "rgb"), (4, "depth"), (5, "tri")):
                    assert torch.equal(it[j], a[name]), (n, one, k, name)
                assert stats[k] == alone_stats[k], (n, one, k)
        # the graph stepper over the same views, with host and device poses
        st = ctx.stepper(items)
        pz = np.stack([np.asarray(it[2], np.float32).reshape(12) for it in items])
        for how in ("host", "device"):
            for it in items:
                for j in (3, 4, 5):
                    it[j].zero_()
            if how == "host":
                st.step(pz)
            else:
                st.step_device(torch.from_numpy(pz).cuda())
            torch.cuda.synchronize()
            for k, (it, a) in enumerate(zip(items, alone)):
                for j, name in ((3, "rgb"), (4, "depth"), (5, "tri")):
                    assert torch.equal(it[j], a[name]), ("stepper", how, n, k, name)
        st.close()
    # the plain entry point: 40 poses of one scene in one call
    poses = np.concatenate([poses_room, poses_room[::-1]])
    got = ctx.render(s_room, sn, poses, out=ctx.alloc(sn, 40, tri=True), stats=True)
    torch.cuda.synchronize()
    for k in range(40):
        a = ctx.render(s_room, sn, poses[k], out=ctx.alloc(sn, 1, tri=True), stats=True)
        torch.cuda.synchronize()
        for name in ("rgb", "depth", "tri"):
            assert torch.equal(got[name][k], a[name][0]), ("plain", k, name)
        assert got["stats"][k] == a["stats"][0], ("plain", k)
    ctx.release(s_room)
    ctx.release(s_apt)


def test_lane_owned_and_balanced_z_tests_agree(ctx):
    """The atomic-free lane-owned z-test (HAB_RENDER_LANE_OWNED_Z) and the
    default balanced steps write the same bits at every tile size, through
    the overflow path, in the stepper, and match the oracle's work counters."""
    import torch
    note("lane-owned vs balanced z-test")
    room = configs.room_2k_128()
    apt = make_apartment(seed=79, target_T=60_000)
    s_room, s_apt = ctx.upload_scene(room.scenes[0]), ctx.upload_scene(apt)
    poses_apt = random_walks(apt, 8, 3, seed=7)[-1]
    cases = [(s_room, room.scenes[0], room.poses[:8, 0]), (s_apt, apt, poses_apt)]
    for h, sc, poses in cases:
        for W, H in ((128, 128), (200, 136)):
            sn = ctx.sensor(W, H)
            for opts in ({"tile_size": 8}, {"tile_size": 16}, {"tile_size": 32},
                         {"tile_size": 8, "tile_cap": 4}):
                a = ctx.render(h, sn, poses, out=ctx.alloc(sn, len(poses), tri=True), stats=True, **opts)
                b = ctx.render(h, sn, poses, out=ctx.alloc(sn, len(poses), tri=True), stats=True,
                               lane_owned_z=True, **opts)
                torch.cuda.synchronize()
                for k in ("rgb", "depth", "tri"):
                    assert torch.equal(a[k], b[k]), (W, H, opts, k)
                assert a["stats"] == b["stats"], (W, H, opts)
            o = oracle.render_view(sc.positions, sc.colors, sc.indices, W, H, poses[0])
            assert b["stats"][0]["covered"] == o["stats"]["covered"]
            assert np.array_equal(b["tri"].cpu().numpy()[0].view(np.uint32), o["tri"])
    # the stepper with the lane-owned z-test equals the eager default
    sn = ctx.sensor(128, 128)
    outs = [ctx.alloc(sn, 1, tri=True) for _ in range(4)]
    items = [(s_room, sn, room.poses[k, 0], o_["rgb"], o_["depth"], o_["tri"]) for k, o_ in enumerate(outs)]
    st = ctx.stepper(items, lane_owned_z=True)
    st.step(room.poses[10:14, 0])
    torch.cuda.synchronize()
    for k, o_ in enumerate(outs):
        ref = ctx.render(s_room, sn, room.poses[10 + k, 0], out=ctx.alloc(sn, 1, tri=True))
        torch.cuda.synchronize()
        for name in ("rgb", "depth", "tri"):
            assert torch.equal(o_[name], ref[name]), (k, name)
    st.close()
    ctx.release(s_room)
    ctx.release(s_apt)


def test_stepper_graph_replay(ctx):
    """Graph-captured steps: each replay (new poses) equals an eager batch
    render of the same poses; eager work runs between replays."""
    import torch
    note("stepper")
    w = configs.room_2k_128()
    sc = ctx.upload_scene(w.scenes[0])
    s = ctx.sensor(128, 128)
    outs = [ctx.alloc(s, 1, tri=True) for _ in range(4)]
    items = [(sc, s, w.poses[k, 0], o["rgb"], o["depth"], o["tri"]) for k, o in enumerate(outs)]
    st = ctx.stepper(items)
    for step in range(4):
        poses = w.poses[4 * step: 4 * step + 4, 0]
        st.step(poses)
        torch.cuda.synchronize()
        got = [{k: o[k].clone() for k in o} for o in outs]
        ref = [ctx.render(sc, s, p, out=ctx.alloc(s, 1, tri=True)) for p in poses]
        torch.cuda.synchronize()
        for a, b in zip(got, ref):
            for k in a:
                assert torch.equal(a[k], b[k]), (step, k)
    st.close()
    ctx.release(sc)


def test_plain_entry_point(ctx):
    """hab_render (no options) writes the same bits as hab_render_ex."""
    import torch
    note("hab_render")
    w = configs.room_2k_128()
    sc = ctx.upload_scene(w.scenes[0])
    s = ctx.sensor(128, 128)
    a = ctx.alloc(s, 5)
    ctx.render_plain(sc, s, w.poses[:5, 0], a["rgb"], a["depth"])
    b = ctx.render(sc, s, w.poses[:5, 0])
    torch.cuda.synchronize()
    assert torch.equal(a["rgb"], b["rgb"]) and torch.equal(a["depth"], b["depth"])
    ctx.release(sc)


def test_profile_phase_mask(ctx):
    """Only the selected phases are timed; an empty selection is refused."""
    import paper_1904_01201_amd as P
    note("profile phase mask")
    w = configs.room_2k_128()
    sc = ctx.upload_scene(w.scenes[0])
    s = ctx.sensor(128, 128)
    ctx.profile_phases(["raster8", "raster16", "raster32"])
    ctx.profile(True)
    ctx.render(sc, s, w.poses[:4, 0], tile_size=8)
    ctx.profile(False)
    ph = ctx.profile_read()
    ctx.profile_phases(None)
    assert set(ph) == {"raster8"} and ph["raster8"]["launches"] == 1, ph
    ctx.profile(True)
    ctx.render(sc, s, w.poses[:4, 0], tile_size=8)
    ctx.profile(False)
    assert {"reset", "setup", "raster8", "resolve"} <= set(ctx.profile_read())
    with pytest.raises(P.HabError):
        ctx.profile_phases([])
    ctx.release(sc)


def test_argument_errors(ctx):
    import paper_1904_01201_amd as P
    note("argument errors")
    pos, idx = quad([-1, -1, -2], [1, -1, -2], [1, 1, -2], [-1, 1, -2])
    sc = ctx.upload(pos, None, idx)
    s = ctx.sensor(64, 64)
    with pytest.raises(P.HabError) as e:
        ctx.render(sc, s, pose_at(0, 0, 1e6))
    assert e.value.status == P.HAB_ERR_RANGE
    with pytest.raises(P.HabError) as e:
        ctx.render(sc, s, pose_at(0, 0, 0, R=[[2, 0, 0], [0, 1, 0], [0, 0, 1]]))
    assert e.value.status == P.HAB_ERR_INVALID_ARG
    with pytest.raises(P.HabError) as e:
        ctx.upload(pos, None, idx + 7)
    assert e.value.status == P.HAB_ERR_INVALID_ARG
    # an unknown launch-option flag, on every entry point that takes options
    import ctypes as C
    from paper_1904_01201_amd import binding as B
    good, bad = B.RenderOpts(0, 0.0, 0, 3, None), B.RenderOpts(0, 0.0, 0, 4, None)
    o = ctx.alloc(s, 1)
    views = ctx.make_views([(sc, s, pose_at(0, 0, 0), o["rgb"], o["depth"], None)])
    assert ctx.lib.hab_render_batch(ctx.h, views, 1, C.byref(bad), None) == P.HAB_ERR_INVALID_ARG
    assert ctx.lib.hab_render_batch(ctx.h, views, 1, C.byref(good), None) == P.HAB_OK
    pc = B.poses_to_c(np.asarray(pose_at(0, 0, 0), np.float32).reshape(1, 12))
    assert ctx.lib.hab_render_ex(ctx.h, C.c_void_p(sc.ptr), C.byref(s), pc, 1, o["rgb"].data_ptr(),
                                 o["depth"].data_ptr(), None, C.byref(bad), None) == P.HAB_ERR_INVALID_ARG
    h = C.c_void_p()
    assert ctx.lib.hab_stepper_create(ctx.h, views, 1, C.byref(bad), None, C.byref(h)) == \
        P.HAB_ERR_INVALID_ARG
    assert ctx.get_error() == 0
    ctx.release(sc)
