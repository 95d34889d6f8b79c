"""Semantic instance sensor on the GPU (the third attachment of the single
render pass, Sec. 3 "Rendering engine").

The mask is the instance id of each pixel's visible triangle, so its bar is
the triangle id's: bit-exact with the oracle.  Covered: closed-form and room
views, an apartment walk, ragged resolutions and semantic-only sensors in a
heterogeneous batch, the captured stepper, the server, the full-size
64-environment batch, and the errors (no instance table, wrong table size).
"""
import numpy as np
import pytest

import oracle
from scenegen import configs, make_apartment, random_walks
from tests.geom import merge, pose_at, unit_cube
from tests.gpu_common import (NONE, check_any_size, compare, gpu_ctx, note, oracle_compare_many,
                              to_np)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = gpu_ctx()
    yield c
    c.close()


def _sem_sensor(ctx, W, H, hfov=90.0, near=0.01, extra=None):
    import paper_1904_01201_amd as P
    outs = P.OUT_RGB | P.OUT_DEPTH | P.OUT_SEMANTIC if extra is None else extra | P.OUT_SEMANTIC
    return ctx.sensor(W, H, hfov, near, outs)


def _render_batch_np(ctx, scene_h, sensor, poses):
    import torch
    outs = [ctx.alloc(sensor, 1, tri=True) for _ in poses]
    items = [(scene_h, sensor, p, o.get("rgb"), o.get("depth"), o["tri"], o["semantic"])
             for p, o in zip(poses, outs)]
    ctx.render_batch(items)
    torch.cuda.synchronize()
    return [{k: v[0] for k, v in to_np(o).items()} for o in outs]


def test_two_cubes_closed_form(ctx):
    """Two face-on cubes with ids 11 (left) and 4 (right): each id covers
    its own cube's pixels, the 32 x 32 front blocks included."""
    note("semantic: two cubes")
    a = unit_cube(-1.5, -0.5, 1.0, 2.0, -3.0, -2.0)
    b = unit_cube(0.5, 1.5, 1.0, 2.0, -3.0, -2.0)
    pos, idx = merge(a, b)[:2]
    inst = np.array([11] * 12 + [4] * 12, np.uint32)
    h = ctx.upload(pos, None, idx, instances=inst)
    sn = _sem_sensor(ctx, 128, 128)
    g = _render_batch_np(ctx, h, sn, [pose_at(0, 1.5, 0)])[0]
    sem = g["semantic"]
    assert (sem[48:80, 16:48] == 11).all() and (sem[48:80, 80:112] == 4).all()
    o = oracle.render_view(pos, None, idx, 128, 128, pose_at(0, 1.5, 0), instances=inst)
    compare(g, o, "two cubes")
    ctx.release(h)


def test_room_views(ctx):
    """All 16 environments' first poses of the 2k-triangle room at 128^2."""
    note("semantic: room views")
    w = configs.room_2k_128()
    sc = w.scenes[0]
    h = ctx.upload_scene(sc)
    sn = _sem_sensor(ctx, 128, 128)
    poses = w.poses[:16, 0]
    g = _render_batch_np(ctx, h, sn, poses)
    for k, p in enumerate(poses):
        o = oracle.render_view(sc.positions, sc.colors, sc.indices, 128, 128, p,
                               instances=sc.instances)
        compare(g[k], o, f"room view {k}")
        hit = o["tri"] != NONE
        assert len(np.unique(g[k]["semantic"][hit])) >= 1
    ctx.release(h)


def test_apartment_walk_ragged(ctx):
    """A 100k-triangle apartment walk at a ragged 200 x 136 (tiles cut on
    both axes), 75-degree field of view, semantic + depth only."""
    import paper_1904_01201_amd as P
    note("semantic: apartment walk 200x136")
    apt = make_apartment(seed=21, target_T=100_000, jitter_sigma=0.01)
    h = ctx.upload_scene(apt)
    sn = _sem_sensor(ctx, 200, 136, 75.0, 0.05, extra=P.OUT_DEPTH)
    poses = random_walks(apt, 30, 4, seed=3)[::6].reshape(-1, 12)
    g = _render_batch_np(ctx, h, sn, poses)
    for k, p in enumerate(poses):
        o = oracle.render_view(apt.positions, apt.colors, apt.indices, 200, 136, p,
                               hfov_deg=75.0, near_m=0.05, instances=apt.instances)
        compare(g[k], o, f"apartment view {k}")
    ctx.release(h)


def test_mixed_batch_semantic_only_and_without(ctx):
    """One batch: the same scene with a semantic-only sensor (97 x 61), an
    RGB+D+semantic sensor and a plain RGB+D sensor; a scene uploaded
    without a table rides along with RGB+D.  Every view equals its oracle
    and the RGB+D views equal a batch without any semantic view."""
    import torch
    import paper_1904_01201_amd as P
    note("semantic: mixed batch")
    room = configs.room_2k_128().scenes[0]
    apt = make_apartment(seed=5, target_T=40_000)
    h_room = ctx.upload_scene(room)
    h_apt = ctx.upload_scene(apt)
    h_plain = ctx.upload(room.positions, room.colors, room.indices)   # no table
    s_only = ctx.sensor(97, 61, 90.0, 0.01, P.OUT_SEMANTIC)
    s_all = _sem_sensor(ctx, 128, 96)
    s_rgbd = ctx.sensor(128, 96)
    poses_room = configs.room_2k_128().poses[:4, 0]
    poses_apt = random_walks(apt, 10, 2, seed=8)[-1]
    items, meta = [], []
    for k in range(4):
        for sc, h, p in ((room, h_room, poses_room[k]), (apt, h_apt, poses_apt[k % 2])):
            for sn in (s_only, s_all, s_rgbd):
                o = ctx.alloc(sn, 1, tri=True)
                items.append((h, sn, p, o.get("rgb"), o.get("depth"), o["tri"], o.get("semantic")))
                meta.append((sc, sn, p, o))
        o = ctx.alloc(s_rgbd, 1, tri=True)
        items.append((h_plain, s_rgbd, poses_room[k], o["rgb"], o["depth"], o["tri"], None))
        meta.append((room, s_rgbd, poses_room[k], o))
    ctx.render_batch(items)
    torch.cuda.synchronize()
    jobs = []
    for k, (sc, sn, p, o) in enumerate(meta):
        g = {key: v[0] for key, v in to_np(o).items()}
        if "semantic" in g:
            miss = g["tri"] == NONE
            assert (g["semantic"][miss] == NONE).all()
            assert (g["semantic"][~miss] == sc.instances[g["tri"][~miss]]).all()
        jobs.append((sc, sn, p, g, None, f"mixed {k}"))
    assert oracle_compare_many(jobs) == len(jobs)
    # the RGB+D views are unchanged by the semantic views beside them
    ref_items, refs = [], []
    for (h, sn, p, *_), (sc, _, _, o) in zip(items, meta):
        if sn is s_rgbd:
            r = ctx.alloc(sn, 1, tri=True)
            ref_items.append((h, sn, p, r["rgb"], r["depth"], r["tri"]))
            refs.append((o, r))
    ctx.render_batch(ref_items)
    torch.cuda.synchronize()
    for o, r in refs:
        for key in ("rgb", "depth", "tri"):
            assert torch.equal(o[key], r[key]), key
    for h in (h_room, h_apt, h_plain):
        ctx.release(h)


def test_stepper_and_server_semantic(ctx):
    """The captured stepper and the server write the same masks as an eager
    batch."""
    import torch
    import paper_1904_01201_amd as P
    note("semantic: stepper and server")
    w = configs.room_2k_128()
    h = ctx.upload_scene(w.scenes[0])
    sn = _sem_sensor(ctx, 128, 128)
    outs = [ctx.alloc(sn, 1, tri=True) for _ in range(4)]
    items = [(h, sn, w.poses[k, 0], o["rgb"], o["depth"], o["tri"], o["semantic"])
             for k, o in enumerate(outs)]
    st = ctx.stepper(items)
    for step in range(3):
        poses = w.poses[4 * step + 1: 4 * step + 5, 0]
        st.step(poses)
        torch.cuda.synchronize()
        got = [o["semantic"].clone() for o in outs]
        ref = _render_batch_np(ctx, h, sn, poses)
        for a, b in zip(got, ref):
            assert np.array_equal(a.cpu().numpy().view(np.uint32)[0], b["semantic"]), step
    st.close()
    srv = P.Server(ctx, num_streams=2, max_batch=16)
    poses = w.poses[:40, 0]
    res = [ctx.alloc(sn, 1) for _ in poses]
    tickets = [srv.submit(h, sn, p, r["rgb"], r["depth"], None, r["semantic"])
               for p, r in zip(poses, res)]
    for t in tickets:
        srv.wait(t)
    srv.close()
    ref = _render_batch_np(ctx, h, sn, poses)
    for r, b in zip(res, ref):
        assert np.array_equal(r["semantic"].cpu().numpy().view(np.uint32)[0], b["semantic"])
    ctx.release(h)


def test_batch64_full_size_semantic(ctx):
    """The 64-environment benchmark batch (4 apartments of 100k-1M
    triangles, 256^2) with the semantic attachment added, in its timed
    launch form (one hab_render_batch, default options): two sampled steps
    against the oracle, every view checked for what holds at any size."""
    import torch
    note("semantic: batch64_4scenes_256 sampled steps")
    w = configs.batch64_4scenes_256(steps=500)
    hs = [ctx.upload_scene(s) for s in w.scenes]
    sn = _sem_sensor(ctx, 256, 256)
    out = ctx.alloc(sn, w.num_envs, tri=True)
    for step in (0, 250):
        note(f"semantic batch64 step {step}")
        items = [(hs[w.env_scene[e]], sn, w.poses[step, e], out["rgb"][e], out["depth"][e],
                  out["tri"][e], out["semantic"][e]) for e in range(w.num_envs)]
        ctx.render_batch(items)
        torch.cuda.synchronize()
        g = to_np(out)
        jobs = []
        for e in range(w.num_envs):
            sc = w.scenes[w.env_scene[e]]
            ge = {k: v[e] for k, v in g.items()}
            check_any_size(ge, sc.num_triangles, f"step {step} env {e}")
            miss = ge["tri"] == NONE
            assert (ge["semantic"][miss] == NONE).all()
            assert (ge["semantic"][~miss] == sc.instances[ge["tri"][~miss]]).all()
            if e % 4 == step // 250:
                jobs.append((sc, sn, w.poses[step, e], ge, None, f"step {step} env {e}"))
        oracle_compare_many(jobs)
    for h in hs:
        ctx.release(h)


def test_semantic_errors(ctx):
    """A semantic request on a scene without an instance table is refused
    before anything runs; so is a table of the wrong length (host side)."""
    import paper_1904_01201_amd as P
    note("semantic: errors")
    room = configs.room_2k_128().scenes[0]
    h = ctx.upload(room.positions, room.colors, room.indices)
    sn = _sem_sensor(ctx, 64, 64)
    o = ctx.alloc(sn, 1, tri=True)
    with pytest.raises(P.HabError) as e:
        ctx.render_batch([(h, sn, configs.room_2k_128().poses[0, 0], o["rgb"], o["depth"],
                           o["tri"], o["semantic"])])
    assert e.value.status == P.HAB_ERR_INVALID_ARG
    with pytest.raises(ValueError):
        ctx.upload(room.positions, room.colors, room.indices, instances=room.instances[:-1])
    assert ctx.get_error() == 0
    ctx.release(h)
