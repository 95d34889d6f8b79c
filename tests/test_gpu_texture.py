"""Textured shading on the GPU: perspective-correct texture coordinates,
bilinear fetch, repeat wrap.

Bar: the colour bar (within 1 of 255; the coordinates are the same fp32
sequence on both sides and the fetch position is exact, so only the blend's
fp32 rounding can move a value across a half), ids bit-exact, depth within
1e-5.  Covered: the one-texel-per-pixel wall (the texture itself), room
and apartment views (near-clipped floors included) at ragged sizes,
textured and plain scenes in one batch, the stepper, the 64-environment
benchmark batch with 2048^2 textures, and upload errors.
"""
import numpy as np
import pytest

import oracle
from scenegen import configs, make_apartment, random_walks, with_texture
from tests.geom import pose_at
from tests.gpu_common import NONE, compare, gpu_ctx, note, oracle_compare_many, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = gpu_ctx()
    yield c
    c.close()


def batch(ctx, items):
    import torch
    ctx.render_batch(items)
    torch.cuda.synchronize()


def test_one_texel_per_pixel_wall(ctx):
    note("texture: one texel per pixel")
    rng = np.random.default_rng(1)
    tex = rng.integers(0, 256, size=(64, 64, 3), dtype=np.uint8)
    pos = np.array([[-2, 2, -2], [2, 2, -2], [2, -2, -2], [-2, -2, -2]], np.float32)
    idx = np.array([[0, 1, 2], [0, 2, 3]], np.uint32)
    uv = np.array([[0, 0], [1, 0], [1, 1], [0, 1]], np.float32)
    h = ctx.upload(pos, None, idx, uvs=uv, texture=tex)
    sn = ctx.sensor(64, 64)
    o = ctx.alloc(sn, 1, tri=True)
    batch(ctx, [(h, sn, pose_at(0, 0, 0), o["rgb"], o["depth"], o["tri"])])
    g = {k: v[0] for k, v in to_np(o).items()}
    assert np.array_equal(g["rgb"], tex)
    ctx.release(h)


def test_room_and_apartment_views(ctx):
    """Room views at 128^2 with a 256^2 texture; a 100k-triangle apartment
    walk at 200 x 136 and 75 degrees with its 2048^2 texture (the walk's
    floors and near walls cross the near plane)."""
    note("texture: room + apartment views")
    room = with_texture(configs.room_2k_128().scenes[0], seed=4, size=256)
    apt = with_texture(make_apartment(seed=21, target_T=100_000, jitter_sigma=0.01), seed=5)
    jobs, keep = [], []
    for sc, W, H, hfov, near, poses in (
            (room, 128, 128, 90.0, 0.01, configs.room_2k_128().poses[:12, 0]),
            (apt, 200, 136, 75.0, 0.05, random_walks(apt, 30, 4, seed=3)[::6].reshape(-1, 12))):
        h = ctx.upload_scene(sc)
        sn = ctx.sensor(W, H, hfov, near)
        outs = [ctx.alloc(sn, 1, tri=True) for _ in poses]
        batch(ctx, [(h, sn, p, o["rgb"], o["depth"], o["tri"]) for p, o in zip(poses, outs)])
        for k, (p, o) in enumerate(zip(poses, outs)):
            jobs.append((sc, sn, p, {key: v[0] for key, v in to_np(o).items()}, None,
                         f"{sc.name} view {k}"))
        keep.append(h)
    assert oracle_compare_many(jobs) == len(jobs)
    exact = sum(int((j[3]["rgb"] == oracle.render_view(
        j[0].positions, None, j[0].indices, j[1].width, j[1].height, j[2], j[1].hfov_deg,
        j[1].near_m, uvs=j[0].uvs, texture=j[0].texture)["rgb"]).all()) for j in jobs[:4])
    note(f"texture: {exact} of 4 room views bit-identical in colour")
    for h in keep:
        ctx.release(h)


def test_textured_and_plain_in_one_batch(ctx):
    """The same room uploaded plain and textured, views interleaved in one
    batch with semantic and noisy-depth sensors: every view matches its
    oracle; the plain views equal a batch of plain views alone."""
    import torch
    import paper_1904_01201_amd as P
    note("texture: mixed batch")
    plain = configs.room_2k_128().scenes[0]
    tex = with_texture(plain, seed=9, size=512)
    hp, ht = ctx.upload_scene(plain), ctx.upload_scene(tex)
    s_sem = ctx.sensor(96, 72, 90.0, 0.01, P.OUT_RGB | P.OUT_DEPTH | P.OUT_SEMANTIC)
    poses = configs.room_2k_128().poses[:6, 0]
    items, meta = [], []
    for k, p in enumerate(poses):
        for sc, h in ((plain, hp), (tex, ht)):
            o = ctx.alloc(s_sem, 1, tri=True)
            items.append((h, s_sem, p, o["rgb"], o["depth"], o["tri"], o["semantic"]))
            meta.append((sc, o, p))
    batch(ctx, items)
    jobs = [(sc, s_sem, p, {k: v[0] for k, v in to_np(o).items()}, None, f"mixed {n}")
            for n, (sc, o, p) in enumerate(meta)]
    assert oracle_compare_many(jobs) == len(jobs)
    ref = [ctx.alloc(s_sem, 1, tri=True) for _ in poses]
    batch(ctx, [(hp, s_sem, p, r["rgb"], r["depth"], r["tri"], r["semantic"])
                for p, r in zip(poses, ref)])
    for (sc, o, _), r in zip(meta[0::2], ref):
        for key in ("rgb", "depth", "tri", "semantic"):
            assert torch.equal(o[key], r[key]), key
    ctx.release(hp)
    ctx.release(ht)


def test_stepper_textured(ctx):
    import torch
    note("texture: stepper")
    sc = with_texture(configs.room_2k_128().scenes[0], seed=2, size=256)
    h = ctx.upload_scene(sc)
    sn = ctx.sensor(128, 128)
    w = configs.room_2k_128()
    outs = [ctx.alloc(sn, 1) for _ in range(4)]
    st = ctx.stepper([(h, sn, w.poses[k, 0], o["rgb"], o["depth"], None) for k, o in enumerate(outs)])
    for step in range(3):
        poses = w.poses[4 * step + 2: 4 * step + 6, 0]
        st.step(poses)
        torch.cuda.synchronize()
        got = [o["rgb"].clone() for o in outs]
        ref = [ctx.alloc(sn, 1) for _ in range(4)]
        batch(ctx, [(h, sn, p, r["rgb"], r["depth"], None) for p, r in zip(poses, ref)])
        for a, r in zip(got, ref):
            assert torch.equal(a, r["rgb"]), step
    st.close()
    ctx.release(h)


def test_batch64_full_size_textured(ctx):
    """The 64-environment benchmark batch (4 apartments of 100k-1M
    triangles, 256^2 RGB+D) with 2048^2 textures, in its timed launch form:
    8 sampled views of two steps against the oracle."""
    note("texture: batch64_4scenes_256 sampled")
    w = configs.batch64_4scenes_256(steps=500)
    scenes = [with_texture(s) for s in w.scenes]
    hs = [ctx.upload_scene(s) for s in scenes]
    sn = ctx.sensor(256, 256)
    out = ctx.alloc(sn, w.num_envs, tri=True)
    for step in (0, 400):
        note(f"texture batch64 step {step}")
        batch(ctx, [(hs[w.env_scene[e]], sn, w.poses[step, e], out["rgb"][e], out["depth"][e],
                     out["tri"][e]) for e in range(w.num_envs)])
        g = to_np(out)
        jobs = [(scenes[w.env_scene[e]], sn, w.poses[step, e], {k: v[e] for k, v in g.items()},
                 None, f"step {step} env {e}") for e in range(step // 400, w.num_envs, 8)]
        oracle_compare_many(jobs)
    for h in hs:
        ctx.release(h)


def test_texture_upload_errors(ctx):
    import paper_1904_01201_amd as P
    note("texture: upload errors")
    pos = np.array([[-1, -1, -2], [1, -1, -2], [1, 1, -2]], np.float32)
    idx = np.array([[0, 1, 2]], np.uint32)
    uv = np.zeros((3, 2), np.float32)
    for tex, u in ((np.zeros((24, 32, 3), np.uint8), uv),                   # not a power of two
                   (np.zeros((64, 64, 3), np.uint8), uv + 70000.0),         # |u| tw >= 2^22
                   (np.zeros((64, 64, 3), np.uint8), uv + np.float32(np.nan))):
        with pytest.raises(P.HabError) as e:
            ctx.upload(pos, None, idx, uvs=u, texture=tex)
        assert e.value.status == P.HAB_ERR_INVALID_ARG
    with pytest.raises(ValueError):
        ctx.upload(pos, None, idx, uvs=uv)
    assert ctx.get_error() == 0
