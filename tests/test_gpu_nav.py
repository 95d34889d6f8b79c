"""Obstacles from the scene's own mesh and free-space queries on the GPU,
against the oracle (Sec. 4 "Agent embodiment and action space", "Collision
dynamics").

Bar: bit-exact.  The cross-section segments (fp64 cuts rounded once to
fp32) equal the oracle's in value and order; the free-space answers equal
the oracle's for every point (the same fp64 point-segment test; the GPU
visits only the grid cells under the disc, the oracle every segment); agents
walking against the mesh-derived obstacles end in states bit-identical to
the oracle's collide-and-slide over the oracle's own cross-sections.
Covered: an unjittered room, jittered apartments (the benchmark's
100k-triangle scene and its 1M-triangle scene at full size), several
heights, points placed within 1e-9 m of the blocking distance, an empty
obstacle set, argument errors.
"""
import math

import numpy as np
import pytest

import oracle
from scenegen import AGENT_RADIUS, FORWARD_M, TURN_DEG, agents_from_states, configs
from scenegen.walks import random_free_states
from tests.gpu_common import gpu_ctx, note

pytestmark = pytest.mark.gpu

C10, S10 = math.cos(math.radians(TURN_DEG)), math.sin(math.radians(TURN_DEG))
HEIGHTS = (0.1, 1.5)


@pytest.fixture(scope="module")
def ctx():
    c = gpu_ctx()
    yield c
    c.close()


@pytest.fixture(scope="module")
def bench_scenes():
    return configs.batch64_4scenes_256(steps=1).scenes


def gpu_free(ctx, nav, pts, r):
    import torch
    p = torch.from_numpy(np.ascontiguousarray(pts, np.float64)).cuda()
    out = ctx.nav_free(nav, p, r)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(bool)


def near_threshold_points(segs, r, n, seed):
    """Points at distance r (+- up to 1e-9 m) from random segment points,
    off either side, plus points around the endpoints."""
    rng = np.random.default_rng(seed)
    k = rng.integers(0, segs.shape[0], n)
    s = segs[k].astype(np.float64)
    t = rng.uniform(-0.2, 1.2, n)
    ax, az, bx, bz = s[:, 0], s[:, 1], s[:, 2], s[:, 3]
    ex, ez = bx - ax, bz - az
    L = np.maximum(np.hypot(ex, ez), 1e-12)
    nx, nz = -ez / L, ex / L
    sign = np.where(rng.random(n) < 0.5, -1.0, 1.0)
    d = r + rng.uniform(-1e-9, 1e-9, n)
    return np.stack([ax + t * ex + sign * d * nx, az + t * ez + sign * d * nz], 1)


def check_scene(ctx, sc, heights, what, n_pts=8_000, seed=0):
    h = ctx.upload_scene(sc)
    nav = ctx.nav_from_scene(h, heights)
    got = ctx.nav_segments(nav)
    want = oracle.nav_slice(sc.positions, sc.indices, heights)
    assert got.shape == want.shape, (what, got.shape, want.shape)
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32)), what
    lo, hi = sc.positions.min(0), sc.positions.max(0)
    rng = np.random.default_rng(seed)
    pts = np.concatenate([
        np.stack([rng.uniform(lo[0] - 0.5, hi[0] + 0.5, n_pts), rng.uniform(lo[2] - 0.5, hi[2] + 0.5, n_pts)], 1),
        near_threshold_points(want, AGENT_RADIUS, n_pts // 2, seed + 1)])
    g = gpu_free(ctx, nav, pts, AGENT_RADIUS)
    o = oracle.nav_free(want, pts, AGENT_RADIUS)
    bad = g != o
    assert not bad.any(), (what, int(bad.sum()), pts[bad][:3].tolist())
    assert 0.02 < (~g).mean() < 0.98, (what, (~g).mean())
    return h, nav, want


def test_room_segments_and_free_space(ctx):
    note("nav: room_2k_128 cross-sections at 0.1 and 1.5 m, free space")
    sc = configs.room_2k_128().scenes[0]
    h, nav, segs = check_scene(ctx, sc, HEIGHTS, "room")
    assert segs.shape[0] > 0
    ctx.nav_release(nav)
    ctx.release(h)


def test_jittered_apartment_many_heights(ctx, bench_scenes):
    note("nav: 100k-triangle jittered apartment, five heights")
    h, nav, segs = check_scene(ctx, bench_scenes[0], (0.05, 0.1, 0.5, 1.0, 1.5), "apartment 100k, 5 heights",
                               seed=3)
    ctx.nav_release(nav)
    ctx.release(h)


def test_full_size_1m_scene(ctx, bench_scenes):
    note("nav: 1M-triangle jittered apartment (full size)")
    h, nav, segs = check_scene(ctx, bench_scenes[3], HEIGHTS, "apartment 1M", n_pts=16_384, seed=5)
    ctx.nav_release(nav)
    ctx.release(h)


def test_walk_against_mesh_obstacles(ctx, bench_scenes):
    """1,024 agents per scene on two jittered apartments (the benchmark's
    100k and 250k scenes, interleaved) for 40 steps: GPU collide-and-slide
    against hab_nav_from_scene's obstacles equals the oracle's against its
    own cross-sections, bit for bit."""
    import torch
    note("nav: 2 x 1024 agents, 40 steps against mesh obstacles")
    scenes = bench_scenes[:2]
    hs = [ctx.upload_scene(s) for s in scenes]
    navs_h = [ctx.nav_from_scene(h, HEIGHTS) for h in hs]
    segs = [oracle.nav_slice(s.positions, s.indices, HEIGHTS) for s in scenes]
    parts, owner = [], []
    for i, s in enumerate(scenes):
        x, z, yaw = random_free_states(s, 1024, seed=40 + i)
        parts.append(agents_from_states(x, z, yaw))
        owner += [i] * 1024
    owner = np.asarray(owner)
    perm = np.random.default_rng(9).permutation(len(owner))
    agents, owner = np.concatenate(parts)[perm], owner[perm]
    navs = [navs_h[i] for i in owner]
    rng = np.random.default_rng(11)
    hits = 0
    for step in range(40):
        acts = rng.choice([1, 1, 2, 3], size=len(agents)).astype(np.uint8)
        ag = torch.from_numpy(np.ascontiguousarray(agents)).cuda()
        act = torch.from_numpy(acts).cuda()
        hit = torch.empty(len(agents), dtype=torch.uint8, device="cuda")
        ctx.actuate(navs, ag, act, hit, None, 1.5, ctx.actuation(AGENT_RADIUS, FORWARD_M, TURN_DEG))
        torch.cuda.synchronize()
        g, gh = ag.cpu().numpy(), hit.cpu().numpy().astype(bool)
        o = np.empty_like(agents)
        oh = np.zeros(len(agents), bool)
        for i, seg in enumerate(segs):
            idx = np.nonzero(owner == i)[0]
            o[idx], oh[idx] = oracle.actuate(seg, agents[idx], acts[idx], AGENT_RADIUS, FORWARD_M, C10, S10)
        bad = ~(g == o).all(axis=1)
        assert not bad.any(), (step, int(bad.sum()))
        assert np.array_equal(gh, oh), step
        hits += int(gh.sum())
        agents = g
    assert hits > 200, hits
    # every agent ends in free space of its scene's mesh obstacles
    for i, nv in enumerate(navs_h):
        idx = np.nonzero(owner == i)[0]
        free = gpu_free(ctx, nv, agents[idx][:, :2], AGENT_RADIUS - 1e-5)
        assert free.all(), (i, int((~free).sum()))
    for nv in navs_h:
        ctx.nav_release(nv)
    for h in hs:
        ctx.release(h)


def test_empty_and_errors(ctx):
    import ctypes as C
    import torch
    import paper_1904_01201_amd as P
    note("nav: empty obstacle set, argument errors")
    # a floor alone: no triangle crosses 0.1 or 1.5 m
    pos = np.array([[0, 0, 0], [4, 0, 0], [4, 0, 4], [0, 0, 4]], np.float32)
    idx = np.array([[0, 1, 2], [0, 2, 3]], np.uint32)
    h = ctx.upload(pos, None, idx)
    nav = ctx.nav_from_scene(h, HEIGHTS)
    assert nav.num_segments == 0 and ctx.nav_segments(nav).shape == (0, 4)
    assert gpu_free(ctx, nav, [[1.0, 1.0], [100.0, -5.0]], 0.1).all()
    lib = ctx.lib
    hs = (C.c_double * 17)(*([0.5] * 17))
    out = C.c_void_p()
    assert lib.hab_nav_from_scene(ctx.h, C.c_void_p(h.ptr), hs, 0, None, C.byref(out)) == P.HAB_ERR_INVALID_ARG
    assert lib.hab_nav_from_scene(ctx.h, C.c_void_p(h.ptr), hs, 17, None, C.byref(out)) == P.HAB_ERR_INVALID_ARG
    bad = (C.c_double * 1)(float("nan"))
    assert lib.hab_nav_from_scene(ctx.h, C.c_void_p(h.ptr), bad, 1, None, C.byref(out)) == P.HAB_ERR_INVALID_ARG
    assert lib.hab_nav_from_scene(ctx.h, None, hs, 1, None, C.byref(out)) == P.HAB_ERR_INVALID_ARG
    p = torch.zeros((4, 2), dtype=torch.float64, device="cuda")
    o = torch.zeros(4, dtype=torch.uint8, device="cuda")
    for r in (0.0, -1.0, float("inf")):
        assert lib.hab_nav_free(ctx.h, C.c_void_p(nav.ptr), p.data_ptr(), 4, r, o.data_ptr(), None) \
            == P.HAB_ERR_INVALID_ARG
    assert lib.hab_nav_free(ctx.h, C.c_void_p(nav.ptr), None, 4, 0.1, o.data_ptr(), None) == P.HAB_ERR_INVALID_ARG
    assert lib.hab_nav_free(ctx.h, C.c_void_p(nav.ptr), None, 0, 0.1, None, None) == P.HAB_OK
    ctx.nav_release(nav)
    ctx.release(h)
