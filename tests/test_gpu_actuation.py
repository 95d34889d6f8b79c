"""Batched actuation and collide-and-slide on the GPU, against the oracle.

Bar: agent states (fp64 position and forward vector) and collision flags
bit-identical to the oracle's (the same fp64 operation sequence, IEEE
division and square root on both sides); camera poses equal to the
oracle's camera poses of those states.  Covered: the closed-form cases, a
2,048-agent walk over two apartments with interleaved scenes, the
4 x 1,024-agent walk over the benchmark's four apartments, a scene with no
obstacles, action values above 3, and argument errors.
"""
import math

import numpy as np
import pytest

import oracle
from scenegen import (AGENT_RADIUS, FORWARD_M, TURN_DEG, agents_from_states, configs,
                      make_apartment, nav_segments)
from scenegen.walks import random_free_states
from tests.gpu_common import gpu_ctx, note

pytestmark = pytest.mark.gpu

C10, S10 = math.cos(math.radians(TURN_DEG)), math.sin(math.radians(TURN_DEG))


@pytest.fixture(scope="module")
def ctx():
    c = gpu_ctx()
    yield c
    c.close()


def gpu_step(ctx, navs, agents, actions):
    import torch
    n = agents.shape[0]
    ag = torch.from_numpy(np.ascontiguousarray(agents)).cuda()
    act = torch.from_numpy(np.asarray(actions, np.uint8)).cuda()
    hit = torch.empty(n, dtype=torch.uint8, device="cuda")
    poses = torch.empty((n, 12), dtype=torch.float32, device="cuda")
    ctx.actuate(navs, ag, act, hit, poses, 1.5,
                ctx.actuation(AGENT_RADIUS, FORWARD_M, TURN_DEG))
    torch.cuda.synchronize()
    return ag.cpu().numpy(), hit.cpu().numpy().astype(bool), poses.cpu().numpy()


def test_closed_form_cases(ctx):
    note("actuation: closed forms")
    h = math.sqrt(0.5)
    cases = [([[1.0, -5.0, 1.0, 5.0]], [0.8, 0.3, 1.0, 0.0], 1),
             ([[1.0, -5.0, 1.0, 5.0]], [0.8, 0.0, h, h], 1),
             ([[1.0, -5.0, 1.0, 1.0], [-5.0, 1.0, 1.0, 1.0]], [0.8, 0.8, h, h], 1),
             ([[1.0, 0.0, 1.0, 0.0]], [0.7, 0.05, 1.0, 0.0], 1),
             ([[1.0, 1.0, 1.0, 2.0]], [0.9, 0.95, 1.0, 0.0], 1),
             ([], [0.0, 0.0, 0.6, -0.8], 2), ([], [0.0, 0.0, 0.6, -0.8], 3),
             ([], [0.3, 0.2, 0.6, -0.8], 1), ([], [0.3, 0.2, 0.6, -0.8], 0),
             ([], [0.3, 0.2, 0.6, -0.8], 200)]
    navs, agents, actions, segs = [], [], [], []
    for seg, a, act in cases:
        seg = np.asarray(seg, np.float32).reshape(-1, 4)
        navs.append(ctx.nav_upload(seg))
        agents.append(a)
        actions.append(act)
        segs.append(seg)
    agents = np.asarray(agents, np.float64)
    g, gh, gp = gpu_step(ctx, navs, agents, actions)
    for k, (seg, a, act) in enumerate(cases):
        o, oh = oracle.actuate(segs[k], agents[k:k + 1], [0 if act > 3 else act],   # > 3: stop
                               AGENT_RADIUS, FORWARD_M, C10, S10)
        assert np.array_equal(g[k], o[0]), (k, g[k], o[0])
        assert gh[k] == oh[0], k
    assert np.array_equal(gp, oracle.agent_pose(g, 1.5))
    for nv in navs:
        ctx.nav_release(nv)


def walk(ctx, scenes, n_per, steps, seed):
    navs_h = [ctx.nav_upload(nav_segments(s)) for s in scenes]
    segs = [nav_segments(s) for s in scenes]
    parts, owner = [], []
    for i, s in enumerate(scenes):
        x, z, yaw = random_free_states(s, n_per, seed=seed + i)
        parts.append(agents_from_states(x, z, yaw))
        owner += [i] * n_per
    owner = np.asarray(owner)
    perm = np.random.default_rng(seed).permutation(len(owner))     # interleave the scenes
    agents, owner = np.concatenate(parts)[perm], owner[perm]
    navs = [navs_h[i] for i in owner]
    rng = np.random.default_rng(seed + 50)
    hits = 0
    for step in range(steps):
        actions = rng.choice([1, 1, 2, 3], size=len(agents)).astype(np.uint8)
        g, gh, gp = gpu_step(ctx, navs, agents, actions)
        o, oh = _oracle_by_owner(segs, owner, agents, actions)
        bad = ~(g == o).all(axis=1)
        assert not bad.any(), (step, int(bad.sum()), np.argwhere(bad)[:3].ravel().tolist())
        assert np.array_equal(gh, oh), step
        assert np.array_equal(gp, oracle.agent_pose(g, 1.5)), step
        hits += int(gh.sum())
        agents = g
    for nv in navs_h:
        ctx.nav_release(nv)
    return hits


def _oracle_by_owner(segs, owner, agents, actions):
    out = np.empty_like(agents)
    hit = np.zeros(agents.shape[0], bool)
    for i, seg in enumerate(segs):
        idx = np.nonzero(owner == i)[0]
        o, h = oracle.actuate(seg, agents[idx], actions[idx], AGENT_RADIUS, FORWARD_M, C10, S10)
        out[idx], hit[idx] = o, h
    return out, hit


def test_walk_two_apartments(ctx):
    note("actuation: 2048 agents, 2 apartments, 30 steps")
    scenes = [make_apartment(seed=31, target_T=20_000), make_apartment(seed=32, target_T=20_000)]
    hits = walk(ctx, scenes, 1024, 30, seed=7)
    assert hits > 500


def test_walk_benchmark_apartments(ctx):
    """4 x 1,024 agents in the benchmark's four apartments (about 1,900
    obstacle segments each: more than one LDS chunk), 12 steps."""
    note("actuation: 4096 agents, benchmark apartments")
    w = configs.batch64_4scenes_256(steps=2)
    assert max(nav_segments(s).shape[0] for s in w.scenes) > 1024
    hits = walk(ctx, w.scenes, 1024, 12, seed=11)
    assert hits > 100


def test_argument_errors(ctx):
    import torch
    import paper_1904_01201_amd as P
    note("actuation: errors")
    nav = ctx.nav_upload(np.zeros((0, 4), np.float32))
    ag = torch.zeros((2, 4), dtype=torch.float64, device="cuda")
    act = torch.zeros(2, dtype=torch.uint8, device="cuda")
    with pytest.raises(P.HabError) as e:
        ctx.actuate([nav, nav], ag, act, params=ctx.actuation(radius=0.0))
    assert e.value.status == P.HAB_ERR_INVALID_ARG
    other = gpu_ctx()
    nav2 = other.nav_upload(np.zeros((1, 4), np.float32))
    with pytest.raises(P.HabError) as e:
        ctx.actuate([nav, nav2], ag, act)
    assert e.value.status == P.HAB_ERR_INVALID_ARG
    other.close()
    with pytest.raises(P.HabError):
        ctx.nav_upload(np.array([[0, 0, np.nan, 1]], np.float32))
    with pytest.raises(ValueError):
        ctx.actuate([nav, nav], ag.float(), act)
    ctx.nav_release(nav)
    assert ctx.get_error() == 0


def test_device_resident_env_loop(ctx):
    """Agents step on the GPU and the captured stepper renders from the poses
    they produce, without a host round trip: every step's images equal an
    eager batch rendered from the same poses copied to the host, for 16
    environments over two apartments, host-pose steps interleaved."""
    import torch
    note("actuation: device-resident env loop")
    scenes = [make_apartment(seed=41, target_T=30_000), make_apartment(seed=42, target_T=30_000)]
    hs = [ctx.upload_scene(s) for s in scenes]
    navs_h = [ctx.nav_upload(nav_segments(s)) for s in scenes]
    owner = np.arange(16) % 2
    parts = [agents_from_states(*random_free_states(scenes[i], 8, seed=60 + i)) for i in range(2)]
    agents = np.empty((16, 4))
    for i in range(2):
        agents[owner == i] = parts[i]
    sn = ctx.sensor(128, 96, 90.0, 0.01, depth_noise_sigma=0.05)
    outs = [ctx.alloc(sn, 1, tri=True) for _ in range(16)]
    poses0 = oracle.agent_pose(agents, 1.5)
    items = [(hs[owner[e]], sn, poses0[e], outs[e]["rgb"], outs[e]["depth"], outs[e]["tri"], None, 10 * e)
             for e in range(16)]
    st = ctx.stepper(items)
    navs = ctx.nav_array([navs_h[i] for i in owner])
    ag = torch.from_numpy(agents).cuda()
    poses = torch.empty((16, 12), dtype=torch.float32, device="cuda")
    rng = np.random.default_rng(3)
    for step in range(8):
        act = torch.from_numpy(rng.choice([1, 1, 2, 3], size=16).astype(np.uint8)).cuda()
        ctx.actuate(navs, ag, act, None, poses)
        if step % 3 == 2:
            torch.cuda.synchronize()
            st.step(poses.cpu().numpy())
        else:
            st.step_device(poses)
        torch.cuda.synchronize()
        got = [{k: o[k].clone() for k in o} for o in outs]
        hp = poses.cpu().numpy()
        ref = [ctx.alloc(sn, 1, tri=True) for _ in range(16)]
        ctx.render_batch([(hs[owner[e]], sn, hp[e], ref[e]["rgb"], ref[e]["depth"], ref[e]["tri"], None,
                           10 * e + step) for e in range(16)])
        torch.cuda.synchronize()
        for e in range(16):
            for k in ("rgb", "depth", "tri"):
                assert torch.equal(got[e][k], ref[e][k]), (step, e, k)
    st.close()
    assert ctx.get_error() == 0
    for h in hs:
        ctx.release(h)
    for nv in navs_h:
        ctx.nav_release(nv)
