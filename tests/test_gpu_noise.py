"""Noisy depth sensor on the GPU (the appendix's noise study: iid Gaussian
noise on the inverse depth).

Parity with the oracle uses the derived bar of compare_noisy_depth (1e-5 of
rho + sigma on the inverse depth, validity exact outside that band); colour
and triangle ids stay bit-exact.  Covered: walls, room and apartment views
at the paper's two sigma values and a small one, ragged sizes, the plain
entry point (seed = pose index), the stepper (seed + step), the server, the
normality of the deviates at full resolution, sigma = 0, and the
64-environment benchmark batch.
"""
import numpy as np
import pytest
from scipy import stats

import oracle
from scenegen import configs, make_apartment, random_walks
from tests.geom import pose_at, quad
from tests.gpu_common import NONE, compare, compare_noisy_depth, gpu_ctx, note, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = gpu_ctx()
    yield c
    c.close()


def render_items(ctx, items):
    import torch
    ctx.render_batch(items)
    torch.cuda.synchronize()


def check_view(g, sc, sn, pose, seed, what):
    o = oracle.render_view(sc.positions, sc.colors, sc.indices, sn.width, sn.height, pose,
                           hfov_deg=sn.hfov_deg, near_m=sn.near_m,
                           noise_sigma=float(sn.depth_noise_sigma), noise_seed=seed)
    ideal = {k: v for k, v in g.items() if k != "depth"}
    compare(ideal, o, what)
    return compare_noisy_depth(g["depth"], o, float(sn.depth_noise_sigma), what)


def test_room_views_three_sigmas(ctx):
    note("noise: room views, sigma 0.4 / 0.1 / 0.01")
    w = configs.room_2k_128()
    sc = w.scenes[0]
    h = ctx.upload_scene(sc)
    band = 0
    for sigma in (0.4, 0.1, 0.01):
        sn = ctx.sensor(128, 128, depth_noise_sigma=sigma)
        outs = [ctx.alloc(sn, 1, tri=True) for _ in range(8)]
        seeds = [1000 * k + 7 for k in range(8)]
        items = [(h, sn, w.poses[k, 0], o["rgb"], o["depth"], o["tri"], None, s)
                 for k, (o, s) in enumerate(zip(outs, seeds))]
        render_items(ctx, items)
        for k, o in enumerate(outs):
            g = {key: v[0] for key, v in to_np(o).items()}
            band += check_view(g, sc, sn, w.poses[k, 0], seeds[k], f"sigma {sigma} view {k}")
    note(f"noise: {band} band pixels")
    ctx.release(h)


def test_apartment_ragged_and_plain_entry(ctx):
    """A 100k-triangle apartment at 200 x 136, 75 degrees, depth only,
    through hab_render_ex (seed = pose index)."""
    import paper_1904_01201_amd as P
    note("noise: apartment 200x136 via hab_render_ex")
    apt = make_apartment(seed=21, target_T=100_000, jitter_sigma=0.01)
    h = ctx.upload_scene(apt)
    sn = ctx.sensor(200, 136, 75.0, 0.05, P.OUT_DEPTH, depth_noise_sigma=0.1)
    poses = random_walks(apt, 30, 4, seed=3)[::10].reshape(-1, 12)
    out = ctx.render(h, sn, poses, out=ctx.alloc(sn, len(poses), tri=True))
    import torch
    torch.cuda.synchronize()
    g = to_np(out)
    for k, p in enumerate(poses):
        check_view({key: v[k] for key, v in g.items()}, apt, sn, p, k, f"apartment view {k}")
    ctx.release(h)


def test_sigma_zero_is_ideal(ctx):
    """sigma = 0 and an ideal sensor write the same bits."""
    import torch
    note("noise: sigma 0")
    w = configs.room_2k_128()
    h = ctx.upload_scene(w.scenes[0])
    a = ctx.render(h, ctx.sensor(128, 128, depth_noise_sigma=0.0), w.poses[:4, 0])
    b = ctx.render(h, ctx.sensor(128, 128), w.poses[:4, 0])
    torch.cuda.synchronize()
    assert torch.equal(a["depth"], b["depth"]) and torch.equal(a["rgb"], b["rgb"])
    ctx.release(h)


def test_deviates_normal_at_full_resolution(ctx):
    """A wall at depth 2 (rho = 1/2 exactly) filling a 512 x 512 view with
    sigma = 0.01: the recovered deviates (1/d - 1/2)/sigma are standard
    normal and uncorrelated between neighbours; two seeds differ."""
    import torch
    note("noise: normality at 512^2")
    e = 4.0
    pos, idx = quad([-e, -e, -2], [e, -e, -2], [e, e, -2], [-e, e, -2])
    h = ctx.upload(pos, None, idx)
    sn = ctx.sensor(512, 512, depth_noise_sigma=0.01)
    outs = [ctx.alloc(sn, 1) for _ in range(2)]
    render_items(ctx, [(h, sn, pose_at(0, 0, 0), o["rgb"], o["depth"], None, None, s)
                       for o, s in zip(outs, (3, 4))])
    n = [((1.0 / o["depth"][0].double() - 0.5) / 0.01).cpu().numpy().ravel() for o in outs]
    assert abs(n[0].mean()) < 0.01 and abs(n[0].std() - 1.0) < 0.01
    assert stats.kstest(n[0][::7], "norm").pvalue > 1e-3
    assert abs(np.corrcoef(n[0][:-1], n[0][1:])[0, 1]) < 0.01
    assert abs(np.corrcoef(n[0], n[1])[0, 1]) < 0.01
    # spot check a few pixels against the oracle's deviate
    for p in (0, 1, 511, 512 * 300 + 17, 512 * 512 - 1):
        assert n[0][p] == pytest.approx(oracle.depth_noise_normal(3, p), abs=1e-3)
    ctx.release(h)


def test_stepper_advances_seed_and_server(ctx):
    """Stepper step s renders with seed + s (equal to an eager batch with
    those seeds); the server takes the seed per request."""
    import torch
    import paper_1904_01201_amd as P
    note("noise: stepper and server")
    w = configs.room_2k_128()
    h = ctx.upload_scene(w.scenes[0])
    sn = ctx.sensor(128, 128, depth_noise_sigma=0.1)
    outs = [ctx.alloc(sn, 1) for _ in range(4)]
    base = [11, 22, 33, 44]
    st = ctx.stepper([(h, sn, w.poses[k, 0], o["rgb"], o["depth"], None, None, base[k])
                      for k, o in enumerate(outs)])
    for step in range(3):
        poses = w.poses[4 * step: 4 * step + 4, 0]
        st.step(poses)
        torch.cuda.synchronize()
        got = [o["depth"].clone() for o in outs]
        ref = [ctx.alloc(sn, 1) for _ in range(4)]
        render_items(ctx, [(h, sn, poses[k], r["rgb"], r["depth"], None, None, base[k] + step)
                           for k, r in enumerate(ref)])
        for a, r in zip(got, ref):
            assert torch.equal(a, r["depth"]), step
    st.close()
    srv = P.Server(ctx, num_streams=2, max_batch=8)
    res = [ctx.alloc(sn, 1) for _ in range(20)]
    tickets = [srv.submit(h, sn, w.poses[k, 0], r["rgb"], r["depth"], noise_seed=500 + k)
               for k, r in enumerate(res)]
    for t in tickets:
        srv.wait(t)
    srv.close()
    ref = [ctx.alloc(sn, 1) for _ in range(20)]
    render_items(ctx, [(h, sn, w.poses[k, 0], r["rgb"], r["depth"], None, None, 500 + k)
                       for k, r in enumerate(ref)])
    for a, r in zip(res, ref):
        assert torch.equal(a["depth"], r["depth"])
    ctx.release(h)


def test_batch64_full_size_noisy(ctx):
    """The 64-environment benchmark batch (4 apartments of 100k-1M
    triangles, 256^2 RGB+D) with sigma = 0.1, in its timed launch form:
    16 sampled views of two steps against the oracle."""
    note("noise: batch64_4scenes_256 sampled")
    w = configs.batch64_4scenes_256(steps=500)
    hs = [ctx.upload_scene(s) for s in w.scenes]
    sn = ctx.sensor(256, 256, depth_noise_sigma=0.1)
    out = ctx.alloc(sn, w.num_envs, tri=True)
    for step in (0, 300):
        note(f"noise batch64 step {step}")
        items = [(hs[w.env_scene[e]], sn, w.poses[step, e], out["rgb"][e], out["depth"][e],
                  out["tri"][e], None, (step << 8) | e) for e in range(w.num_envs)]
        render_items(ctx, items)
        g = to_np(out)
        for e in range(step // 300, w.num_envs, 8):
            sc = w.scenes[w.env_scene[e]]
            check_view({k: v[e] for k, v in g.items()}, sc, sn, w.poses[step, e],
                       (step << 8) | e, f"step {step} env {e}")
    for h in hs:
        ctx.release(h)
