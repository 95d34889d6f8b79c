"""Full-size workloads, in the launch configurations the benchmark times.

The 64-environment batch (4 jittered apartments of 100k-1M triangles,
256x256 RGB+D) is one hab_render_batch call per step; it runs at each tile
size the autotuner may pick (8, 16 and 32 pixels), with the autotuner's own
choice, through the lossless overflow path (a tile capacity of 64 list
entries; a bin capacity of a quarter of the triangle count), and with the
atomic-free lane-owned z-test instead of the default balanced steps.  The
256-environment mixed batch (16 apartments of 50k-1.5M triangles, 128/256/
512 px, depth / RGB / RGB+D sensors) runs through the captured stepper at
the default tile and at 8 and 32 pixels.  One view per environment every
50 steps of the 500-step walks is compared with the oracle (ids
bit-exact, depth within 1e-5 relative, colour within 1/255, work counters
exact); every view is checked for what holds at any size; the stepper's
replay must equal an eager batch bit for bit; the autotuner's choice must
not change a bit.
"""
import numpy as np
import pytest

from scenegen import configs
from tests.gpu_common import check_any_size, gpu_ctx, note, oracle_compare_many, to_np

pytestmark = pytest.mark.gpu

SAMPLE_STEPS = range(0, 500, 50)


@pytest.fixture(scope="module")
def ctx():
    c = gpu_ctx()
    yield c
    c.close()


@pytest.fixture(scope="module")
def batch64(ctx):
    w = configs.batch64_4scenes_256(steps=500)
    hs = [ctx.upload_scene(s) for s in w.scenes]
    yield w, hs
    for h in hs:
        ctx.release(h)


# (label, render options): the default tile, each autotuner candidate, and
# the overflow path at the 8-pixel tile the benchmark's autotune picks (its
# tile lists hold about 100 entries on average, so a cap of 64 sends many
# tiles through the overflow scan; a quarter of T bin entries per view runs
# out of list space for the last tiles of most views)
BATCH64_OPTS = [
    ("default", {}),
    ("tile8", {"tile_size": 8}),
    ("tile32", {"tile_size": 32}),
    ("tile8_cap64", {"tile_size": 8, "tile_cap": 64}),
    ("tile8_bins0.25", {"tile_size": 8, "bin_factor": 0.25}),
    ("autotuned", None),
    # the atomic-free lane-owned z-test (HAB_RENDER_LANE_OWNED_Z)
    ("tile8_lane_owned", {"tile_size": 8, "lane_owned_z": True}),
    ("tile32_lane_owned", {"tile_size": 32, "lane_owned_z": True}),
    ("tile8_cap64_lane_owned", {"tile_size": 8, "tile_cap": 64, "lane_owned_z": True}),
]


@pytest.mark.parametrize("label,opts", BATCH64_OPTS, ids=[o[0] for o in BATCH64_OPTS])
def test_batch64_sampled_steps(ctx, batch64, label, opts):
    import torch
    w, hs = batch64
    note(f"batch64_4scenes_256 [{label}]: hab_render_batch, every 50th step vs oracle")
    sn = ctx.sensor(256, 256)
    if opts is None:
        # the benchmark's own tuning call: step-0 poses, RGB + depth only
        o0 = ctx.alloc(sn, w.num_envs)
        items0 = [(hs[w.env_scene[e]], sn, w.poses[0, e], o0["rgb"][e], o0["depth"][e], None)
                  for e in range(w.num_envs)]
        ts, bf = ctx.autotune(items0)
        assert ts in (8, 16, 32) and bf in (1.0, 2.0, 4.0), (ts, bf)
        note(f"batch64 autotuned: tile {ts}, bin factor {bf}")
        del o0, items0
        opts = {}
    out = ctx.alloc(sn, w.num_envs, tri=True)
    views = 0
    for step in SAMPLE_STEPS:
        note(f"batch64 [{label}] step {step}")
        items = [(hs[w.env_scene[e]], sn, w.poses[step, e], out["rgb"][e], out["depth"][e],
                  out["tri"][e]) for e in range(w.num_envs)]
        stats = ctx.render_batch(items, stats=True, **opts)
        torch.cuda.synchronize()
        g = to_np(out)
        jobs = []
        for e in range(w.num_envs):
            sc = w.scenes[w.env_scene[e]]
            ge = {k: v[e] for k, v in g.items()}
            check_any_size(ge, sc.num_triangles, f"[{label}] step {step} env {e}")
            jobs.append((sc, w.env_sensor[e], w.poses[step, e], ge, stats[e],
                         f"[{label}] step {step} env {e}"))
        views += oracle_compare_many(jobs)
    note(f"batch64 [{label}]: {views} views match the oracle")
    assert ctx.get_error() == 0


@pytest.mark.parametrize("tile_size", [0, 8, 32], ids=["default", "tile8", "tile32"])
def test_mixed256_stepper_sampled_steps(ctx, tile_size):
    import torch
    note(f"batch256_16scenes_mixed [tile {tile_size}]: stepper, every 50th step vs oracle")
    w = configs.batch256_16scenes_mixed(steps=500)
    hs = [ctx.upload_scene(s) for s in w.scenes]
    sensors = {}
    for s in w.env_sensor:
        key = (s.width, s.outputs)
        if key not in sensors:
            sensors[key] = ctx.sensor(s.width, s.height, s.hfov_deg, s.near_m, s.outputs)
    env_sn = [sensors[(s.width, s.outputs)] for s in w.env_sensor]

    def make_items(step):
        outs = [ctx.alloc(env_sn[e], 1, tri=True) for e in range(w.num_envs)]
        items = [(hs[w.env_scene[e]], env_sn[e], w.poses[step, e], outs[e].get("rgb"),
                  outs[e].get("depth"), outs[e]["tri"]) for e in range(w.num_envs)]
        return outs, items

    outs_g, items_g = make_items(0)
    st = ctx.stepper(items_g, tile_size=tile_size)
    views = 0
    for n, step in enumerate(SAMPLE_STEPS):
        note(f"mixed256 step {step}")
        st.step(w.poses[step])
        torch.cuda.synchronize()
        if n == 0:
            outs_e, items_e = make_items(step)
            ctx.render_batch(items_e, tile_size=tile_size)
            torch.cuda.synchronize()
            for e in range(w.num_envs):
                for k in outs_g[e]:
                    assert torch.equal(outs_g[e][k], outs_e[e][k]), (e, k)
            del outs_e, items_e
        g = [{k: v[0] for k, v in to_np(o).items()} for o in outs_g]
        jobs = []
        for e in range(w.num_envs):
            sc = w.scenes[w.env_scene[e]]
            check_any_size(g[e], sc.num_triangles, f"step {step} env {e}")
            jobs.append((sc, w.env_sensor[e], w.poses[step, e], g[e], None, f"step {step} env {e}"))
        views += oracle_compare_many(jobs)
    note(f"mixed256: {views} views match the oracle")
    st.close()
    for h in hs:
        ctx.release(h)


def test_autotune_choice_and_invariance():
    """The autotuner picks a tile size and bin factor from its candidate
    sets, later default calls use them, and the output stays bit-identical
    to a fixed 16-pixel tiling."""
    import torch
    import paper_1904_01201_amd as P
    note("autotune")
    c = gpu_ctx()
    try:
        w = configs.batch64_4scenes_256(steps=2, scene_T=(20_000, 120_000))
        hs = [c.upload_scene(s) for s in w.scenes]
        sn = c.sensor(256, 256)
        ref = c.alloc(sn, w.num_envs, tri=True)
        items = [(hs[w.env_scene[e]], sn, w.poses[1, e], ref["rgb"][e], ref["depth"][e], ref["tri"][e])
                 for e in range(w.num_envs)]
        c.render_batch(items, tile_size=16)
        ts, bf = c.autotune(items)
        assert ts in (8, 16, 32) and bf in (1.0, 2.0, 4.0), (ts, bf)
        got = c.alloc(sn, w.num_envs, tri=True)
        items2 = [(it[0], it[1], it[2], got["rgb"][e], got["depth"][e], got["tri"][e])
                  for e, it in enumerate(items)]
        c.profile(True)
        c.render_batch(items2)
        c.profile(False)
        phases = c.profile_read()
        assert f"raster{ts}" in phases, (ts, sorted(phases))
        torch.cuda.synchronize()
        for k in ref:
            assert torch.equal(ref[k], got[k]), k
        assert c.get_error() == P.HAB_OK
        for h in hs:
            c.release(h)
    finally:
        c.close()


def test_batch64_z_test_forms_and_sequences_bit_identical(ctx, batch64):
    """Every view of the full-size 64-view batch, at 8- and 32-pixel tiles:
    the default (two launch sequences, balanced z-test), one launch
    sequence, and the atomic-free lane-owned z-test write the same bits."""
    import torch
    w, hs = batch64
    sn = ctx.sensor(256, 256)
    for step in (0, 250, 499):
        for ts in (8, 32):
            note(f"batch64 step {step} tile {ts}: z-test forms and launch sequences")
            outs = []
            for opts in ({}, {"one_sequence": True}, {"lane_owned_z": True},
                         {"lane_owned_z": True, "one_sequence": True}):
                o = ctx.alloc(sn, w.num_envs, tri=True)
                items = [(hs[w.env_scene[e]], sn, w.poses[step, e], o["rgb"][e], o["depth"][e], o["tri"][e])
                         for e in range(w.num_envs)]
                ctx.render_batch(items, tile_size=ts, **opts)
                outs.append(o)
            torch.cuda.synchronize()
            for o in outs[1:]:
                for k in ("rgb", "depth", "tri"):
                    assert torch.equal(o[k], outs[0][k]), (step, ts, k)
    assert ctx.get_error() == 0

