"""Serving form: continuous batching over resident scenes.

Every served result must be bitwise the same as the same view rendered
alone, whatever batch it rode in and whatever else was in flight; memory
admission must keep the in-flight footprint under the budget and still
complete every request."""
import numpy as np
import pytest

from scenegen import configs, make_apartment, random_walks
from tests.gpu_common import gpu_ctx, note

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import paper_1904_01201_amd as P
    ctx = gpu_ctx()
    room = configs.room_2k_128()
    apt = make_apartment(seed=91, target_T=60_000, jitter_sigma=0.01)
    scenes = [ctx.upload_scene(room.scenes[0]), ctx.upload_scene(apt)]
    poses = [room.poses[:, 0], random_walks(apt, 40, 4, seed=9).reshape(-1, 12)]
    sensors = [ctx.sensor(128, 128), ctx.sensor(64, 96, 80.0, 0.02, P.OUT_DEPTH),
               ctx.sensor(96, 96, 90.0, 0.01, P.OUT_RGB), ctx.sensor(32, 32)]
    yield ctx, scenes, poses, sensors
    ctx.close()


def make_requests(ctx, scenes, poses, sensors, n, seed):
    rng = np.random.default_rng(seed)
    reqs = []
    for k in range(n):
        si = int(rng.integers(0, 2))
        pose = poses[si][int(rng.integers(0, len(poses[si])))]
        sn = sensors[int(rng.integers(0, len(sensors)))]
        out = ctx.alloc(sn, 1, tri=True)
        reqs.append((scenes[si], sn, pose, out))
    return reqs


def check_against_alone(ctx, reqs):
    import torch
    torch.cuda.synchronize()
    for k, (scene, sn, pose, out) in enumerate(reqs):
        ref = ctx.render(scene, sn, pose, out=ctx.alloc(sn, 1, tri=True))
        torch.cuda.synchronize()
        for name in out:
            assert torch.equal(out[name], ref[name]), (k, name)


def test_served_results_equal_alone(env):
    import paper_1904_01201_amd as P
    ctx, scenes, poses, sensors = env
    note("server: mixed requests vs alone")
    reqs = make_requests(ctx, scenes, poses, sensors, 300, seed=1)
    srv = P.Server(ctx, num_streams=3, max_batch=32)
    tickets = []
    for k, (scene, sn, pose, out) in enumerate(reqs):
        tickets.append(srv.submit(scene, sn, pose, out.get("rgb"), out.get("depth"), out.get("tri")))
    stats = [srv.wait(t) for t in tickets]
    st = srv.stats()
    srv.close()
    assert st["completed"] == 300 and st["submitted"] == 300
    assert st["batches"] > 1 and st["peak_batch"] <= 32
    assert all(s["done_ns"] >= s["launch_ns"] >= s["submit_ns"] for s in stats)
    assert len({s["batch_id"] for s in stats}) == st["batches"]
    check_against_alone(ctx, reqs)


def test_admission_under_tight_budget(env):
    """A budget that fits only a few requests at a time: everything still
    completes, the in-flight footprint never exceeds the budget, and a
    request that can never fit is refused up front."""
    import paper_1904_01201_amd as P
    ctx, scenes, poses, sensors = env
    note("server: tight budget")
    reqs = make_requests(ctx, scenes, poses, sensors, 60, seed=2)
    budget = 24 << 20
    srv = P.Server(ctx, num_streams=2, max_batch=64, memory_budget=budget)
    tickets = [srv.submit(s, sn, p, o.get("rgb"), o.get("depth"), o.get("tri")) for s, sn, p, o in reqs]
    for t in tickets:
        srv.wait(t)
    st = srv.stats()
    assert st["completed"] == 60
    assert 0 < st["peak_inflight_bytes"] <= budget
    # the budget is the server's whole device scratch, not only a count
    assert st["scratch_bytes"] == budget
    big = ctx.sensor(4096, 4096, 90.0, 1.0)       # near 1 m keeps the pose in range
    out = ctx.alloc(ctx.sensor(4096, 4096, 90.0, 1.0, P.OUT_DEPTH), 1)
    with pytest.raises(P.HabError) as e:
        srv.submit(scenes[1], big, poses[1][0], None, out["depth"], None)
    assert e.value.status == P.HAB_ERR_CAPACITY
    assert st["rejected"] == 0 and srv.stats()["rejected"] == 1
    srv.close()
    check_against_alone(ctx, reqs)


def test_cancel_and_timeout(env):
    """With one stream and one request per batch a burst queues up:
    cancelling queued requests makes their tickets report
    HAB_ERR_CANCELLED, a request already launched cannot be cancelled and
    completes, requests with a 1 us deadline behind the backlog time out;
    everything that completes equals the view rendered alone."""
    import paper_1904_01201_amd as P
    ctx, scenes, poses, sensors = env
    note("server: cancel and timeout")
    reqs = make_requests(ctx, scenes, poses, [sensors[0]], 60, seed=3)
    srv = P.Server(ctx, num_streams=1, max_batch=1)
    tickets = [srv.submit(s, sn, p, o.get("rgb"), o.get("depth"), o.get("tri")) for s, sn, p, o in reqs[:40]]
    cancelled = [t for t in tickets[10::3] if srv.cancel(t)]
    assert len(cancelled) >= 5, len(cancelled)
    timed = [srv.submit(s, sn, p, o.get("rgb"), o.get("depth"), o.get("tri"), timeout_us=1)
             for s, sn, p, o in reqs[40:]]
    done, outcome = [], {}
    for k, t in enumerate(tickets + timed):
        try:
            srv.wait(t)
            outcome[t] = P.HAB_OK
            done.append(reqs[k])
        except P.HabError as e:
            outcome[t] = e.status
    for t in cancelled:
        assert outcome[t] == P.HAB_ERR_CANCELLED, t
    for t in tickets:
        if t not in cancelled:
            assert outcome[t] == P.HAB_OK, t
    expired = [t for t in timed if outcome[t] == P.HAB_ERR_TIMEOUT]
    assert len(expired) >= 10 and all(outcome[t] in (P.HAB_OK, P.HAB_ERR_TIMEOUT) for t in timed)
    with pytest.raises(P.HabError) as e:   # collected: unknown now
        srv.cancel(tickets[0])
    assert e.value.status == P.HAB_ERR_INVALID_ARG
    st = srv.stats()
    assert st["cancelled"] == len(cancelled) and st["expired"] == len(expired)
    assert st["completed"] == len(done)
    srv.close()
    check_against_alone(ctx, done)


def test_ticket_semantics(env):
    import paper_1904_01201_amd as P
    ctx, scenes, poses, sensors = env
    note("server: tickets")
    srv = P.Server(ctx, num_streams=1, max_batch=4)
    o = ctx.alloc(sensors[0], 1)
    t = srv.submit(scenes[0], sensors[0], poses[0][0], o["rgb"], o["depth"])
    s = srv.wait(t)
    assert s["batch_size"] >= 1
    with pytest.raises(P.HabError) as e:      # already collected
        srv.poll(t)
    assert e.value.status == P.HAB_ERR_INVALID_ARG
    with pytest.raises(P.HabError):
        srv.poll(10 ** 9)
    srv.close()


def test_served_full_scale():
    """serve_32scenes at full size: 32 resident apartments (about 20M
    triangles), 512 agents with mixed sensors, four steps; each agent has at
    most one request in flight.  Every result is checked for what holds at
    any size (on the device); 1% of the requests are compared with the
    oracle."""
    import torch
    import paper_1904_01201_amd as P
    from tests.gpu_common import NONE, check_any_size, oracle_compare_many, to_np
    note("server: serve_32scenes full scale")
    w = configs.serve_32scenes(num_agents=512, steps=4)
    ctx = gpu_ctx()
    try:
        hs = [ctx.upload_scene(s) for s in w.scenes]
        sensors = {}
        for s in w.env_sensor:
            if (s.width, s.outputs) not in sensors:
                sensors[(s.width, s.outputs)] = ctx.sensor(s.width, s.height, s.hfov_deg, s.near_m,
                                                           s.outputs)
        srv = P.Server(ctx, num_streams=4, max_batch=256)
        rng = np.random.default_rng(11)
        total = w.num_steps * w.num_envs
        sample = set(rng.choice(total, size=max(1, total // 100), replace=False).tolist())
        jobs = []
        for step in range(w.num_steps):
            note(f"serve full scale: step {step}")
            reqs = []
            for e in range(w.num_envs):
                sn = sensors[(w.env_sensor[e].width, w.env_sensor[e].outputs)]
                out = ctx.alloc(sn, 1, tri=True)
                t = srv.submit(hs[w.env_scene[e]], sn, w.poses[step, e], out.get("rgb"), out.get("depth"),
                               out["tri"])
                reqs.append((e, t, out))
            for e, t, out in reqs:
                srv.wait(t)
            torch.cuda.synchronize()
            for e, t, out in reqs:
                tri = out["tri"].view(torch.int32)
                miss = tri == -1
                assert int(tri[~miss].max().item() if (~miss).any() else 0) < w.scenes[w.env_scene[e]].num_triangles
                if "depth" in out:
                    d = out["depth"]
                    assert not bool((d[miss] != 0).any()), (step, e)
                    assert bool((d[~miss] > 0).all()), (step, e)
                if "rgb" in out:
                    assert not bool((out["rgb"][miss] != 0).any()), (step, e)
                if step * w.num_envs + e in sample:
                    g = {k: v[0] for k, v in to_np(out).items()}
                    sc = w.scenes[w.env_scene[e]]
                    check_any_size(g, sc.num_triangles, f"served step {step} env {e}")
                    jobs.append((sc, w.env_sensor[e], w.poses[step, e], g, None, f"served step {step} env {e}"))
        st = srv.stats()
        srv.close()
        assert st["completed"] == total and st["rejected"] == 0
        assert oracle_compare_many(jobs) == len(sample)
        assert ctx.get_error() == P.HAB_OK
        for h in hs:
            ctx.release(h)
    finally:
        ctx.close()
