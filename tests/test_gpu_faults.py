"""Allocation failures, forced from the host (hab_test_fail_alloc makes the
library's device and pinned allocations fail as if out of memory from the
n-th on; no kernel is involved).

For every allocation an entry point makes, in turn: the call returns
HAB_ERR_OUT_OF_MEMORY, the same call then succeeds and renders what the
oracle renders, and once the context is shut down the library holds
exactly what it held before the context was created
(hab_test_live_allocations): nothing leaks on any failure path."""
import ctypes as C

import numpy as np
import pytest

import oracle
from scenegen import configs
from tests.gpu_common import note

pytestmark = pytest.mark.gpu


def live(lib):
    n, b = C.c_uint64(), C.c_uint64()
    assert lib.hab_test_live_allocations(C.byref(n), C.byref(b)) == 0
    return n.value, b.value


@pytest.fixture(scope="module")
def room():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return configs.room_2k_128()


def check_render(ctx, h, sc, pose):
    import torch
    sn = ctx.sensor(128, 128)
    out = ctx.render(h, sn, pose[None], out=ctx.alloc(sn, 1, tri=True))
    torch.cuda.synchronize()
    o = oracle.render_view(sc.positions, sc.colors, sc.indices, 128, 128, pose)
    assert np.array_equal(out["tri"].cpu().numpy()[0].view(np.uint32), o["tri"])


def test_every_allocation_can_fail_without_leaking(room):
    import paper_1904_01201_amd as P
    from paper_1904_01201_amd import binding as B
    lib = B.load()
    sc = room.scenes[0]
    pose = room.poses[0, 0]
    base = live(lib)
    counts = {}

    # context creation
    note("faults: hab_init")
    for k in range(40):
        lib.hab_test_fail_alloc(k)
        try:
            ctx = P.Context(0)
        except P.HabError as e:
            assert e.status == P.HAB_ERR_OUT_OF_MEMORY, e.status
            assert live(lib) == base, k
            continue
        finally:
            lib.hab_test_fail_alloc(-1)
        ctx.close()
        assert live(lib) == base
        counts["init"] = k
        break

    # each entry point on a fresh context: fail its k-th allocation, check
    # the error, that nothing it allocated is still held, and that the call
    # then succeeds
    def upload(ctx):
        n_before = live(lib)
        lib.hab_test_fail_alloc(upload.k)
        try:
            h = ctx.upload_scene(sc)
        except P.HabError as e:
            assert e.status == P.HAB_ERR_OUT_OF_MEMORY
            assert live(lib) == n_before
            lib.hab_test_fail_alloc(-1)
            check_render(ctx, ctx.upload_scene(sc), sc, pose)
            return False
        lib.hab_test_fail_alloc(-1)
        check_render(ctx, h, sc, pose)
        return True

    def render(ctx):
        lib.hab_test_fail_alloc(-1)
        h = ctx.upload_scene(sc)
        lib.hab_test_fail_alloc(render.k)
        try:
            check_render(ctx, h, sc, pose)
        except P.HabError as e:
            assert e.status == P.HAB_ERR_OUT_OF_MEMORY
            lib.hab_test_fail_alloc(-1)
            check_render(ctx, h, sc, pose)   # the retry succeeds
            return False
        return True

    def split(ctx):
        # 32 views: two launch sequences, the second with its own workspace
        import torch
        lib.hab_test_fail_alloc(-1)
        h = ctx.upload_scene(sc)
        sn = ctx.sensor(32, 32)
        poses = np.stack([room.poses[k % room.poses.shape[0], 0] for k in range(32)])
        ref = ctx.render(h, sn, poses, out=ctx.alloc(sn, 32, tri=True), one_sequence=True)
        out = ctx.alloc(sn, 32, tri=True)
        torch.cuda.synchronize()
        lib.hab_test_fail_alloc(split.k)
        try:
            ctx.render(h, sn, poses, out=out)
        except P.HabError as e:
            assert e.status == P.HAB_ERR_OUT_OF_MEMORY
            lib.hab_test_fail_alloc(-1)
            ctx.render(h, sn, poses, out=out)   # the retry succeeds
            torch.cuda.synchronize()
            assert torch.equal(out["tri"], ref["tri"])
            return False
        lib.hab_test_fail_alloc(-1)
        torch.cuda.synchronize()
        assert torch.equal(out["tri"], ref["tri"])
        return True

    def nav(ctx):
        lib.hab_test_fail_alloc(-1)
        h = ctx.upload_scene(sc)
        n_before = live(lib)
        lib.hab_test_fail_alloc(nav.k)
        try:
            nv = ctx.nav_from_scene(h)
        except P.HabError as e:
            assert e.status == P.HAB_ERR_OUT_OF_MEMORY
            assert live(lib) == n_before
            lib.hab_test_fail_alloc(-1)
            nv = ctx.nav_from_scene(h)
            assert nv.num_segments > 0
            return False
        assert nv.num_segments > 0
        return True

    def stepper(ctx):
        lib.hab_test_fail_alloc(-1)
        h = ctx.upload_scene(sc)
        sn = ctx.sensor(128, 128)
        out = ctx.alloc(sn, 2)
        items = [(h, sn, room.poses[k, 0], out["rgb"][k], out["depth"][k], None) for k in range(2)]
        n_before = live(lib)
        lib.hab_test_fail_alloc(stepper.k)
        try:
            st = ctx.stepper(items)
        except P.HabError as e:
            assert e.status == P.HAB_ERR_OUT_OF_MEMORY
            assert live(lib) == n_before
            return False
        st.close()
        return True

    def split_stepper(ctx):
        # 32 views: the graph holds two launch sequences, each with its own arena
        lib.hab_test_fail_alloc(-1)
        h = ctx.upload_scene(sc)
        sn = ctx.sensor(32, 32)
        out = ctx.alloc(sn, 32)
        items = [(h, sn, room.poses[k, 0], out["rgb"][k], out["depth"][k], None) for k in range(32)]
        n_before = live(lib)
        lib.hab_test_fail_alloc(split_stepper.k)
        try:
            st = ctx.stepper(items)
        except P.HabError as e:
            assert e.status == P.HAB_ERR_OUT_OF_MEMORY
            assert live(lib) == n_before
            return False
        lib.hab_test_fail_alloc(-1)
        st.step(np.stack([room.poses[k, 0] for k in range(32)]))
        st.close()
        return True

    def server(ctx):
        lib.hab_test_fail_alloc(-1)
        h = ctx.upload_scene(sc)
        n_before = live(lib)
        lib.hab_test_fail_alloc(server.k)
        try:
            srv = P.Server(ctx, num_streams=2, memory_budget=64 << 20)
        except P.HabError as e:
            assert e.status == P.HAB_ERR_OUT_OF_MEMORY
            assert live(lib) == n_before
            return False
        lib.hab_test_fail_alloc(-1)
        sn = ctx.sensor(128, 128)
        o = ctx.alloc(sn, 1)
        srv.wait(srv.submit(h, sn, pose, o["rgb"], o["depth"]))
        assert srv.stats()["scratch_bytes"] == 64 << 20
        srv.close()
        return True

    for name, fn in (("scene upload", upload), ("render", render), ("split render", split),
                     ("nav_from_scene", nav), ("stepper", stepper), ("split stepper", split_stepper),
                     ("server", server)):
        for k in range(40):
            fn.k = k
            note(f"faults: {name}, allocation {k}")
            ctx = P.Context(0)
            try:
                ok = fn(ctx)
            finally:
                lib.hab_test_fail_alloc(-1)
                ctx.close()
            assert live(lib) == base, (name, k)
            if ok:
                counts[name] = k
                break
        else:
            raise AssertionError(name)
    note(f"faults: injected failures per entry point {counts}")
    # every entry point allocates something, so each saw at least one failure
    assert all(v >= 1 for v in counts.values()), counts
