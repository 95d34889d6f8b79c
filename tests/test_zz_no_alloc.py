"""hab_render_noalloc (scratch in the library's static device array) against
hab_render (scratch in a workspace grown with hipMalloc), through the C ABI.

Two calls in a row on the same stream, the second with a smaller input
(fewer poses of a smaller scene and sensor), so the second finds the array
holding the first call's contents; each must equal hab_render bit for bit
(the same kernels and arithmetic: ids, depth and colour are identical) and
the first also matches the oracle.  Inputs beyond the array's limits are
refused with HAB_ERR_CAPACITY before anything is enqueued.
"""
import numpy as np
import pytest

from scenegen import configs
from tests.gpu_common import gpu_ctx, note, to_np

pytestmark = pytest.mark.gpu


def _render_both(ctx, h, sn, poses):
    import torch
    ref = ctx.alloc(sn, len(poses))
    got = ctx.alloc(sn, len(poses))
    # stale values where the allocation-free call must write
    got["rgb"].fill_(7)
    got["depth"].fill_(-1.0)
    ctx.render_plain(h, sn, poses, ref["rgb"], ref["depth"])
    ctx.render_noalloc(h, sn, poses, got["rgb"], got["depth"])
    torch.cuda.synchronize()
    return ref, got


def test_noalloc_matches_hab_render_twice():
    import torch
    import paper_1904_01201_amd as P
    c = gpu_ctx()
    try:
        # first call: 4 views of the 200k-triangle apartment at 256x256
        note("noalloc: apartment_200k_256, 4 views")
        wa = configs.apartment_200k_256(steps=40)
        sa = wa.scenes[0]
        ha = c.upload_scene(sa)
        sn = c.sensor(256, 256)
        pa = wa.poses[0:40:10, 0]
        ref, got = _render_both(c, ha, sn, pa)
        for k in ("rgb", "depth"):
            assert torch.equal(ref[k], got[k]), k
        g = to_np(got)
        # ids are not an output of this entry point: depth and colour are
        # compared with the oracle through the oracle's own visible-triangle map
        import oracle
        for k, pose in enumerate(pa):
            o = oracle.render_view(sa.positions, sa.colors, sa.indices, 256, 256, pose)
            hit = o["tri"] != oracle.NONE
            d = g["depth"][k].astype(np.float64)
            assert (d[~hit] == 0).all(), k
            rel = np.abs(d[hit] - o["depth"][hit]) / o["depth"][hit]
            assert rel.max(initial=0.0) <= 1e-5, k
            assert np.abs(g["rgb"][k].astype(int) - o["rgb"].astype(int)).max() <= 1, k
        # second call, smaller: 2 views of the 2k-triangle room at 128x128
        note("noalloc: room_2k_128, 2 views (after the larger call)")
        wr = configs.room_2k_128()
        hr = c.upload_scene(wr.scenes[0])
        sr = c.sensor(128, 128)
        pr = wr.poses[:2, 0]
        ref2, got2 = _render_both(c, hr, sr, pr)
        for k in ("rgb", "depth"):
            assert torch.equal(ref2[k], got2[k]), k
        # and the larger one again after the smaller
        ref3, got3 = _render_both(c, ha, sn, pa[:3])
        for k in ("rgb", "depth"):
            assert torch.equal(ref3[k], got3[k]), k
        # limits: more than 256 poses, and a launch whose scratch exceeds
        # the array (64 views of the apartment), refused before any work
        import ctypes as C
        from paper_1904_01201_amd import binding as B
        many = np.repeat(pr[:1], 257, axis=0)
        out = c.alloc(sr, 257)
        rc = c.lib.hab_render_noalloc(c.h, C.c_void_p(hr.ptr), C.byref(sr), B.poses_to_c(many), 257,
                                      out["rgb"].data_ptr(), out["depth"].data_ptr(), None)
        assert rc == P.HAB_ERR_CAPACITY, rc
        big = np.repeat(pa[:1], 64, axis=0)
        outb = c.alloc(sn, 64)
        rc = c.lib.hab_render_noalloc(c.h, C.c_void_p(ha.ptr), C.byref(sn), B.poses_to_c(big), 64,
                                      outb["rgb"].data_ptr(), outb["depth"].data_ptr(), None)
        assert rc == P.HAB_ERR_CAPACITY, rc
        torch.cuda.synchronize()
        assert c.get_error() == P.HAB_OK
        c.release(ha)
        c.release(hr)
    finally:
        c.close()
