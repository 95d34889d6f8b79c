"""Helpers for the GPU parity tests: context fixture and comparison with the
oracle (visible triangle bit-exact, depth within 1e-5 relative, colour
within 1 of 255)."""
import os
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

NONE = 0xFFFFFFFF
DEPTH_RTOL = 1e-5
RGB_ATOL = 1


def note(msg):
    """Name the case on stderr before a GPU step (survives a lost box)."""
    print(f"[gpu] {msg}", file=sys.stderr, flush=True)


def gpu_ctx():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1904_01201_amd as P
    return P.Context(0)


def to_np(out):
    res = {}
    for k in ("rgb", "depth", "tri", "semantic"):
        if k in out and out[k] is not None:
            a = out[k].cpu().numpy()
            if k in ("tri", "semantic"):
                a = a.view(np.uint32)
            res[k] = a
    return res


def compare(g, o, what=""):
    """g: numpy outputs of one GPU view; o: oracle dict.  Asserts parity and
    returns the number of depth values that are not bit-identical."""
    if "tri" in g:
        bad = g["tri"] != o["tri"]
        assert not bad.any(), f"{what}: {int(bad.sum())} triangle ids differ, first at {np.argwhere(bad)[:3].tolist()}"
    if "semantic" in g:
        bad = g["semantic"] != o["semantic"]
        assert not bad.any(), f"{what}: {int(bad.sum())} instance ids differ, first at {np.argwhere(bad)[:3].tolist()}"
    if "depth" in g:
        od = o["depth"].astype(np.float64)
        gd = g["depth"].astype(np.float64)
        hit = o["tri"] != NONE
        assert (gd[~hit] == 0).all(), f"{what}: depth written where nothing is visible"
        rel = np.abs(gd[hit] - od[hit]) / np.maximum(od[hit], 1e-30)
        assert rel.size == 0 or rel.max() <= DEPTH_RTOL, f"{what}: depth rel err {rel.max()}"
    if "rgb" in g:
        d = np.abs(g["rgb"].astype(np.int32) - o["rgb"].astype(np.int32))
        assert d.max(initial=0) <= RGB_ATOL, f"{what}: colour diff {d.max()}"
    if "depth" in g:
        return int((g["depth"].view(np.uint32) != o["depth"].view(np.uint32)).sum())
    return 0


def compare_noisy_depth(gd, o, sigma, what=""):
    """Noisy depth parity.  The GPU evaluates the Box-Muller deviate in
    fp32 (logf, sqrtf, cospif: a few ulp each, |n| <= 5.8) and the oracle in
    fp64 from the same 24-bit uniforms, so the inverse depths differ by at
    most ~3e-6 sigma + 2e-7 rho; the bar is 1e-5 (rho + sigma) on
    1/depth.  Where the oracle's noisy inverse depth lies within that band
    of 0 the GPU may read either side (a return or none); elsewhere the
    validity must agree.  Returns the number of band pixels."""
    hit = o["tri"] != NONE
    rho = o["rho"].astype(np.float64)
    rp = o["rho_noisy"]
    tol = 1e-5 * (rho + sigma)
    gd = gd.astype(np.float64)
    assert (gd[~hit] == 0).all(), f"{what}: noisy depth where nothing is visible"
    sure_pos = hit & (rp > tol)
    sure_neg = hit & (rp < -tol)
    assert (gd[sure_pos] > 0).all(), f"{what}: {int((gd[sure_pos] <= 0).sum())} returns lost"
    assert (gd[sure_neg] == 0).all(), f"{what}: {int((gd[sure_neg] != 0).sum())} spurious returns"
    err = np.abs(1.0 / gd[sure_pos] - rp[sure_pos])
    assert err.size == 0 or (err <= tol[sure_pos]).all(), \
        f"{what}: inverse depth error {(err / tol[sure_pos]).max():.3g} x the bar"
    return int((hit & ~sure_pos & ~sure_neg).sum())


def check_any_size(out, T, what):
    """Properties of one view's outputs that need no oracle: ids in range,
    nothing written where nothing is visible, positive finite depth."""
    tri = out["tri"]
    miss = tri == NONE
    assert (tri[~miss] < T).all(), f"{what}: triangle id out of range"
    if "depth" in out:
        d = out["depth"]
        assert (d[miss] == 0).all(), f"{what}: depth where nothing is visible"
        assert np.isfinite(d[~miss]).all() and (d[~miss] > 0).all(), f"{what}: bad depth"
    if "rgb" in out:
        assert (out["rgb"][miss] == 0).all(), f"{what}: colour where nothing is visible"


def oracle_compare_many(jobs, threads=None):
    """jobs: (scene, sensor, pose, gpu_outputs, gpu_stats or None, label).
    Renders each view with the oracle on a thread pool (the C oracle runs
    without the GIL) and asserts parity; returns the number of views."""
    import oracle

    def one(job):
        sc, sn, pose, g, st, what = job
        tex = getattr(sc, "texture", None)
        o = oracle.render_view(sc.positions, sc.colors, sc.indices, sn.width, sn.height, pose,
                               hfov_deg=sn.hfov_deg, near_m=sn.near_m,
                               instances=sc.instances if "semantic" in g else None,
                               uvs=None if tex is None else sc.uvs, texture=tex)
        compare(g, o, what)
        if st is not None:
            for k in ("survivors", "bbox_tests", "covered"):
                assert st[k] == o["stats"][k], (what, k, st[k], o["stats"][k])
        return 1

    n = threads or max(1, min(16, os.cpu_count() or 1))
    with ThreadPoolExecutor(max_workers=n) as ex:
        return sum(ex.map(one, jobs))
