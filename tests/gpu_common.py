"""Helpers for the GPU parity tests: context fixture and comparison with the
oracle (visible triangle bit-exact, depth within 1e-5 relative, colour
within 1 of 255)."""
import sys

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
    for k in ("rgb", "depth", "tri"):
        if k in out and out[k] is not None:
            a = out[k].cpu().numpy()
            if k == "tri":
                a = a.view(np.uint32)
            res[k] = a
    return res


def compare(g, o, what=""):
    """g: numpy outputs of one GPU view; o: oracle dict.  Asserts parity and
    returns the number of depth values that are not bit-identical."""
    if "tri" in g:
        bad = g["tri"] != o["tri"]
        assert not bad.any(), f"{what}: {int(bad.sum())} triangle ids differ, first at {np.argwhere(bad)[:3].tolist()}"
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
