"""Invariants of the oracle that any correct rasteriser with the pinned
fill rule and tie rule must satisfy:

* watertightness: a tessellated surface that fills the view covers every
  pixel exactly once (shared edges and shared vertices go to exactly one
  triangle), also when the tessellation is clipped at the near plane;
* order independence: permuting the triangles permutes the ids and leaves
  depth and colour unchanged;
* a render equals the per-pixel merge (largest 1/w, then smallest key) of
  the single-triangle renders.
"""
import numpy as np
import pytest
from scipy.spatial import Delaunay

from tests.geom import IDENT_POSE, pose_at

NONE = 0xFFFFFFFF


def wall_tessellation(rng, n_random, z=-2.0, extent=3.0, centre_px=None, W=64):
    """Delaunay triangulation of random points on the plane z (camera looks
    -Z from the origin) plus the corners of a square of half-size ``extent``
    (which covers the view for 90 degrees at |z| = 2).  Optionally one point
    projects exactly onto a pixel centre and a line of points runs through a
    row of pixel centres."""
    f = W / 2.0
    pts = [(-extent, -extent), (extent, -extent), (extent, extent), (-extent, extent)]
    pts += [tuple(p) for p in rng.uniform(-extent, extent, size=(n_random, 2))]
    if centre_px is not None:
        i, j = centre_px
        w = -z
        pts.append(((i + 0.5 - W / 2) * w / f, -(j + 0.5 - W / 2) * w / f))
        # points on the row through pixel centres of row j
        for i2 in range(0, W, 7):
            pts.append(((i2 + 0.5 - W / 2) * w / f, -(j + 0.5 - W / 2) * w / f))
    pts = np.array(pts, np.float64)
    tri = Delaunay(pts).simplices.astype(np.uint32)
    pos = np.concatenate([pts, np.full((len(pts), 1), z)], axis=1)
    pos = pos[:, [0, 1, 2]].astype(np.float32)
    return pos, tri


@pytest.mark.parametrize("seed", range(6))
def test_watertight_wall(oracle_lib, seed):
    rng = np.random.default_rng(seed)
    pos, tri = wall_tessellation(rng, 40 + 30 * seed, centre_px=(17 + seed, 23 + seed))
    cnt, st = oracle_lib.coverage_count(pos, tri, 64, 64, IDENT_POSE)
    assert cnt.min() == 1 and cnt.max() == 1, (np.unique(cnt, return_counts=True))


@pytest.mark.parametrize("seed", range(4))
def test_watertight_near_clipped_floor(oracle_lib, seed):
    """A Delaunay-tessellated floor y = 0 around and behind the camera (at
    height 1.5, pitched down 30 degrees): many triangles straddle the near
    plane.  Every pixel whose ray meets the floor inside the tessellated
    square is covered exactly once; no pixel is covered twice."""
    rng = np.random.default_rng(100 + seed)
    xz = np.concatenate([[[-30, -30], [30, -30], [30, 30], [-30, 30]],
                         rng.uniform(-6, 6, size=(150, 2)),
                         rng.uniform(-0.3, 0.3, size=(20, 2))])
    tri = Delaunay(xz).simplices.astype(np.uint32)
    pos = np.stack([xz[:, 0], np.zeros(len(xz)), xz[:, 1]], axis=1).astype(np.float32)
    a = np.deg2rad(-30.0)        # pitch down: rotate about +X
    R = [[1, 0, 0], [0, np.cos(a), -np.sin(a)], [0, np.sin(a), np.cos(a)]]
    pose = pose_at(0.1, 1.5, 0.2, R)
    cnt, st = oracle_lib.coverage_count(pos, tri, 64, 64, pose)
    assert st["clipped"] > 0
    assert cnt.max() == 1
    # the lower part of the image sees the floor close by: all covered
    assert (cnt[40:] == 1).all()


def test_permutation_invariance(oracle_lib):
    from scenegen import configs
    w = configs.room_2k_128()
    sc = w.scenes[0]
    rng = np.random.default_rng(5)
    perm = rng.permutation(sc.num_triangles)
    inv = np.argsort(perm)
    for k in (0, 1, 2, 7):
        pose = w.poses[k, 0]
        a = oracle_lib.render_view(sc.positions, sc.colors, sc.indices, 96, 64, pose)
        b = oracle_lib.render_view(sc.positions, sc.colors, sc.indices[perm], 96, 64, pose)
        assert np.array_equal(a["depth"], b["depth"])
        assert np.array_equal(a["rgb"], b["rgb"])
        mapped = np.where(b["tri"] == NONE, NONE, perm[np.minimum(b["tri"], len(perm) - 1)])
        assert np.array_equal(a["tri"], mapped.astype(np.uint32))
        assert a["stats"] == b["stats"]
    del inv


def test_render_equals_merge_of_single_triangle_renders(oracle_lib):
    """Per-pixel maximum of rho with the smaller key on ties, over renders of
    each triangle on its own, reproduces the full render's raw z-buffer."""
    rng = np.random.default_rng(9)
    n = 24
    ctr = rng.uniform([-1.5, -1.5, -4.0], [1.5, 1.5, -0.5], size=(n, 1, 3))
    pos = (ctr + rng.normal(0, 0.6, size=(n, 3, 3))).reshape(-1, 3).astype(np.float32)
    pos[:6, 2] = rng.uniform(-0.2, 0.3, size=6)          # some cross the near plane
    idx = np.arange(3 * n, dtype=np.uint32).reshape(n, 3)
    col = rng.integers(0, 256, size=(3 * n, 3)).astype(np.uint8)
    full = oracle_lib.render_view(pos, col, idx, 48, 40, IDENT_POSE, raw=True)
    best_rho = np.zeros((40, 48), np.float32)
    best_key = np.full((40, 48), NONE, np.uint32)
    best_rgb = np.zeros((40, 48, 3), np.uint8)
    best_depth = np.zeros((40, 48), np.float32)
    for t in range(n):
        one = oracle_lib.render_view(pos, col, idx[t:t + 1], 48, 40, IDENT_POSE, raw=True)
        key = np.where(one["key"] == NONE, NONE, one["key"] + 2 * t).astype(np.uint32)
        better = (one["rho"] > best_rho) | ((one["rho"] == best_rho) & (key < best_key))
        better &= key != NONE
        best_rho = np.where(better, one["rho"], best_rho)
        best_key = np.where(better, key, best_key)
        best_depth = np.where(better, one["depth"], best_depth)
        best_rgb = np.where(better[..., None], one["rgb"], best_rgb)
    assert np.array_equal(full["rho"], best_rho)
    assert np.array_equal(full["key"], best_key)
    assert np.array_equal(full["depth"], best_depth)
    assert np.array_equal(full["rgb"], best_rgb)
