"""Pins of the oracle's textured shading (perspective-correct texture
coordinates, bilinear fetch at texel centres, repeat wrap).

Expected values come from the geometry: a face-on wall whose texture maps
one texel to one pixel must reproduce the texture; at two pixels per texel
the bilinear weights are 1/4 and 3/4 with a wrap at the border; a receding
floor must show the texel coordinate of the exact ray-plane hit, not the
screen-affine one; integer shifts of the coordinates change nothing.
"""
import numpy as np
import pytest

from tests.geom import pose_at

NONE = 0xFFFFFFFF


def wall_quad(z=-2.0, half=2.0):
    """A face-on square at depth -z spanning [-half, half]^2, vertices
    top-left, top-right, bottom-right, bottom-left."""
    pos = np.array([[-half, half, z], [half, half, z], [half, -half, z], [-half, -half, z]],
                   np.float32)
    idx = np.array([[0, 1, 2], [0, 2, 3]], np.uint32)
    return pos, idx


def rand_tex(rng, th, tw):
    return rng.integers(0, 256, size=(th, tw, 3), dtype=np.uint8)


def test_one_texel_per_pixel_reproduces_the_texture(oracle_lib):
    """64^2 at 90 degrees (f = 32): the wall at depth 2 spanning [-2, 2]^2
    fills the image exactly; uv (0,0) top-left .. (1,1) bottom-right on a
    64^2 texture puts every pixel centre on a texel centre."""
    rng = np.random.default_rng(1)
    tex = rand_tex(rng, 64, 64)
    pos, idx = wall_quad()
    uv = np.array([[0, 0], [1, 0], [1, 1], [0, 1]], np.float32)
    r = oracle_lib.render_view(pos, None, idx, 64, 64, pose_at(0, 0, 0), uvs=uv, texture=tex)
    assert (r["tri"] != NONE).all()
    assert np.array_equal(r["rgb"], tex)


def test_two_pixels_per_texel_bilinear_weights_and_wrap(oracle_lib):
    """A 32^2 texture on the same wall: pixel i samples x = i/2 - 1/4, so
    even pixels blend texels (i/2 - 1, i/2) with weights (1/4, 3/4) and odd
    pixels (k, k + 1) with (3/4, 1/4); pixel 0 wraps to texel 31."""
    rng = np.random.default_rng(2)
    tex = rand_tex(rng, 32, 32).astype(np.float64)
    pos, idx = wall_quad()
    uv = np.array([[0, 0], [1, 0], [1, 1], [0, 1]], np.float32)
    r = oracle_lib.render_view(pos, None, idx, 64, 64, pose_at(0, 0, 0), uvs=uv,
                               texture=tex.astype(np.uint8))
    k = np.arange(64)
    lo = np.where(k % 2 == 0, k // 2 - 1, k // 2) % 32
    hi = (lo + 1) % 32
    wlo = np.where(k % 2 == 0, 0.25, 0.75)
    rows = tex[lo] * wlo[:, None, None] + tex[hi] * (1 - wlo)[:, None, None]       # blend in y
    full = rows[:, lo] * wlo[None, :, None] + rows[:, hi] * (1 - wlo)[None, :, None]
    assert np.array_equal(r["rgb"], np.clip(np.rint(full), 0, 255).astype(np.uint8))


def test_integer_shift_of_coordinates_changes_nothing(oracle_lib):
    """Repeat wrap: uv + (2, -3) (negative coordinates included) give the
    same image on an oblique view, up to the fp32 rounding of the larger
    interpolated coordinates (a colour step of 1 in rare pixels)."""
    rng = np.random.default_rng(3)
    tex = rand_tex(rng, 16, 64)
    pos, idx = wall_quad(-3.0, 3.0)
    uv = np.array([[0.1, 0.2], [1.7, 0.1], [1.9, 1.3], [0.0, 1.1]], np.float32)
    R = [[0.9, 0.0, 0.43588989], [0.0, 1.0, 0.0], [-0.43588989, 0.0, 0.9]]
    pose = pose_at(0.4, 0.2, 0.5, R)
    a = oracle_lib.render_view(pos, None, idx, 80, 60, pose, uvs=uv, texture=tex)
    b = oracle_lib.render_view(pos, None, idx, 80, 60, pose, uvs=uv + np.float32([2, -3]),
                               texture=tex)
    hit = a["tri"] != NONE
    assert hit.sum() > 1000
    d = np.abs(a["rgb"].astype(int) - b["rgb"].astype(int))
    assert d.max() <= 1 and (d.max(axis=-1)[hit] == 0).mean() > 0.99


def smooth_tex(tw, th):
    """Texture whose red channel is a linear ramp in u (0.5 .. 254.5 over
    one period) and green in v: bilinear sampling reproduces the ramp
    exactly away from the wrap."""
    x = (np.arange(tw) + 0.5) / tw
    y = (np.arange(th) + 0.5) / th
    t = np.zeros((th, tw, 3), np.uint8)
    t[..., 0] = np.rint(x * 254)[None, :]
    t[..., 1] = np.rint(y * 254)[:, None]
    t[..., 2] = 90
    return t


@pytest.mark.parametrize("near_clip", [False, True])
def test_receding_floor_is_perspective_correct(oracle_lib, near_clip):
    """A floor y = 0 seen from 1.5 m, pitched down 30 degrees; u = x/8 +
    1/2, v = (z + 8)/16 over x in [-4, 4], z in [-8, 0] (or z up to +2
    behind the camera, so the floor straddles the near plane).  Every
    covered pixel's red/green must match the ramp at the exact ray-floor
    hit within 2 (the texels' own rounding and the snap); a screen-affine
    interpolation misses by tens."""
    tw = th = 256
    tex = smooth_tex(tw, th)
    z1 = 2.0 if near_clip else 0.0
    pos = np.array([[-4, 0, -8], [4, 0, -8], [4, 0, z1], [-4, 0, z1]], np.float32)
    idx = np.array([[0, 1, 2], [0, 2, 3]], np.uint32)
    uv = np.array([[x / 8 + 0.5, (z + 8) / 16 * (8 / (8 + z1))] for x, _, z in pos], np.float32)
    c, s = np.cos(np.radians(30)), np.sin(np.radians(30))
    R = np.array([[1, 0, 0], [0, c, s], [0, -s, c]])      # pitch down: camera -Z -> (0, -s, -c)
    W = H = 96
    r = oracle_lib.render_view(pos, None, idx, W, H, pose_at(0, 1.5, 0, R), uvs=uv, texture=tex)
    f = oracle_lib.focal(W, 90.0)
    jj, ii = np.mgrid[0:H, 0:W]
    d_cam = np.stack([(ii + 0.5 - W / 2) / f, -(jj + 0.5 - H / 2) / f, -np.ones_like(ii, float)], -1)
    d_w = d_cam @ R.T
    t = -1.5 / d_w[..., 1]
    X, Z = t * d_w[..., 0], t * d_w[..., 2]
    u_exact = X / 8 + 0.5
    v_exact = (Z + 8) / 16 * (8 / (8 + z1))
    hit = r["tri"] != NONE
    inner = hit & (np.abs(X) < 3.9) & (Z > -7.9) & (Z < z1 - 0.1)
    assert inner.sum() > 2000
    red = np.clip(u_exact * 254, 0, 254)
    green = np.clip(v_exact * 254, 0, 254)
    assert np.abs(r["rgb"][..., 0][inner] - red[inner]).max() <= 2.0
    assert np.abs(r["rgb"][..., 1][inner] - green[inner]).max() <= 2.0
    assert (r["rgb"][..., 2][hit] == 90).all()


def test_texture_argument_errors(oracle_lib):
    pos, idx = wall_quad()
    uv = np.array([[0, 0], [1, 0], [1, 1], [0, 1]], np.float32)
    with pytest.raises(Exception):
        oracle_lib.render_view(pos, None, idx, 16, 16, pose_at(0, 0, 0), uvs=uv,
                               texture=np.zeros((24, 32, 3), np.uint8))      # not a power of two
    with pytest.raises(Exception):
        oracle_lib.render_view(pos, None, idx, 16, 16, pose_at(0, 0, 0), uvs=uv * 5000,
                               texture=np.zeros((1024, 1024, 3), np.uint8))  # |u| tw >= 2^22
