"""Pins of the oracle's noisy-depth model (the appendix's noise study: iid
Gaussian noise, mean 0, standard deviation sigma, added per pixel to the
inverse depth).

* the counter-based generator equals numpy's Philox4x64-10, an independent
  implementation of the same published definition;
* the per-pixel deviates are standard normal (Kolmogorov-Smirnov), with
  no correlation between neighbouring pixels or between seeds;
* the model's structure: the inverse depth moves by sigma * n exactly, the
  spread in depth grows as depth squared, sigma = 0 is the ideal sensor,
  nothing-visible pixels and non-positive inverse depths give 0.
"""
import numpy as np
import pytest
from scipy import stats

from tests.geom import merge, pose_at, quad

NONE = 0xFFFFFFFF
M64 = (1 << 64) - 1


def numpy_philox_block(counter, key):
    """One Philox4x64-10 block from numpy's generator: numpy advances its
    counter before each block, so start it one below."""
    c = [int(x) for x in counter]
    v = (c[0] | c[1] << 64 | c[2] << 128 | c[3] << 192) - 1
    v &= (1 << 256) - 1
    start = np.array([(v >> (64 * k)) & M64 for k in range(4)], np.uint64)
    bg = np.random.Philox(key=np.array(key, np.uint64), counter=start)
    return bg.random_raw(4)


def test_philox_matches_numpy(oracle_lib):
    rng = np.random.default_rng(0)
    cases = [([0, 0, 0, 0], [0, 0]), ([1, 0, 0, 0], [5, 7]), ([M64, M64, M64, M64], [M64, M64]),
             ([123456, 0, 0, 0], [2 ** 63, 0x6465707468])]
    for _ in range(200):
        cases.append((rng.integers(0, 2 ** 63, size=4, dtype=np.uint64).tolist(),
                      rng.integers(0, 2 ** 63, size=2, dtype=np.uint64).tolist()))
    for ctr, key in cases:
        assert np.array_equal(oracle_lib.philox4x64_10(ctr, key), numpy_philox_block(ctr, key)), (ctr, key)


def test_pixel_deviates_are_standard_normal(oracle_lib):
    n = np.array([oracle_lib.depth_noise_normal(11, p) for p in range(60000)])
    assert abs(n.mean()) < 0.02 and abs(n.std() - 1.0) < 0.02
    assert stats.kstest(n, "norm").pvalue > 1e-3
    lag = np.corrcoef(n[:-1], n[1:])[0, 1]
    other = np.array([oracle_lib.depth_noise_normal(12, p) for p in range(60000)])
    assert abs(lag) < 0.02 and abs(np.corrcoef(n, other)[0, 1]) < 0.02
    # the tails reach as far as 24-bit uniforms allow (|n| <= sqrt(2 ln 2^24))
    assert np.abs(n).max() > 3.5 and np.abs(n).max() <= np.sqrt(2 * np.log(2.0 ** 24)) + 1e-12


def test_deviate_sign_follows_the_angle(oracle_lib):
    """Box-Muller's angle is 2 pi u2, with u2 the top 24 bits of the
    block's second word: a pixel's deviate is positive exactly when u2 lies
    in [0, 1/4) or (3/4, 1).  u2 comes from numpy's generator here, so
    this ties the oracle's deviate to the definition's bits and angle (a
    different angle scale keeps the distribution but breaks this)."""
    seed, tag = 77, 0x6465707468
    checked = 0
    for p in range(4000):
        x = numpy_philox_block([p, 0, 0, 0], [seed, tag])
        k = int(x[1]) >> 40
        if k in (1 << 22, 3 << 22):
            continue
        u2 = k / 2.0 ** 24
        n = oracle_lib.depth_noise_normal(seed, p)
        assert (n > 0) == (u2 < 0.25 or u2 > 0.75), (p, u2, n)
        checked += 1
    assert checked > 3990


def wall(z):
    """A fronto-parallel quad covering the whole 90-degree view at depth -z."""
    e = 2.0 * abs(z)
    return quad([-e, -e, z], [e, -e, z], [e, e, z], [-e, e, z])


def test_inverse_depth_moves_by_sigma_n(oracle_lib):
    """On a wall at depth 2 (rho = 1/2 exactly), every pixel's noisy inverse
    depth is 1/2 + sigma * n(seed, j W + i), its depth the reciprocal."""
    pos, idx = wall(-2.0)
    W, H, sigma, seed = 48, 40, 0.05, 99
    r = oracle_lib.render_view(pos, None, idx, W, H, pose_at(0, 0, 0), noise_sigma=sigma,
                               noise_seed=seed)
    assert (r["tri"] != NONE).all() and (r["rho"] == 0.5).all()
    n = np.array([oracle_lib.depth_noise_normal(seed, p) for p in range(W * H)]).reshape(H, W)
    assert np.array_equal(r["rho_noisy"], 0.5 + sigma * n)
    assert np.array_equal(r["depth_noisy"], 1.0 / (0.5 + sigma * n))


def test_spread_grows_with_depth_squared(oracle_lib):
    """Small sigma: d' = 1/(rho + sigma n) ~ d - sigma n d^2, so the depth
    spread at 4 m is 4 times the spread at 2 m (same deviates, same
    pixels)."""
    W = H = 96
    sigma = 1e-3
    sd = []
    for z in (-2.0, -4.0):
        pos, idx = wall(z)
        r = oracle_lib.render_view(pos, None, idx, W, H, pose_at(0, 0, 0), noise_sigma=sigma,
                                   noise_seed=5)
        sd.append((r["depth_noisy"] - r["depth"]).std())
    assert sd[1] / sd[0] == pytest.approx(4.0, rel=0.01)
    assert sd[0] == pytest.approx(sigma * 4.0, rel=0.02)


def test_sigma_zero_misses_and_negative_inverse_depth(oracle_lib):
    """sigma = 0 gives the ideal depth; pixels with nothing visible stay 0;
    a large sigma drives some inverse depths to <= 0, which read 0."""
    pos, idx = merge(quad([-1, -1, -2], [1, -1, -2], [1, 1, -2], [-1, 1, -2]))[:2]
    r = oracle_lib.render_view(pos, None, idx, 64, 64, pose_at(0, 0, 0), noise_sigma=1e-300,
                               noise_seed=1)
    hit = r["tri"] != NONE
    assert 0 < hit.sum() < 64 * 64
    assert np.array_equal(r["depth_noisy"][hit], 1.0 / r["rho"][hit].astype(np.float64))
    assert (r["depth_noisy"][~hit] == 0).all() and (r["rho_noisy"][~hit] == 0).all()
    r = oracle_lib.render_view(pos, None, idx, 64, 64, pose_at(0, 0, 0), noise_sigma=0.5,
                               noise_seed=1)
    neg = hit & (r["rho_noisy"] <= 0)
    assert neg.sum() > 50
    assert (r["depth_noisy"][neg] == 0).all()
    pos_ = hit & (r["rho_noisy"] > 0)
    assert (r["depth_noisy"][pos_] == 1.0 / r["rho_noisy"][pos_]).all()
