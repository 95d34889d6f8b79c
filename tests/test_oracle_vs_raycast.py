"""The oracle against an independent FP64 brute-force ray caster on random
tiny scenes (at most 64 triangles, at most 48x48 pixels), including
triangles that cross the near plane.

The oracle snaps vertices to 1/256 px, so it may legitimately disagree with
exact geometry only
  (a) at pixel centres within the snapping band of an edge of either
      candidate triangle: delta = sqrt(2)/512 px plus the fp32 projection
      error, bounded by 2^-19 (|projected coordinate| + f) px, or
  (b) where the two candidate surfaces are at nearly the same depth (their
      exact depths differ by less than twice the depth bound below).
Everywhere else the visible triangle must be the same.  Where it is, the
depth must agree within |grad(1/d)| delta / (1/d) + 2e-6 relative (the
snapped interpolant of 1/d is a convex combination of values displaced by
at most delta, plus fp32 rounding), and the colour within 1 (rounding) plus
the change of the exact colour over a displacement of delta.
"""
import numpy as np
from hypothesis import given, settings, strategies as st, HealthCheck

from oracle import raycast_fp64 as rc
from tests.geom import pose_at

NONE = 0xFFFFFFFF


def random_scene(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 65))
    ctr = np.stack([rng.uniform(-3, 3, n), rng.uniform(-3, 3, n), rng.uniform(-6, -0.3, n)], 1)
    size = rng.uniform(0.05, 2.0, size=(n, 1, 1))
    pos = ctr[:, None, :] + rng.normal(0, 1, size=(n, 3, 3)) * size
    cross = rng.random(n) < 0.15
    pos[cross, 0, 2] = rng.uniform(-0.2, 0.5, size=cross.sum())       # straddle the near plane
    if n > 2 and rng.random() < 0.5:
        pos[1] = pos[0][[1, 2, 0]]                                     # coplanar duplicate
    pos = pos.reshape(-1, 3).astype(np.float32)
    idx = np.arange(3 * n, dtype=np.uint32).reshape(n, 3)
    col = rng.integers(0, 256, size=(3 * n, 3)).astype(np.uint8)
    W = int(rng.integers(8, 49))
    H = int(rng.integers(8, 49))
    hfov = float(rng.uniform(40, 120))
    yaw, pitch = rng.uniform(-0.3, 0.3), rng.uniform(-0.3, 0.3)
    cy, sy, cp, sp = np.cos(yaw), np.sin(yaw), np.cos(pitch), np.sin(pitch)
    Ry = np.array([[cy, 0, sy], [0, 1, 0], [-sy, 0, cy]])
    Rx = np.array([[1, 0, 0], [0, cp, -sp], [0, sp, cp]])
    pose = pose_at(*rng.uniform(-0.2, 0.2, 3), R=(Ry @ Rx))
    return pos, col, idx, W, H, hfov, pose


@settings(max_examples=60, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(st.integers(0, 2 ** 31 - 1))
def test_oracle_matches_fp64_raycast(oracle_lib, seed):
    pos, col, idx, W, H, hfov, pose = random_scene(seed)
    near = 0.01
    f = oracle_lib.focal(W, hfov)
    o = oracle_lib.render_view(pos, col, idx, W, H, pose, hfov_deg=hfov, near_m=near)
    r = rc.raycast(pos, col, idx, W, H, float(f), pose, near=near)
    ys, xs = np.mgrid[0:H, 0:W]
    px, py = xs + 0.5, ys + 0.5
    T = idx.shape[0]
    polys = [rc.projected_polygon(pos[idx[t]], pose, f, W, H, near) for t in range(T)]

    def delta(t):
        M = max([max(abs(x - W / 2), abs(y - H / 2)) for x, y in polys[t]] + [0.0])
        return np.sqrt(2) / 512 + 2.0 ** -19 * (M + f)

    def near_edge(t, mask):
        if t == NONE or not polys[t]:
            return np.zeros(mask.sum(), bool)
        return rc.dist_to_polygon_edges(px[mask], py[mask], polys[t]) <= delta(t)

    def dbound(t):
        g = rc.inv_depth_gradient(pos[idx[t]], pose, f, W, H)
        return g * delta(t)

    t_all = r["t_all"].reshape(H, W, T)
    ot, rt = o["tri"], r["tri"]
    bad = []
    for t_o in np.unique(ot):
        for t_r in np.unique(rt[ot == t_o]):
            m = (ot == t_o) & (rt == t_r)
            if t_o == t_r:
                continue
            amb = near_edge(t_o, m) | near_edge(t_r, m)
            if t_o != NONE and t_r != NONE:
                d1 = t_all[m][:, t_o]
                d2 = t_all[m][:, t_r]
                rho = 1.0 / np.minimum(d1, d2)
                slack = 2 * (dbound(t_o) + dbound(t_r)) + 4e-6 * rho
                amb |= np.isfinite(d1) & (np.abs(1 / d1 - 1 / d2) <= slack)
            if not amb.all():
                bad.append((int(t_o), int(t_r), int((~amb).sum())))
    assert not bad, bad

    same = (ot == rt) & (ot != NONE)
    for t in np.unique(ot[same]):
        m = same & (ot == t)
        rho_true = 1.0 / r["depth"][m]
        rho_or = 1.0 / o["depth"][m].astype(np.float64)
        assert np.all(np.abs(rho_or - rho_true) <= dbound(t) + 2e-6 * rho_true), t
        # colour, away from edges
        inner = ~near_edge(t, m)
        if not inner.any():
            continue
        dl = delta(t)
        cx, cy = px[m][inner], py[m][inner]
        c0 = rc.colour_at(pos[idx[t]], col[idx[t]], pose, f, W, H, cx, cy)
        var = np.zeros_like(c0)
        for ddx, ddy in ((dl, 0), (-dl, 0), (0, dl), (0, -dl), (dl, dl), (-dl, -dl), (dl, -dl), (-dl, dl)):
            c1 = rc.colour_at(pos[idx[t]], col[idx[t]], pose, f, W, H, cx + ddx, cy + ddy)
            var = np.maximum(var, np.abs(c1 - c0))
        got = o["rgb"][m][inner].astype(np.float64)
        exp = np.clip(r["rgb_f"][m][inner], 0, 255)
        assert np.all(np.abs(got - exp) <= 0.5 + var + 0.5 + 1e-6), t
