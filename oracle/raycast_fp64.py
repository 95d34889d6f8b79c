"""FP64 brute-force ray caster.  TEST INFRASTRUCTURE ONLY.

An independent ground truth for the oracle on tiny scenes (a few dozen
triangles, a few thousand pixels): for every pixel centre, a ray from the
camera through the centre is intersected with every triangle (Moller and
Trumbore 1997, double-sided), and the nearest hit at planar depth >= near
wins (smaller index on an exact tie).  The ray direction in camera space is
(x'/f, -y'/f, -1) with x' = i + 1/2 - W/2 and y' = j + 1/2 - H/2, so the ray
parameter t is the planar depth itself.  It shares no code with the oracle
and never snaps: it sees the exact geometry.

Besides depth, index and perspective-correct colour it returns, per pixel,
what the tests need to decide whether a disagreement with the snapped
rasteriser is legitimate: the screen-space gradient of 1/depth of the hit
triangle and the distance (px) from the pixel centre to the nearest edge of
that triangle's projection (clipped at the near plane).
"""
from __future__ import annotations

import numpy as np

NONE = 0xFFFFFFFF


def camera_rays(W, H, f, pose):
    pose = np.asarray(pose, np.float64)
    p = pose[:3]
    R = pose[3:].reshape(3, 3)
    i = np.arange(W, dtype=np.float64) + 0.5 - W / 2.0
    j = np.arange(H, dtype=np.float64) + 0.5 - H / 2.0
    jj, ii = np.meshgrid(j, i, indexing="ij")
    dc = np.stack([ii / f, -jj / f, -np.ones_like(ii)], axis=-1)      # camera space
    dw = dc @ R.T                                                     # world = R cam
    return p, dw.reshape(-1, 3)


def raycast(positions, colors, indices, W, H, f, pose, near=0.01):
    """Returns dict(depth [H,W], tri [H,W] uint32, rgb_f [H,W,3] float64
    (unrounded), t_all [P,T] (inf where missed))."""
    P = np.asarray(positions, np.float64)
    I = np.asarray(indices, np.int64).reshape(-1, 3)
    Cc = (np.full((P.shape[0], 3), 255.0) if colors is None
          else np.asarray(colors, np.float64).reshape(-1, 3))
    o, d = camera_rays(W, H, f, pose)
    v0, v1, v2 = P[I[:, 0]], P[I[:, 1]], P[I[:, 2]]
    e1 = v1 - v0
    e2 = v2 - v0
    # Moller-Trumbore, vectorised over (pixel, triangle)
    pvec = np.cross(d[:, None, :], e2[None, :, :])
    det = np.einsum("tk,ptk->pt", e1, pvec)
    ok = np.abs(det) > 1e-300
    inv = np.where(ok, 1.0 / np.where(ok, det, 1.0), 0.0)
    tvec = o[None, :] - v0                                           # [T,3]
    u = np.einsum("tk,ptk->pt", tvec, pvec) * inv
    qvec = np.cross(tvec, e1)                                        # [T,3]
    v = np.einsum("pk,tk->pt", d, qvec) * inv
    t = np.einsum("tk,tk->t", e2, qvec)[None, :] * inv
    hit = ok & (u >= 0) & (v >= 0) & (u + v <= 1) & (t >= near)
    tt = np.where(hit, t, np.inf)
    best = np.argmin(tt, axis=1)                                     # first index on ties
    bt = tt[np.arange(tt.shape[0]), best]
    has = np.isfinite(bt)
    depth = np.where(has, bt, 0.0)
    tri = np.where(has, best, NONE).astype(np.uint32)
    bu = u[np.arange(u.shape[0]), best]
    bv = v[np.arange(v.shape[0]), best]
    c0, c1, c2 = Cc[I[best, 0]], Cc[I[best, 1]], Cc[I[best, 2]]
    rgb = ((1 - bu - bv)[:, None] * c0 + bu[:, None] * c1 + bv[:, None] * c2)
    rgb = np.where(has[:, None], rgb, 0.0)
    return {"depth": depth.reshape(H, W), "tri": tri.reshape(H, W),
            "rgb_f": rgb.reshape(H, W, 3), "t_all": tt}


def projected_polygon(tri_world, pose, f, W, H, near):
    """Exact (fp64) screen polygon, in pixels, of a triangle clipped to
    w >= near; empty list if entirely behind."""
    pose = np.asarray(pose, np.float64)
    p = pose[:3]
    R = pose[3:].reshape(3, 3)
    cam = (np.asarray(tri_world, np.float64) - p) @ R          # R^T (P - p)
    pts = [(c[0], c[1], -c[2]) for c in cam]
    poly = []
    for k in range(3):
        a, b = pts[k], pts[(k + 1) % 3]
        ia, ib = a[2] >= near, b[2] >= near
        if ia:
            poly.append(a)
        if ia != ib:
            s, o = (a, b) if ia else (b, a)
            t = (s[2] - near) / (s[2] - o[2])
            poly.append((s[0] + t * (o[0] - s[0]), s[1] + t * (o[1] - s[1]), near))
    return [(W / 2.0 + x * f / w, H / 2.0 - y * f / w) for (x, y, w) in poly]


def dist_to_polygon_edges(px, py, poly):
    """Distance from (px, py) [N] to the edges of a screen polygon."""
    best = np.full(np.shape(px), np.inf)
    n = len(poly)
    for k in range(n):
        ax, ay = poly[k]
        bx, by = poly[(k + 1) % n]
        dx, dy = bx - ax, by - ay
        L2 = dx * dx + dy * dy
        if L2 == 0:
            dd = np.hypot(px - ax, py - ay)
        else:
            t = np.clip(((px - ax) * dx + (py - ay) * dy) / L2, 0.0, 1.0)
            dd = np.hypot(px - (ax + t * dx), py - (ay + t * dy))
        best = np.minimum(best, dd)
    return best


def inv_depth_gradient(tri_world, pose, f, W, H):
    """|grad_screen (1/depth)| (per px) of the plane through a triangle, and
    the plane's 1/depth function.  For a plane n.X = c in camera space and a
    pixel ray (x'/f, -y'/f, -1), 1/depth = (n_x x'/f - n_y y'/f - n_z)/c,
    which is affine in (x', y')."""
    pose = np.asarray(pose, np.float64)
    p = pose[:3]
    R = pose[3:].reshape(3, 3)
    cam = (np.asarray(tri_world, np.float64) - p) @ R
    n = np.cross(cam[1] - cam[0], cam[2] - cam[0])
    c = float(n @ cam[0])
    if c == 0.0:
        return np.inf
    gx = n[0] / (f * c)
    gy = -n[1] / (f * c)
    return float(np.hypot(gx, gy))


def colour_at(tri_world, tri_cols, pose, f, W, H, xs, ys):
    """Perspective-correct colour [N, 3] of the plane through one triangle at
    screen points (xs, ys) in px (no inside test): the ray through the point
    is intersected with the plane and the hit's barycentrics weight the
    vertex colours."""
    pose = np.asarray(pose, np.float64)
    p = pose[:3]
    R = pose[3:].reshape(3, 3)
    xs = np.asarray(xs, np.float64).ravel()
    ys = np.asarray(ys, np.float64).ravel()
    dc = np.stack([(xs - W / 2.0) / f, -(ys - H / 2.0) / f, -np.ones_like(xs)], axis=-1)
    d = dc @ R.T
    v = np.asarray(tri_world, np.float64)
    e1, e2 = v[1] - v[0], v[2] - v[0]
    pvec = np.cross(d, e2)
    det = pvec @ e1
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / det
        tvec = p - v[0]
        u = (pvec @ tvec) * inv
        qvec = np.cross(tvec, e1)
        vv = (d @ qvec) * inv
    c = np.asarray(tri_cols, np.float64)
    return (1 - u - vv)[:, None] * c[0] + u[:, None] * c[1] + vv[:, None] * c[2]
