"""Seeded synthetic indoor scenes: rooms, apartments, furniture boxes.

These stand in for the scanned Matterport3D / Gibson / Replica scenes the
paper evaluates on (Sec. 4 "Episode dataset preparation"; Table 1 uses one
Matterport3D scene), which are not available here.  The generator keeps the
shape of that workload: indoor rooms with floor, ceiling, walls and furniture,
measured in metres with +Y up, dense surface tessellation, and optional
scan-like vertex noise.

This module holds no rendering arithmetic.  It only produces meshes
(float32 positions, uint8 vertex colours, uint32 triangle indices) and the 2D
obstacle layout that the walk generator uses.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

ROOM_HEIGHT = 2.8
DOOR_WIDTH = 0.9
DOOR_HEIGHT = 2.1


@dataclass
class Rect:
    """Axis-aligned rectangle: ``axis`` fixed at ``value``; the other two axes
    span [u_lo, u_hi] x [v_lo, v_hi].  Corners are given as coordinate ranges so
    that faces meeting at an edge reproduce the same float values there."""
    axis: int
    value: float
    ua: int
    u_lo: float
    u_hi: float
    va: int
    v_lo: float
    v_hi: float
    nu: int = 0          # explicit subdivision (0 = derive from the cell edge)
    nv: int = 0


@dataclass
class Scene:
    positions: np.ndarray          # float32 [V, 3], metres, +Y up
    colors: np.ndarray             # uint8 [V, 3]
    indices: np.ndarray            # uint32 [T, 3]
    walls: np.ndarray              # float64 [Nw, 4] solid wall segments (x0, z0, x1, z1)
    boxes: np.ndarray              # float64 [Nb, 4] box footprints (xmin, zmin, xmax, zmax)
    bounds: np.ndarray             # float64 [4] floor extent (xmin, zmin, xmax, zmax)
    free_discs: np.ndarray         # float64 [Nr, 3] (cx, cz, r) kept free of boxes
    name: str = ""
    meta: dict = field(default_factory=dict)
    # uint32 [T] object instance per triangle: one per structural surface
    # (floor, ceiling, wall piece), one per furniture box (its five faces)
    instances: np.ndarray | None = None
    # float32 [V, 2] texture coordinates: each surface maps the texture
    # planarly at TEXEL_PER_M texels per metre of a TEX_SIZE^2 texture,
    # from a random offset; the texture itself ([TEX_SIZE, TEX_SIZE, 3]
    # uint8) is attached by with_texture()
    uvs: np.ndarray | None = None
    texture: np.ndarray | None = None

    @property
    def num_triangles(self) -> int:
        return int(self.indices.shape[0])

    @property
    def num_vertices(self) -> int:
        return int(self.positions.shape[0])


def _counts(rects, cell):
    """Per-rect (nu, nv) for a uniform cell edge ``cell`` (explicit counts win)."""
    nu = np.empty(len(rects), np.int64)
    nv = np.empty(len(rects), np.int64)
    for k, r in enumerate(rects):
        if r.nu > 0:
            nu[k], nv[k] = r.nu, r.nv
        else:
            nu[k] = max(1, int(round((r.u_hi - r.u_lo) / cell)))
            nv[k] = max(1, int(round((r.v_hi - r.v_lo) / cell)))
    return nu, nv


def _axis_coords(lo, hi, n):
    t = np.arange(n + 1, dtype=np.float64) / n
    c = lo + (hi - lo) * t
    c[0] = lo
    c[-1] = hi
    return c


TEX_SIZE = 2048
TEXEL_PER_M = 256.0


def _tessellate(rects, cell, rng_colors, rng_uv=None):
    """Grid-tessellate every rect.  Each quad (i,j)-(i+1,j+1) is split along
    its (i,j)->(i+1,j+1) diagonal.  Returns float64 positions, uint8 colours,
    uint32 indices and float32 texture coordinates (from ``rng_uv``'s
    per-rect offsets; None without it)."""
    nu, nv = _counts(rects, cell)
    pos_parts, col_parts, idx_parts, uv_parts = [], [], [], []
    rep = TEXEL_PER_M / TEX_SIZE          # texture periods per metre
    base = 0
    for k, r in enumerate(rects):
        a, b = int(nu[k]), int(nv[k])
        cu = _axis_coords(r.u_lo, r.u_hi, a)
        cv = _axis_coords(r.v_lo, r.v_hi, b)
        U, Vv = np.meshgrid(cu, cv, indexing="ij")          # [a+1, b+1]
        p = np.empty((a + 1, b + 1, 3), np.float64)
        p[..., r.axis] = r.value
        p[..., r.ua] = U
        p[..., r.va] = Vv
        p = p.reshape(-1, 3)
        vid = np.arange((a + 1) * (b + 1), dtype=np.int64).reshape(a + 1, b + 1) + base
        v00 = vid[:-1, :-1].ravel()
        v10 = vid[1:, :-1].ravel()
        v11 = vid[1:, 1:].ravel()
        v01 = vid[:-1, 1:].ravel()
        t0 = np.stack([v00, v10, v11], axis=1)
        t1 = np.stack([v00, v11, v01], axis=1)
        tri = np.stack([t0, t1], axis=1).reshape(-1, 3)
        basecol = rng_colors.integers(32, 225, size=3)
        jit = rng_colors.integers(-31, 32, size=(p.shape[0], 3))
        col = np.clip(basecol[None, :] + jit, 0, 255).astype(np.uint8)
        pos_parts.append(p)
        col_parts.append(col)
        idx_parts.append(tri)
        if rng_uv is not None:
            off = rng_uv.random(2)
            uv = np.stack([off[0] + (U - r.u_lo) * rep, off[1] + (Vv - r.v_lo) * rep], axis=-1)
            uv_parts.append(uv.reshape(-1, 2))
        base += p.shape[0]
    pos = np.concatenate(pos_parts, axis=0)
    col = np.concatenate(col_parts, axis=0)
    idx = np.concatenate(idx_parts, axis=0).astype(np.uint32)
    uvs = np.concatenate(uv_parts, axis=0).astype(np.float32) if uv_parts else None
    return pos, col, idx, uvs


def triangle_count(rects, cell) -> int:
    nu, nv = _counts(rects, cell)
    return int(2 * np.sum(nu * nv))


def cell_for_target(rects, target_T, tol=0.02):
    """Bisect the uniform cell edge so that the triangle count is within
    ``tol`` of ``target_T`` (closest achievable otherwise)."""
    area = sum((r.u_hi - r.u_lo) * (r.v_hi - r.v_lo) for r in rects)
    lo, hi = 1e-4, 10.0
    best = (None, None)
    guess = float(np.sqrt(2.0 * area / max(target_T, 1)))
    lo, hi = guess / 8.0, guess * 8.0
    for _ in range(80):
        mid = float(np.sqrt(lo * hi))
        T = triangle_count(rects, mid)
        if best[0] is None or abs(T - target_T) < abs(best[1] - target_T):
            best = (mid, T)
        if abs(T - target_T) <= tol * target_T:
            return mid
        if T > target_T:
            lo = mid
        else:
            hi = mid
    return best[0]


def _box_rects(x0, x1, y0, y1, z0, z1, n=0):
    """Five faces of a box (the bottom face is coplanar with the floor and is
    omitted)."""
    return [
        Rect(1, y1, 0, x0, x1, 2, z0, z1, n, n),        # top
        Rect(0, x0, 2, z0, z1, 1, y0, y1, n, n),        # -x side
        Rect(0, x1, 2, z0, z1, 1, y0, y1, n, n),        # +x side
        Rect(2, z0, 0, x0, x1, 1, y0, y1, n, n),        # -z side
        Rect(2, z1, 0, x0, x1, 1, y0, y1, n, n),        # +z side
    ]


def _instances(rects, cell, num_boxes):
    """Instance id per triangle.  The rects end with the five faces of each
    box in placement order; every rect before them is a structural surface
    with an id of its own, and a box's faces share one id."""
    nu, nv = _counts(rects, cell)
    nstruct = len(rects) - 5 * num_boxes
    k = np.arange(len(rects), dtype=np.int64)
    rect_inst = np.where(k < nstruct, k, nstruct + (k - nstruct) // 5)
    return np.repeat(rect_inst, 2 * nu * nv).astype(np.uint32)


def _finish(rects, cell, seed, walls, boxes, bounds, discs, name, meta):
    rng_c = np.random.Generator(np.random.PCG64([seed, 7]))
    rng_uv = np.random.Generator(np.random.PCG64([seed, 11]))
    pos, col, idx, uvs = _tessellate(rects, cell, rng_c, rng_uv)
    return Scene(pos.astype(np.float32), col, idx,
                 np.asarray(walls, np.float64).reshape(-1, 4),
                 np.asarray(boxes, np.float64).reshape(-1, 4),
                 np.asarray(bounds, np.float64),
                 np.asarray(discs, np.float64).reshape(-1, 3), name, meta,
                 _instances(rects, cell, len(boxes)), uvs)


def make_texture(seed: int, size: int = TEX_SIZE) -> np.ndarray:
    """A seeded [size, size, 3] uint8 texture that tiles seamlessly: value
    noise at periods of size/4 .. size/64 texels (bilinear upsampling of
    periodic random grids) in three tinted channels, plus per-texel grain
    of +-12, like a scanned surface's albedo."""
    rng = np.random.Generator(np.random.PCG64([seed, 13]))
    acc = np.zeros((size, size, 3), np.float64)
    amp = 1.0
    for cells in (4, 8, 16, 32, 64):
        g = rng.random((cells, cells, 3))
        t = (np.arange(size) + 0.5) * cells / size - 0.5
        i0 = np.floor(t).astype(np.int64)
        f = t - i0
        a, b = i0 % cells, (i0 + 1) % cells
        rows = g[a] * (1 - f)[:, None, None] + g[b] * f[:, None, None]
        acc += amp * (rows[:, a] * (1 - f)[None, :, None] + rows[:, b] * f[None, :, None])
        amp *= 0.55
    acc /= sum(0.55 ** k for k in range(5))
    tint = rng.uniform(0.6, 1.0, size=3)
    val = 32 + 190 * acc * tint + rng.integers(-12, 13, size=(size, size, 3))
    return np.clip(np.rint(val), 0, 255).astype(np.uint8)


def with_texture(scene: Scene, seed: int | None = None, size: int = TEX_SIZE) -> Scene:
    """The scene with a texture attached (its uvs already map it); the
    default seed is a CRC of the scene's name."""
    import zlib
    from dataclasses import replace
    s = seed if seed is not None else zlib.crc32(scene.name.encode())
    return replace(scene, texture=make_texture(s, size))


def make_room(seed: int, num_boxes: int = 20) -> Scene:
    """One room, Lx ~ U[5,8] x Lz ~ U[4,7] x 2.8 m, six surfaces as 10x10
    grids (1,200 triangles) and ``num_boxes`` furniture boxes, each face a 2x2
    grid (40 triangles per box).  With 20 boxes: T = 2,000, V = 1,626."""
    rng = np.random.Generator(np.random.PCG64([seed, 1]))
    Lx = float(rng.uniform(5.0, 8.0))
    Lz = float(rng.uniform(4.0, 7.0))
    H = ROOM_HEIGHT
    rects = [
        Rect(1, 0.0, 0, 0.0, Lx, 2, 0.0, Lz, 10, 10),   # floor
        Rect(1, H, 0, 0.0, Lx, 2, 0.0, Lz, 10, 10),     # ceiling
        Rect(0, 0.0, 2, 0.0, Lz, 1, 0.0, H, 10, 10),
        Rect(0, Lx, 2, 0.0, Lz, 1, 0.0, H, 10, 10),
        Rect(2, 0.0, 0, 0.0, Lx, 1, 0.0, H, 10, 10),
        Rect(2, Lz, 0, 0.0, Lx, 1, 0.0, H, 10, 10),
    ]
    boxes = []
    for _ in range(num_boxes):
        sx = float(rng.uniform(0.3, 1.5))
        sy = float(rng.uniform(0.3, 2.0))
        sz = float(rng.uniform(0.3, 1.5))
        x0 = float(rng.uniform(0.0, Lx - sx))
        z0 = float(rng.uniform(0.0, Lz - sz))
        x1, z1 = x0 + sx, z0 + sz
        rects += _box_rects(x0, x1, 0.0, sy, z0, z1, n=2)
        boxes.append((x0, z0, x1, z1))
    walls = [(0, 0, Lx, 0), (Lx, 0, Lx, Lz), (Lx, Lz, 0, Lz), (0, Lz, 0, 0)]
    return _finish(rects, 1.0, seed, walls, boxes, (0.0, 0.0, Lx, Lz),
                   np.zeros((0, 3)), f"room{seed}", {"Lx": Lx, "Lz": Lz})


def _door_split(lo, hi, rng):
    d0 = float(rng.uniform(lo + 0.3, hi - 0.3 - DOOR_WIDTH))
    return d0, d0 + DOOR_WIDTH


def make_apartment(seed: int, target_T: int, boxes_per_room: int = 50,
                   jitter_sigma: float = 0.0) -> Scene:
    """A 2 x 4 grid of box rooms (column widths and row depths ~ U[3.5,5.5] m,
    height 2.8 m).  Every interior wall has a 0.9 x 2.1 m doorway at a random
    offset (three rectangles).  ``boxes_per_room`` boxes of size U[0.2,1.2]^3
    stand on each floor, kept out of a free disc at the room centre and out of
    the doorway clearances.  All surfaces use one uniform grid cell edge,
    bisected so that the triangle count is within 2% of ``target_T``."""
    rng = np.random.Generator(np.random.PCG64([seed, 2]))
    H = ROOM_HEIGHT
    cw = rng.uniform(3.5, 5.5, size=2)
    rd = rng.uniform(3.5, 5.5, size=4)
    xs = np.concatenate([[0.0], np.cumsum(cw)])
    zs = np.concatenate([[0.0], np.cumsum(rd)])
    X, Z = float(xs[-1]), float(zs[-1])
    rects: list[Rect] = []
    walls = []
    doors = []      # (x0, z0, x1, z1) clearance rectangles
    discs = []
    for c in range(2):
        for r in range(4):
            x0, x1, z0, z1 = float(xs[c]), float(xs[c + 1]), float(zs[r]), float(zs[r + 1])
            rects.append(Rect(1, 0.0, 0, x0, x1, 2, z0, z1))
            rects.append(Rect(1, H, 0, x0, x1, 2, z0, z1))
            discs.append((0.5 * (x0 + x1), 0.5 * (z0 + z1), 0.8))
    # exterior walls, split per room
    for r in range(4):
        z0, z1 = float(zs[r]), float(zs[r + 1])
        for xw in (0.0, X):
            rects.append(Rect(0, xw, 2, z0, z1, 1, 0.0, H))
            walls.append((xw, z0, xw, z1))
    for c in range(2):
        x0, x1 = float(xs[c]), float(xs[c + 1])
        for zw in (0.0, Z):
            rects.append(Rect(2, zw, 0, x0, x1, 1, 0.0, H))
            walls.append((x0, zw, x1, zw))
    # interior wall between the two columns (one segment per row)
    xw = float(xs[1])
    for r in range(4):
        z0, z1 = float(zs[r]), float(zs[r + 1])
        d0, d1 = _door_split(z0, z1, rng)
        rects.append(Rect(0, xw, 2, z0, d0, 1, 0.0, H))
        rects.append(Rect(0, xw, 2, d1, z1, 1, 0.0, H))
        rects.append(Rect(0, xw, 2, d0, d1, 1, DOOR_HEIGHT, H))
        walls += [(xw, z0, xw, d0), (xw, d1, xw, z1)]
        doors.append((xw - 0.8, d0, xw + 0.8, d1))
    # interior walls between rows (one segment per column)
    for r in range(1, 4):
        zw = float(zs[r])
        for c in range(2):
            x0, x1 = float(xs[c]), float(xs[c + 1])
            d0, d1 = _door_split(x0, x1, rng)
            rects.append(Rect(2, zw, 0, x0, d0, 1, 0.0, H))
            rects.append(Rect(2, zw, 0, d1, x1, 1, 0.0, H))
            rects.append(Rect(2, zw, 0, d0, d1, 1, DOOR_HEIGHT, H))
            walls += [(x0, zw, d0, zw), (d1, zw, x1, zw)]
            doors.append((d0, zw - 0.8, d1, zw + 0.8))
    # furniture boxes
    boxes = []
    for c in range(2):
        for r in range(4):
            rx0, rx1, rz0, rz1 = float(xs[c]), float(xs[c + 1]), float(zs[r]), float(zs[r + 1])
            cx, cz = 0.5 * (rx0 + rx1), 0.5 * (rz0 + rz1)
            placed = 0
            tries = 0
            while placed < boxes_per_room and tries < 200 * boxes_per_room:
                tries += 1
                sx, sy, sz = (float(v) for v in rng.uniform(0.2, 1.2, size=3))
                bx0 = float(rng.uniform(rx0 + 0.05, rx1 - 0.05 - sx))
                bz0 = float(rng.uniform(rz0 + 0.05, rz1 - 0.05 - sz))
                bx1, bz1 = bx0 + sx, bz0 + sz
                # keep the room-centre disc free (closest footprint point)
                qx = min(max(cx, bx0), bx1)
                qz = min(max(cz, bz0), bz1)
                if (qx - cx) ** 2 + (qz - cz) ** 2 < (0.8 + 0.3) ** 2:
                    continue
                if any(bx0 < d[2] and bx1 > d[0] and bz0 < d[3] and bz1 > d[1] for d in doors):
                    continue
                rects += _box_rects(bx0, bx1, 0.0, min(sy, 2.0), bz0, bz1)
                boxes.append((bx0, bz0, bx1, bz1))
                placed += 1
    cell = cell_for_target(rects, target_T)
    sc = _finish(rects, cell, seed, walls, boxes, (0.0, 0.0, X, Z), discs,
                 f"apt{seed}_{target_T}", {"cell": cell, "xs": xs.tolist(), "zs": zs.tolist()})
    if jitter_sigma > 0.0:
        sc.positions = jitter_positions(sc.positions, seed, jitter_sigma)
    return sc


# ---------------------------------------------------------------------------
# scan-like vertex noise, keyed by position so that duplicated vertices move
# together and no cracks open between faces
# ---------------------------------------------------------------------------
_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def _splitmix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser (Steele, Lea, Flood 2014), vectorised, wrapping."""
    with np.errstate(over="ignore"):
        z = x + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def jitter_positions(pos: np.ndarray, seed: int, sigma: float) -> np.ndarray:
    """Displace each vertex by N(0, sigma^2) per axis, drawn from a hash of
    (seed, position quantised to 10 um)."""
    q = np.round(pos.astype(np.float64) * 1e5).astype(np.int64).view(np.uint64)
    with np.errstate(over="ignore"):
        h = _splitmix64(np.uint64(seed) * np.uint64(0xD1B54A32D192ED03) + q[:, 0])
        h = _splitmix64(h ^ q[:, 1])
        h = _splitmix64(h ^ q[:, 2])
        u = []
        for _ in range(4):
            h = _splitmix64(h)
            u.append(((h >> np.uint64(11)).astype(np.float64) + 0.5) / float(1 << 53))
    r1 = np.sqrt(-2.0 * np.log(u[0]))
    r2 = np.sqrt(-2.0 * np.log(u[2]))
    n0 = r1 * np.cos(2 * np.pi * u[1])
    n1 = r1 * np.sin(2 * np.pi * u[1])
    n2 = r2 * np.cos(2 * np.pi * u[3])
    d = np.stack([n0, n1, n2], axis=1) * sigma
    return (pos.astype(np.float64) + d).astype(np.float32)


def aabb(scene: Scene) -> np.ndarray:
    """(min xyz, max xyz) of the vertex positions, float64 [2, 3]."""
    p = scene.positions.astype(np.float64)
    return np.stack([p.min(axis=0), p.max(axis=0)])
