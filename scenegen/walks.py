"""Seeded agent poses: uniform free-space poses and random walks.

Follows the paper's agent model (Sec. 4 "Agent embodiment and action space"
and "Sensory input"): the colour/depth sensor sits 1.5 m above the agent's
base and faces forward; turn actions rotate by 10 degrees and the forward
action moves 0.25 m.  Actions are drawn uniformly from {turn_left, turn_right,
move_forward}, like the paper's Random baseline (Sec. 4 "Baselines").  A
forward move that would bring the 0.1 m-radius agent (0.2 m diameter body)
within reach of a wall or a box footprint is rejected: the agent stays put.
Sliding along obstacles (Sec. 4 "Collision dynamics") is not modelled; the
walk only has to produce realistic camera trajectories.

A pose is 12 float32: camera position p[3] followed by the row-major
world-from-camera rotation R[9] (camera looks along -Z, +Y is up).
"""
from __future__ import annotations

import numpy as np

from .scenes import Scene

SENSOR_HEIGHT = 1.5
TURN_DEG = 10.0
FORWARD_M = 0.25
AGENT_RADIUS = 0.1


def pose_from_yaw(x: float, y: float, z: float, yaw: float) -> np.ndarray:
    """Pose for a level camera at (x, y, z) rotated by ``yaw`` radians about +Y.
    yaw = 0 looks along -Z; increasing yaw turns left."""
    c, s = np.cos(yaw), np.sin(yaw)
    R = np.array([[c, 0.0, s], [0.0, 1.0, 0.0], [-s, 0.0, c]], np.float64)
    return np.concatenate([[x, y, z], R.ravel()]).astype(np.float32)


def poses_from_states(x, z, yaw, y=SENSOR_HEIGHT) -> np.ndarray:
    x = np.asarray(x, np.float64)
    z = np.asarray(z, np.float64)
    yaw = np.asarray(yaw, np.float64)
    c, s = np.cos(yaw), np.sin(yaw)
    zero, one = np.zeros_like(c), np.ones_like(c)
    out = np.stack([x, np.full_like(x, y), z,
                    c, zero, s,
                    zero, one, zero,
                    -s, zero, c], axis=-1)
    return out.astype(np.float32)


def _seg_dist(px, pz, segs):
    """Distance from points [N] to segments [M, 4] -> [N, M]."""
    if segs.shape[0] == 0:
        return np.full((px.shape[0], 0), np.inf)
    ax, az, bx, bz = (segs[:, k][None, :] for k in range(4))
    dx, dz = bx - ax, bz - az
    L2 = np.maximum(dx * dx + dz * dz, 1e-18)
    t = np.clip(((px[:, None] - ax) * dx + (pz[:, None] - az) * dz) / L2, 0.0, 1.0)
    qx = ax + t * dx - px[:, None]
    qz = az + t * dz - pz[:, None]
    return np.sqrt(qx * qx + qz * qz)


def blocked(scene: Scene, px: np.ndarray, pz: np.ndarray, r: float = AGENT_RADIUS) -> np.ndarray:
    """True where a body of radius ``r`` at (px, pz) touches a wall, a box or
    leaves the floor."""
    px = np.asarray(px, np.float64)
    pz = np.asarray(pz, np.float64)
    b = scene.bounds
    out = (px < b[0] + r) | (px > b[2] - r) | (pz < b[1] + r) | (pz > b[3] - r)
    if scene.walls.shape[0]:
        out |= (_seg_dist(px, pz, scene.walls) < r).any(axis=1)
    if scene.boxes.shape[0]:
        bx = scene.boxes
        inside = ((px[:, None] > bx[None, :, 0] - r) & (px[:, None] < bx[None, :, 2] + r) &
                  (pz[:, None] > bx[None, :, 1] - r) & (pz[:, None] < bx[None, :, 3] + r))
        out |= inside.any(axis=1)
    return out


def random_free_states(scene: Scene, n: int, seed: int, margin: float = 0.2):
    """``n`` (x, z, yaw) states uniform over the free floor (rejection
    sampling); yaw ~ U[0, 2 pi)."""
    rng = np.random.Generator(np.random.PCG64([seed, 3]))
    b = scene.bounds
    xs, zs = [], []
    need = n
    for _ in range(10000):
        if need <= 0:
            break
        cx = rng.uniform(b[0] + margin, b[2] - margin, size=4 * need + 16)
        cz = rng.uniform(b[1] + margin, b[3] - margin, size=4 * need + 16)
        ok = ~blocked(scene, cx, cz)
        xs.append(cx[ok][:need])
        zs.append(cz[ok][:need])
        need -= int(min(ok.sum(), need))
    if need > 0:
        raise RuntimeError("could not sample free poses")
    x = np.concatenate(xs)[:n]
    z = np.concatenate(zs)[:n]
    yaw = rng.uniform(0.0, 2.0 * np.pi, size=n)
    return x, z, yaw


def random_poses(scene: Scene, n: int, seed: int) -> np.ndarray:
    """[n, 12] float32 poses uniform over free space at sensor height."""
    x, z, yaw = random_free_states(scene, n, seed)
    return poses_from_states(x, z, yaw)


def random_walks(scene: Scene, num_agents: int, steps: int, seed: int) -> np.ndarray:
    """[steps, num_agents, 12] float32: the pose after each of ``steps``
    uniformly chosen actions, for ``num_agents`` independent agents that start
    at free poses."""
    rng = np.random.Generator(np.random.PCG64([seed, 4]))
    if scene.free_discs.shape[0]:
        # start inside the free disc at a room centre so the walk can roam
        d = scene.free_discs[rng.integers(0, scene.free_discs.shape[0], size=num_agents)]
        rad = 0.6 * d[:, 2] * np.sqrt(rng.uniform(0.0, 1.0, size=num_agents))
        ang = rng.uniform(0.0, 2.0 * np.pi, size=num_agents)
        x = d[:, 0] + rad * np.cos(ang)
        z = d[:, 1] + rad * np.sin(ang)
        yaw = rng.uniform(0.0, 2.0 * np.pi, size=num_agents)
    else:
        x, z, yaw = random_free_states(scene, num_agents, seed + 101)
    turn = np.deg2rad(TURN_DEG)
    out = np.empty((steps, num_agents, 12), np.float32)
    for s in range(steps):
        a = rng.integers(0, 3, size=num_agents)         # 0 forward, 1 left, 2 right
        yaw = yaw + np.where(a == 1, turn, 0.0) - np.where(a == 2, turn, 0.0)
        nx = x - FORWARD_M * np.sin(yaw)
        nz = z - FORWARD_M * np.cos(yaw)
        fwd = a == 0
        if fwd.any():
            ok = ~blocked(scene, nx, nz)
            move = fwd & ok
            x = np.where(move, nx, x)
            z = np.where(move, nz, z)
        out[s] = poses_from_states(x, z, yaw)
    return out


# ---------------------------------------------------------------------------
# inputs of the actuation step: obstacle segments and agent states
# ---------------------------------------------------------------------------
def nav_segments(scene: Scene) -> np.ndarray:
    """float32 [n, 4] obstacle segments (x0, z0, x1, z1) on the floor plane:
    the scene's walls, then the four edges of every box footprint."""
    parts = [np.asarray(scene.walls, np.float64).reshape(-1, 4)]
    if scene.boxes.shape[0]:
        b = scene.boxes
        x0, z0, x1, z1 = b[:, 0], b[:, 1], b[:, 2], b[:, 3]
        edges = np.stack([np.stack([x0, z0, x1, z0], 1), np.stack([x1, z0, x1, z1], 1),
                          np.stack([x1, z1, x0, z1], 1), np.stack([x0, z1, x0, z0], 1)], 1)
        parts.append(edges.reshape(-1, 4))
    return np.concatenate(parts, 0).astype(np.float32)


def agents_from_states(x, z, yaw) -> np.ndarray:
    """float64 [n, 4] agent states (x, z, fx, fz): position and the unit
    forward vector of heading ``yaw`` (yaw 0 looks along -z)."""
    yaw = np.asarray(yaw, np.float64)
    return np.stack([np.asarray(x, np.float64), np.asarray(z, np.float64),
                     -np.sin(yaw), -np.cos(yaw)], axis=1)
