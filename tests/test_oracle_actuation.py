"""Pins of the oracle's actuation and collide-and-slide step (Sec. 4 "Agent
embodiment and action space", "Collision dynamics").

Closed forms: free moves are exactly step * forward; a head-on move stops
one skin short of contact; a 45-degree move into a wall keeps its whole
along-wall component (the slide); a move into a corner ends at radius
from both walls; a disc meeting a point obstacle off-centre is deflected
around it.  Turns: 36 left turns return the heading, left + right cancel.
Invariants on a generated apartment (checked with independent distance
code): no disc ever ends closer than its radius to an obstacle, no move
exceeds the step, moves without contact are exact.
"""
import math

import numpy as np
import pytest

from scenegen import AGENT_RADIUS, FORWARD_M, TURN_DEG, make_apartment, nav_segments
from scenegen.walks import random_free_states, agents_from_states

SKIN = 1e-6
C10, S10 = math.cos(math.radians(TURN_DEG)), math.sin(math.radians(TURN_DEG))


def act(oracle_lib, seg, agents, actions):
    return oracle_lib.actuate(np.asarray(seg, np.float32).reshape(-1, 4), agents, actions,
                              AGENT_RADIUS, FORWARD_M, C10, S10)


def test_free_move_is_exact(oracle_lib):
    rng = np.random.default_rng(0)
    yaw = rng.uniform(0, 2 * np.pi, 50)
    ag = np.stack([rng.uniform(-3, 3, 50), rng.uniform(-3, 3, 50), -np.sin(yaw), -np.cos(yaw)], 1)
    out, hit = act(oracle_lib, np.zeros((0, 4)), ag, np.ones(50))
    assert not hit.any()
    assert np.array_equal(out[:, 0], ag[:, 0] + FORWARD_M * ag[:, 2])
    assert np.array_equal(out[:, 1], ag[:, 1] + FORWARD_M * ag[:, 3])
    out, hit = act(oracle_lib, np.zeros((0, 4)), ag, np.zeros(50))      # stop
    assert np.array_equal(out, ag) and not hit.any()


def test_head_on_stops_one_skin_short(oracle_lib):
    wall = [[1.0, -5.0, 1.0, 5.0]]
    out, hit = act(oracle_lib, wall, np.array([[0.8, 0.3, 1.0, 0.0]]), [1])
    assert hit[0]
    assert out[0, 0] == pytest.approx(1.0 - AGENT_RADIUS - SKIN, abs=1e-15)
    assert out[0, 1] == 0.3
    out, hit = act(oracle_lib, wall, np.array([[0.5, 0.0, 1.0, 0.0]]), [1])   # short of it
    assert not hit[0] and out[0, 0] == 0.75


def test_slide_keeps_the_along_wall_component(oracle_lib):
    """45 degrees into the wall x = 1 from (0.8, 0): contact at x = 0.9; the
    remaining motion loses its x part, so z advances by the full
    0.25 sin 45 and x ends one skin (times cos 45) short of 0.9."""
    h = math.sqrt(0.5)
    out, hit = act(oracle_lib, [[1.0, -5.0, 1.0, 5.0]], np.array([[0.8, 0.0, h, h]]), [1])
    assert hit[0]
    assert out[0, 1] == pytest.approx(FORWARD_M * h, abs=1e-14)
    assert out[0, 0] == pytest.approx(0.9 - SKIN * h / 1.0, abs=1e-12)


def test_passing_beyond_a_segment_end_is_free(oracle_lib):
    """The wall piece x = 1, z in [1, 2] does not block a move along z = 0
    across its line, nor one that passes its end at more than the radius."""
    piece = [[1.0, 1.0, 1.0, 2.0]]
    out, hit = act(oracle_lib, piece, np.array([[0.9, 0.0, 1.0, 0.0]]), [1])
    assert not hit[0] and out[0, 0] == 0.9 + FORWARD_M
    out, hit = act(oracle_lib, piece, np.array([[0.9, 0.85, 1.0, 0.0]]), [1])   # 0.15 from the end
    assert not hit[0]
    out, hit = act(oracle_lib, piece, np.array([[0.9, 0.95, 1.0, 0.0]]), [1])   # grazes the end
    assert hit[0] and math.hypot(out[0, 0] - 1.0, out[0, 1] - 1.0) >= AGENT_RADIUS


def test_corner_ends_at_radius_from_both_walls(oracle_lib):
    walls = [[1.0, -5.0, 1.0, 1.0], [-5.0, 1.0, 1.0, 1.0]]
    h = math.sqrt(0.5)
    out, hit = act(oracle_lib, walls, np.array([[0.8, 0.8, h, h]]), [1])
    assert hit[0]
    assert 0.9 - 3e-6 < out[0, 0] <= 0.9 and 0.9 - 3e-6 < out[0, 1] <= 0.9


def test_point_obstacle_deflects(oracle_lib):
    """A zero-length segment at (1, 0): head-on the disc stops one skin
    short of radius; 5 cm off-centre it first touches at x = 1 -
    sqrt(r^2 - 0.05^2) and slides around to the +z side."""
    pt = [[1.0, 0.0, 1.0, 0.0]]
    out, hit = act(oracle_lib, pt, np.array([[0.7, 0.0, 1.0, 0.0]]), [1])
    assert hit[0] and out[0, 0] == pytest.approx(0.9 - SKIN, abs=1e-15)
    out, hit = act(oracle_lib, pt, np.array([[0.7, 0.05, 1.0, 0.0]]), [1])
    assert hit[0]
    d = math.hypot(out[0, 0] - 1.0, out[0, 1])
    assert d >= AGENT_RADIUS and out[0, 1] > 0.05
    assert out[0, 0] > 1.0 - math.sqrt(AGENT_RADIUS ** 2 - 0.05 ** 2) - 1e-9   # got past first contact


def test_turns(oracle_lib):
    ag = np.array([[0.0, 0.0, 0.6, -0.8]])
    a = ag.copy()
    for _ in range(36):
        a, _ = act(oracle_lib, [], a, [2])
    assert np.abs(a - ag).max() < 1e-14
    b, _ = act(oracle_lib, [], ag, [2])
    b, _ = act(oracle_lib, [], b, [3])
    assert np.abs(b - ag).max() < 2e-16
    one, _ = act(oracle_lib, [], ag, [2])      # left turn = +10 degrees of yaw
    yaw0 = math.atan2(-ag[0, 2], -ag[0, 3])
    yaw1 = math.atan2(-one[0, 2], -one[0, 3])
    assert (yaw1 - yaw0) % (2 * math.pi) == pytest.approx(math.radians(10), abs=1e-14)


def seg_distance(px, pz, seg):
    """[n] distance from each point to the nearest segment (brute force)."""
    a = seg[None, :, 0:2].astype(np.float64)
    b = seg[None, :, 2:4].astype(np.float64)
    p = np.stack([px, pz], 1)[:, None, :]
    e = b - a
    L2 = (e * e).sum(-1)
    t = np.where(L2 > 0, ((p - a) * e).sum(-1) / np.where(L2 > 0, L2, 1), 0.0)
    t = np.clip(t, 0, 1)
    q = a + t[..., None] * e
    return np.sqrt(((p - q) ** 2).sum(-1)).min(1)


def test_invariants_on_an_apartment(oracle_lib):
    sc = make_apartment(seed=4, target_T=20_000)
    seg = nav_segments(sc)
    x, z, yaw = random_free_states(sc, 400, seed=9)
    ag = agents_from_states(x, z, yaw)
    rng = np.random.default_rng(5)
    collided_total = 0
    for step in range(40):
        actions = rng.choice([1, 1, 2, 3], size=len(ag))
        new, hit = act(oracle_lib, seg, ag, actions)
        fwd = actions == 1
        moved = np.hypot(new[:, 0] - ag[:, 0], new[:, 1] - ag[:, 1])
        assert (moved <= FORWARD_M + 1e-12).all()
        assert (moved[~fwd] == 0).all()
        free = fwd & ~hit
        assert np.array_equal(new[free, 0], ag[free, 0] + FORWARD_M * ag[free, 2])
        d = seg_distance(new[:, 0], new[:, 1], seg)
        assert d.min() >= AGENT_RADIUS - 1e-12, (step, d.min())
        collided_total += int(hit.sum())
        ag = new
    assert collided_total > 200          # the walk meets walls and boxes often


# --------------------------------------------------------------- camera pose of an agent
# Sec. 4 "Sensory input": the sensor sits 1.5 m above the agent's base and
# faces the agent's heading.  The expected values below come from the camera
# convention (the camera looks along its -Z axis, +Y up, +X right) and the
# projection pins of the renderer, not from the pose function itself.
HEIGHT = 1.5


def test_pose_at_yaw_zero_is_the_identity(oracle_lib):
    """Heading (0, -1) is yaw 0, the camera's own -Z: rotation I, position
    (x, height, z)."""
    p = oracle_lib.agent_pose([[0.75, -2.5, 0.0, -1.0]], HEIGHT)[0]
    assert np.array_equal(p[:3], np.float32([0.75, HEIGHT, -2.5]))
    assert np.array_equal(p[3:].reshape(3, 3), np.eye(3, dtype=np.float32))


def test_pose_matches_the_yaw_rotation(oracle_lib):
    """For heading (-sin y, -cos y) the rotation is the yaw rotation about +Y,
    [[cos, 0, sin], [0, 1, 0], [-sin, 0, cos]], within one fp32 rounding."""
    yaw = np.linspace(0.0, 2.0 * np.pi, 73)
    ag = np.stack([np.zeros_like(yaw), np.zeros_like(yaw), -np.sin(yaw), -np.cos(yaw)], 1)
    p = oracle_lib.agent_pose(ag, HEIGHT).astype(np.float64)
    c, s = np.cos(yaw), np.sin(yaw)
    R = np.stack([c, 0 * c, s, 0 * c, 1 + 0 * c, 0 * c, -s, 0 * c, c], 1)
    assert np.abs(p[:, 3:] - R).max() <= 2.0 ** -24
    # orthonormal, right-handed
    Rm = p[:, 3:].reshape(-1, 3, 3)
    assert np.abs(np.einsum("nij,nik->njk", Rm, Rm) - np.eye(3)).max() < 1e-6
    assert np.abs(np.linalg.det(Rm) - 1.0).max() < 1e-6


def test_pose_looks_along_the_heading(oracle_lib):
    """A point 2 m ahead of the agent at sensor height projects to the
    principal point (64, 64) of a 128^2, 90 degree sensor (X = Y = 16384);
    a point 2 m ahead and 0.5 m to the agent's right (heading turned 90
    degrees clockwise seen from above: (-fz, fx)) lands at x = 64 + 64 *
    0.5 / 2 = 80 px; a point 0.5 m higher lands at y = 48 px (rows grow
    downwards).  A transposed rotation or a mirrored right vector moves
    them."""
    rng = np.random.default_rng(7)
    for yaw in rng.uniform(0.0, 2.0 * np.pi, 12):
        fx, fz = -math.sin(yaw), -math.cos(yaw)
        x, z = rng.uniform(-3, 3), rng.uniform(-3, 3)
        pose = oracle_lib.agent_pose([[x, z, fx, fz]], HEIGHT)[0]
        ahead = [x + 2 * fx, HEIGHT, z + 2 * fz]
        X, Y, _ = oracle_lib.project_point(ahead, pose, 128, 128)
        assert abs(X - 16384) <= 2 and abs(Y - 16384) <= 2, (yaw, X, Y)
        right = [x + 2 * fx - 0.5 * fz, HEIGHT, z + 2 * fz + 0.5 * fx]
        X, Y, _ = oracle_lib.project_point(right, pose, 128, 128)
        assert abs(X - 80 * 256) <= 2 and abs(Y - 16384) <= 2, (yaw, X, Y)
        up = [x + 2 * fx, HEIGHT + 0.5, z + 2 * fz]
        X, Y, _ = oracle_lib.project_point(up, pose, 128, 128)
        assert abs(X - 16384) <= 2 and abs(Y - 48 * 256) <= 2, (yaw, X, Y)


def test_pose_after_36_left_turns_returns(oracle_lib):
    """36 turns of 10 degrees are a full circle: the pose returns to the
    start within the fp64 turn error (far below one fp32 rounding of 1)."""
    ag = np.array([[1.0, 2.0, 0.0, -1.0]])
    p0 = oracle_lib.agent_pose(ag, HEIGHT)
    for _ in range(36):
        ag, _ = act(oracle_lib, np.zeros((0, 4)), ag, [2])
    assert np.abs(oracle_lib.agent_pose(ag, HEIGHT) - p0).max() < 1e-6
