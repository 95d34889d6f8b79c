"""Seeded synthetic inputs shared by the oracle tests and the HIP path.

Holds scene meshes, poses and walks only; none of the rendering arithmetic.
"""
from .scenes import (Rect, Scene, make_room, make_apartment, jitter_positions,
                     aabb, triangle_count, cell_for_target, make_texture, with_texture,
                     TEX_SIZE, TEXEL_PER_M)
from .walks import (pose_from_yaw, poses_from_states, random_poses, random_walks,
                    random_free_states, blocked, SENSOR_HEIGHT, nav_segments,
                    agents_from_states, AGENT_RADIUS, FORWARD_M, TURN_DEG)
from . import configs

__all__ = ["Rect", "Scene", "make_room", "make_apartment", "jitter_positions",
           "aabb", "triangle_count", "cell_for_target", "make_texture", "with_texture",
           "TEX_SIZE", "TEXEL_PER_M", "pose_from_yaw",
           "poses_from_states", "random_poses", "random_walks", "random_free_states",
           "blocked", "SENSOR_HEIGHT", "nav_segments", "agents_from_states",
           "AGENT_RADIUS", "FORWARD_M", "TURN_DEG", "configs"]
