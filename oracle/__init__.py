"""CPU oracle for the RGB+D sensor renderer.  TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The rendering library
(``paper_1904_01201_amd``) never imports it and shares no code with it.

``oracle.c`` is the plain C reference (built here with gcc, SSE fp32 math,
no FP contraction); ``raycast_fp64`` is an independent FP64 brute-force ray
caster used to pin the oracle on tiny scenes.
"""
from .binding import (build, focal, pose_check, render_view, coverage_count,
                      project_point, render_views, semantic_image, philox4x64_10,
                      depth_noise_normal, depth_noise, actuate, agent_pose, nav_slice, nav_free, OR_OK, OR_ERR_INVALID_ARG,
                      OR_ERR_RANGE, NONE)

__all__ = ["build", "focal", "pose_check", "render_view", "coverage_count",
           "project_point", "render_views", "semantic_image", "philox4x64_10",
           "depth_noise_normal", "depth_noise", "actuate", "agent_pose", "nav_slice", "nav_free", "OR_OK",
           "OR_ERR_INVALID_ARG", "OR_ERR_RANGE", "NONE"]
