"""The five synthetic workloads, each fully determined by fixed seeds.

  room_2k_128       one room (~2k triangles), 128x128 RGB+D, 100 random poses
  apartment_200k_256  2x4-room apartment (~200k triangles), 256x256 RGB+D,
                    1,000-step random walk
  batch64_4scenes_256 64 environments over 4 jittered apartments of
                    100k/250k/500k/1M triangles, 256x256 RGB+D, 500 steps
  batch256_16scenes_mixed 256 environments over 16 jittered apartments of
                    50k-1.5M triangles (log-uniform), per-environment resolution
                    in {128, 256, 512} and sensor in {D, RGB, RGB+D}, 500 steps
  serve_32scenes    32 resident jittered apartments, sum T ~ 20M, mixed
                    sensors as above, for the serving load generator

The sensor defaults follow the paper (Sec. 4 "Sensory input": 256x256 colour
and depth at a 90 degree field of view, mounted 1.5 m high).  Table 1 times
128/256/512 resolutions.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .scenes import Scene, make_room, make_apartment
from .walks import random_poses, random_walks

OUT_RGB = 1
OUT_DEPTH = 2
OUT_RGBD = 3
NEAR_M = 0.01
HFOV_DEG = 90.0


@dataclass
class Sensor:
    width: int
    height: int
    hfov_deg: float = HFOV_DEG
    near_m: float = NEAR_M
    outputs: int = OUT_RGBD


@dataclass
class Workload:
    name: str
    scenes: list
    env_scene: np.ndarray          # [E] scene index per environment
    env_sensor: list               # [E] Sensor per environment
    poses: np.ndarray              # [steps, E, 12] float32
    meta: dict = field(default_factory=dict)

    @property
    def num_envs(self) -> int:
        return int(self.env_scene.shape[0])

    @property
    def num_steps(self) -> int:
        return int(self.poses.shape[0])


def room_2k_128() -> Workload:
    sc = make_room(seed=11)
    poses = random_poses(sc, 100, seed=12)[:, None, :]          # 100 steps x 1 env
    return Workload("room_2k_128", [sc], np.zeros(1, np.int64), [Sensor(128, 128)], poses)


def apartment_200k_256(steps: int = 1000) -> Workload:
    sc = make_apartment(seed=20, target_T=200_000)
    poses = random_walks(sc, 1, steps, seed=21)
    return Workload("apartment_200k_256", [sc], np.zeros(1, np.int64), [Sensor(256, 256)], poses)


def batch64_4scenes_256(steps: int = 500, scene_T=(100_000, 250_000, 500_000, 1_000_000)) -> Workload:
    scenes = [make_apartment(seed=30 + k, target_T=int(t), jitter_sigma=0.01)
              for k, t in enumerate(scene_T)]
    per = 64 // len(scenes)
    env_scene = np.repeat(np.arange(len(scenes)), per)
    walks = [random_walks(scenes[k], per, steps, seed=300 + k) for k in range(len(scenes))]
    poses = np.concatenate(walks, axis=1)
    return Workload("batch64_4scenes_256", scenes, env_scene,
                    [Sensor(256, 256) for _ in range(env_scene.shape[0])], poses)


def _mixed_sensors(n, seed):
    rng = np.random.Generator(np.random.PCG64([seed, 5]))
    res = rng.choice([128, 256, 512], size=n)
    outs = rng.choice([OUT_DEPTH, OUT_RGB, OUT_RGBD], size=n)
    return [Sensor(int(r), int(r), outputs=int(o)) for r, o in zip(res, outs)]


def batch256_16scenes_mixed(steps: int = 500, num_scenes: int = 16, envs_per_scene: int = 16) -> Workload:
    rng = np.random.Generator(np.random.PCG64([40, 6]))
    Ts = np.exp(rng.uniform(np.log(50_000), np.log(1_500_000), size=num_scenes)).astype(np.int64)
    scenes = [make_apartment(seed=400 + k, target_T=int(t), jitter_sigma=0.01) for k, t in enumerate(Ts)]
    env_scene = np.repeat(np.arange(num_scenes), envs_per_scene)
    walks = [random_walks(scenes[k], envs_per_scene, steps, seed=4000 + k) for k in range(num_scenes)]
    poses = np.concatenate(walks, axis=1)
    return Workload("batch256_16scenes_mixed", scenes, env_scene,
                    _mixed_sensors(env_scene.shape[0], 41), poses)


def serve_32scenes(num_agents: int = 512, steps: int = 64, total_T: int = 20_000_000,
                   num_scenes: int = 32) -> Workload:
    rng = np.random.Generator(np.random.PCG64([50, 6]))
    Ts = np.exp(rng.uniform(np.log(100_000), np.log(1_500_000), size=num_scenes))
    Ts = np.maximum(Ts * (total_T / Ts.sum()), 20_000).astype(np.int64)
    scenes = [make_apartment(seed=500 + k, target_T=int(t), jitter_sigma=0.01) for k, t in enumerate(Ts)]
    env_scene = rng.integers(0, num_scenes, size=num_agents)
    poses = np.empty((steps, num_agents, 12), np.float32)
    for k in range(num_scenes):
        sel = np.nonzero(env_scene == k)[0]
        if sel.size:
            poses[:, sel, :] = random_walks(scenes[k], sel.size, steps, seed=5000 + k)
    return Workload("serve_32scenes", scenes, env_scene, _mixed_sensors(num_agents, 51), poses)


ALL = {
    "room_2k_128": room_2k_128,
    "apartment_200k_256": apartment_200k_256,
    "batch64_4scenes_256": batch64_4scenes_256,
    "batch256_16scenes_mixed": batch256_16scenes_mixed,
    "serve_32scenes": serve_32scenes,
}
