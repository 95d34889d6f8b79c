"""ctypes binding for ``oracle.c``.  TEST INFRASTRUCTURE ONLY.

The C source is compiled with gcc, -O2 -ffp-contract=off and no fast-math,
so every fp32 operation is one IEEE-rounded SSE instruction in source order.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading
from concurrent.futures import ThreadPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
# ORACLE_SANITIZE=1: a build instrumented by AddressSanitizer and
# UndefinedBehaviorSanitizer (liboracle_san.so), loaded with gcc's ASan
# runtime preloaded, for the sanitizer runs of the oracle's own tests
SANITIZE = os.environ.get("ORACLE_SANITIZE") == "1"
LIB = os.path.join(HERE, "liboracle_san.so" if SANITIZE else "liboracle.so")

OR_OK = 0
OR_ERR_INVALID_ARG = 1
OR_ERR_RANGE = 3
NONE = 0xFFFFFFFF

CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fno-builtin",
          "-msse2", "-mfpmath=sse", "-fPIC", "-shared", "-Wall", "-Wextra"]
if SANITIZE:
    CFLAGS += ["-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


class Stats(C.Structure):
    _fields_ = [("bbox_tests", C.c_uint64), ("covered", C.c_uint64),
                ("survivors", C.c_uint64), ("clipped", C.c_uint64)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class Agent(C.Structure):
    _fields_ = [("x", C.c_double), ("z", C.c_double), ("fx", C.c_double), ("fz", C.c_double)]


_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile liboracle.so (always when ``force``)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            lib = C.CDLL(build())
            f32p = C.POINTER(C.c_float)
            u8p = C.POINTER(C.c_uint8)
            u32p = C.POINTER(C.c_uint32)
            i64p = C.POINTER(C.c_int64)
            lib.or_focal.restype = C.c_float
            lib.or_focal.argtypes = [C.c_uint32, C.c_double]
            lib.or_pose_check.restype = C.c_int
            lib.or_pose_check.argtypes = [f32p, f32p, f32p, C.c_uint32, C.c_uint32,
                                          C.c_double, C.c_float]
            lib.or_render_view.restype = C.c_int
            lib.or_render_view.argtypes = [f32p, C.c_uint32, u8p, u32p, C.c_uint32,
                                           C.c_uint32, C.c_uint32, C.c_double, C.c_float,
                                           f32p, u8p, f32p, u32p, f32p, u32p,
                                           C.POINTER(Stats)]
            lib.or_render_view_tex.restype = C.c_int
            lib.or_render_view_tex.argtypes = [f32p, C.c_uint32, u32p, C.c_uint32, f32p, u8p,
                                               C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32,
                                               C.c_double, C.c_float, f32p, u8p, f32p, u32p,
                                               f32p, u32p, C.POINTER(Stats)]
            lib.or_coverage_count.restype = C.c_int
            lib.or_coverage_count.argtypes = [f32p, C.c_uint32, u32p, C.c_uint32,
                                              C.c_uint32, C.c_uint32, C.c_double, C.c_float,
                                              f32p, u32p, C.POINTER(Stats)]
            lib.or_project_point.restype = C.c_int
            lib.or_project_point.argtypes = [f32p, f32p, C.c_uint32, C.c_uint32, C.c_double,
                                             C.c_float, i64p, i64p, f32p]
            u64p = C.POINTER(C.c_uint64)
            f64p = C.POINTER(C.c_double)
            lib.or_philox4x64_10.restype = None
            lib.or_philox4x64_10.argtypes = [u64p, u64p, u64p]
            lib.or_depth_noise_normal.restype = C.c_double
            lib.or_depth_noise_normal.argtypes = [C.c_uint64, C.c_uint64]
            lib.or_actuate.restype = C.c_int
            lib.or_actuate.argtypes = [f32p, C.c_uint32, C.c_double, C.c_double, C.c_double,
                                       C.c_double, C.c_uint32, C.POINTER(Agent), u32p]
            lib.or_nav_slice.restype = C.c_int64
            lib.or_nav_slice.argtypes = [f32p, C.c_uint32, u32p, C.c_uint32, f64p, C.c_uint32, f32p,
                                         C.c_uint64]
            lib.or_nav_free.restype = C.c_int
            lib.or_nav_free.argtypes = [f32p, C.c_uint32, C.c_double, C.c_double, C.c_double]
            lib.or_agent_pose.restype = None
            lib.or_agent_pose.argtypes = [C.POINTER(Agent), C.c_float, f32p]
            lib.or_depth_noise.restype = C.c_int
            lib.or_depth_noise.argtypes = [f32p, u32p, C.c_uint32, C.c_uint32, C.c_double,
                                           C.c_uint64, f64p, f64p]
            _lib = lib
    return _lib


def _ptr(a, ctype):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(ctype))


def _geom(positions, colors, indices):
    pos = np.ascontiguousarray(positions, np.float32).reshape(-1, 3)
    idx = np.ascontiguousarray(indices, np.uint32).reshape(-1, 3)
    col = None if colors is None else np.ascontiguousarray(colors, np.uint8).reshape(-1, 3)
    return pos, col, idx


def focal(W: int, hfov_deg: float) -> float:
    return float(_load().or_focal(W, hfov_deg))


def pose_check(lo, hi, pose, W, H, hfov_deg=90.0, near_m=0.01) -> int:
    lo = np.ascontiguousarray(lo, np.float32)
    hi = np.ascontiguousarray(hi, np.float32)
    pose = np.ascontiguousarray(pose, np.float32)
    return int(_load().or_pose_check(_ptr(lo, C.c_float), _ptr(hi, C.c_float),
                                     _ptr(pose, C.c_float), W, H, hfov_deg, near_m))


def semantic_image(tri, instances):
    """Semantic instance mask (the third attachment of the single render
    pass, Sec. 3 "Rendering engine"; the RGB + depth + semantics row of the
    performance table in the appendix on platform details): each pixel holds
    the instance id of the object its visible triangle belongs to, NONE where
    no triangle is visible."""
    tri = np.asarray(tri, np.uint32)
    inst = np.asarray(instances, np.uint32).reshape(-1)
    out = np.full(tri.shape, NONE, np.uint32)
    for j in range(tri.shape[0]):
        for i in range(tri.shape[1]):
            t = int(tri[j, i])
            if t != NONE:
                out[j, i] = inst[t]
    return out


def philox4x64_10(counter, key):
    """Philox4x64-10 block: four 64-bit words for a 4-word counter and a
    2-word key."""
    c = np.ascontiguousarray(counter, np.uint64).reshape(4)
    k = np.ascontiguousarray(key, np.uint64).reshape(2)
    out = np.empty(4, np.uint64)
    _load().or_philox4x64_10(_ptr(c, C.c_uint64), _ptr(k, C.c_uint64), _ptr(out, C.c_uint64))
    return out


def depth_noise_normal(seed, pixel) -> float:
    """The standard normal deviate of one pixel of a view with this seed."""
    return float(_load().or_depth_noise_normal(int(seed), int(pixel)))


def depth_noise(rho, tri, sigma, seed):
    """Noisy inverse depth and depth (fp64 [H, W]) from a render's raw key
    rho and visible triangle."""
    rho = np.ascontiguousarray(rho, np.float32)
    tri = np.ascontiguousarray(tri, np.uint32)
    H, W = rho.shape
    rp = np.empty((H, W), np.float64)
    dp = np.empty((H, W), np.float64)
    rc = _load().or_depth_noise(_ptr(rho, C.c_float), _ptr(tri, C.c_uint32), W, H, float(sigma),
                                int(seed), _ptr(rp, C.c_double), _ptr(dp, C.c_double))
    if rc != OR_OK:
        raise OracleError(rc)
    return rp, dp


def render_view(positions, colors, indices, W, H, pose, hfov_deg=90.0, near_m=0.01,
                raw=False, instances=None, noise_sigma=0.0, noise_seed=0, uvs=None,
                texture=None):
    """Render one view.  Returns dict(rgb [H,W,3] u8, depth [H,W] f32,
    tri [H,W] u32, stats), with ``instances`` ([T] u32 per-triangle ids) also
    semantic [H,W] u32, with ``noise_sigma`` > 0 also the noisy inverse depth
    and depth (rho_noisy, depth_noisy: [H,W] f64), and with ``raw`` rho
    [H,W] f32 and key [H,W] u32.  With ``uvs`` ([V,2] f32) and ``texture``
    ([th,tw,3] u8) the colour is the bilinear texture fetch.  Raises on a
    non-OK status."""
    pos, col, idx = _geom(positions, colors, indices)
    pose = np.ascontiguousarray(pose, np.float32).reshape(12)
    rgb = np.empty((H, W, 3), np.uint8)
    depth = np.empty((H, W), np.float32)
    tri = np.empty((H, W), np.uint32)
    raw = raw or noise_sigma > 0.0
    rho = np.empty((H, W), np.float32) if raw else None
    key = np.empty((H, W), np.uint32) if raw else None
    st = Stats()
    if texture is not None:
        uv = np.ascontiguousarray(uvs, np.float32).reshape(-1, 2)
        tex = np.ascontiguousarray(texture, np.uint8)
        if uv.shape[0] != pos.shape[0] or tex.ndim != 3 or tex.shape[2] != 3:
            raise ValueError("uvs must be [V, 2] and texture [th, tw, 3]")
        rc = _load().or_render_view_tex(_ptr(pos, C.c_float), pos.shape[0], _ptr(idx, C.c_uint32),
                                        idx.shape[0], _ptr(uv, C.c_float), _ptr(tex, C.c_uint8),
                                        tex.shape[1], tex.shape[0], W, H, hfov_deg, near_m,
                                        _ptr(pose, C.c_float), _ptr(rgb, C.c_uint8),
                                        _ptr(depth, C.c_float), _ptr(tri, C.c_uint32),
                                        _ptr(rho, C.c_float), _ptr(key, C.c_uint32), C.byref(st))
    else:
        rc = _load().or_render_view(_ptr(pos, C.c_float), pos.shape[0], _ptr(col, C.c_uint8),
                                    _ptr(idx, C.c_uint32), idx.shape[0], W, H, hfov_deg, near_m,
                                    _ptr(pose, C.c_float), _ptr(rgb, C.c_uint8),
                                    _ptr(depth, C.c_float), _ptr(tri, C.c_uint32),
                                    _ptr(rho, C.c_float), _ptr(key, C.c_uint32), C.byref(st))
    if rc != OR_OK:
        raise OracleError(rc)
    out = {"rgb": rgb, "depth": depth, "tri": tri, "stats": st.as_dict()}
    if instances is not None:
        out["semantic"] = semantic_image(tri, instances)
    if noise_sigma > 0.0:
        out["rho_noisy"], out["depth_noisy"] = depth_noise(rho, tri, noise_sigma, noise_seed)
    if raw:
        out["rho"] = rho
        out["key"] = key
    return out


def coverage_count(positions, indices, W, H, pose, hfov_deg=90.0, near_m=0.01):
    pos, _, idx = _geom(positions, None, indices)
    pose = np.ascontiguousarray(pose, np.float32).reshape(12)
    cnt = np.empty((H, W), np.uint32)
    st = Stats()
    rc = _load().or_coverage_count(_ptr(pos, C.c_float), pos.shape[0], _ptr(idx, C.c_uint32),
                                   idx.shape[0], W, H, hfov_deg, near_m, _ptr(pose, C.c_float),
                                   _ptr(cnt, C.c_uint32), C.byref(st))
    if rc != OR_OK:
        raise OracleError(rc)
    return cnt, st.as_dict()


def project_point(P, pose, W, H, hfov_deg=90.0, near_m=0.01):
    """(X, Y, rw) in 1/256 px for a world point, or None behind the near plane."""
    P = np.ascontiguousarray(P, np.float32).reshape(3)
    pose = np.ascontiguousarray(pose, np.float32).reshape(12)
    X, Y, rw = C.c_int64(), C.c_int64(), C.c_float()
    rc = _load().or_project_point(_ptr(P, C.c_float), _ptr(pose, C.c_float), W, H, hfov_deg,
                                  near_m, C.byref(X), C.byref(Y), C.byref(rw))
    if rc == 1:
        return None
    if rc != OR_OK:
        raise OracleError(rc)
    return int(X.value), int(Y.value), float(rw.value)


def render_views(positions, colors, indices, W, H, poses, hfov_deg=90.0, near_m=0.01,
                 threads=1):
    """Render several views, one view per thread (ctypes releases the GIL)."""
    poses = np.asarray(poses, np.float32).reshape(-1, 12)
    pos, col, idx = _geom(positions, colors, indices)
    if threads <= 1:
        return [render_view(pos, col, idx, W, H, p, hfov_deg, near_m) for p in poses]
    with ThreadPoolExecutor(max_workers=threads) as ex:
        return list(ex.map(lambda p: render_view(pos, col, idx, W, H, p, hfov_deg, near_m), poses))


class OracleError(RuntimeError):
    def __init__(self, rc):
        super().__init__(f"oracle status {rc}")
        self.status = rc


def actuate(segments, agents, actions, radius, step, turn_cos, turn_sin):
    """Apply one action per agent (0 stop, 1 forward, 2 left, 3 right).
    segments [n, 4] f32 obstacle segments; agents [N, 4] f64 (x, z, fx, fz).
    Returns (new agents [N, 4] f64, collided [N] bool)."""
    seg = np.ascontiguousarray(segments, np.float32).reshape(-1, 4)
    ag = np.ascontiguousarray(agents, np.float64).reshape(-1, 4)
    act = np.asarray(actions, np.uint32).reshape(-1)
    out = ag.copy()
    hit = np.zeros(ag.shape[0], bool)
    lib = _load()
    flag = C.c_uint32()
    for k in range(ag.shape[0]):
        a = Agent(*out[k])
        rc = lib.or_actuate(_ptr(seg, C.c_float), seg.shape[0], float(radius), float(step),
                            float(turn_cos), float(turn_sin), int(act[k]), C.byref(a), C.byref(flag))
        if rc != OR_OK:
            raise OracleError(rc)
        out[k] = (a.x, a.z, a.fx, a.fz)
        hit[k] = bool(flag.value)
    return out, hit


def nav_slice(positions, indices, heights):
    """float32 [n, 4] obstacle segments: the mesh's cross-sections at the
    given heights, in (triangle, height) order."""
    pos = np.ascontiguousarray(positions, np.float32).reshape(-1, 3)
    idx = np.ascontiguousarray(indices, np.uint32).reshape(-1, 3)
    hs = np.ascontiguousarray(heights, np.float64).reshape(-1)
    lib = _load()
    n = lib.or_nav_slice(_ptr(pos, C.c_float), pos.shape[0], _ptr(idx, C.c_uint32), idx.shape[0],
                         _ptr(hs, C.c_double), hs.shape[0], None, 0)
    if n < 0:
        raise OracleError(OR_ERR_INVALID_ARG)
    out = np.zeros((max(n, 1), 4), np.float32)
    m = lib.or_nav_slice(_ptr(pos, C.c_float), pos.shape[0], _ptr(idx, C.c_uint32), idx.shape[0],
                         _ptr(hs, C.c_double), hs.shape[0], _ptr(out, C.c_float), n)
    assert m == n
    return out[:n]


def nav_free(segments, points, radius):
    """bool [N]: is a disc of ``radius`` at each (x, z) of points [N, 2] free
    of every segment?"""
    seg = np.ascontiguousarray(segments, np.float32).reshape(-1, 4)
    pts = np.asarray(points, np.float64).reshape(-1, 2)
    lib = _load()
    sp = _ptr(seg, C.c_float)
    return np.array([bool(lib.or_nav_free(sp, seg.shape[0], float(x), float(z), float(radius)))
                     for x, z in pts], bool)


def agent_pose(agents, height):
    """float32 [N, 12] camera poses (position, row-major world-from-camera
    rotation) of agent states [N, 4] f64 (x, z, fx, fz), the sensor at
    ``height`` above the floor."""
    ag = np.ascontiguousarray(agents, np.float64).reshape(-1, 4)
    out = np.empty((ag.shape[0], 12), np.float32)
    lib = _load()
    buf = (C.c_float * 12)()
    for k in range(ag.shape[0]):
        a = Agent(*ag[k])
        lib.or_agent_pose(C.byref(a), C.c_float(height), buf)
        out[k] = np.frombuffer(buf, np.float32)
    return out
