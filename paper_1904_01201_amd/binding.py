"""ctypes binding of libhabmi.so (the C ABI in include/hab.h).

Argument marshalling only: every step of rendering runs in the library's
HIP kernels.  PyTorch supplies device memory (output tensors) and the HIP
stream (``torch.cuda.current_stream().cuda_stream``).  If the library is
missing, every entry point raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# HABMI_LIBRARY names another build of this library (the sanitizer build of
# the host runtime, for CPU tests); by default the one built next to this file
LIB_PATH = os.environ.get("HABMI_LIBRARY") or os.path.join(HERE, "libhabmi.so")

HAB_OK = 0
HAB_ERR_INVALID_ARG = 1
HAB_ERR_OUT_OF_MEMORY = 2
HAB_ERR_RANGE = 3
HAB_ERR_DEVICE = 4
HAB_ERR_NOT_READY = 5
HAB_ERR_CAPACITY = 6
HAB_ERR_CANCELLED = 7
HAB_ERR_TIMEOUT = 8
HAB_NO_HIT = 0xFFFFFFFF
OUT_RGB, OUT_DEPTH, OUT_TRI, OUT_SEMANTIC = 1, 2, 4, 8
RENDER_ONE_SEQUENCE = 1
RENDER_LANE_OWNED_Z = 2

EXPORTED = [
    "hab_init", "hab_shutdown", "hab_status_string", "hab_get_error",
    "hab_scene_upload", "hab_scene_release", "hab_scene_info", "hab_sensor_spec",
    "hab_render", "hab_render_ex", "hab_render_batch", "hab_render_noalloc",
    "hab_stepper_create", "hab_stepper_step", "hab_stepper_step_device", "hab_stepper_destroy",
    "hab_server_create", "hab_server_submit", "hab_server_submit_ex", "hab_server_cancel",
    "hab_server_poll", "hab_server_wait",
    "hab_server_stats_get", "hab_server_destroy", "hab_autotune",
    "hab_profile_enable", "hab_profile_phases", "hab_profile_read",
    "hab_nav_upload", "hab_nav_from_scene", "hab_nav_segments", "hab_nav_free", "hab_nav_release",
    "hab_actuate", "hab_selfcheck_reciprocal", "hab_test_fail_alloc", "hab_test_live_allocations",
]
ACT_STOP, ACT_FORWARD, ACT_LEFT, ACT_RIGHT = 0, 1, 2, 3
PHASES = ["reset", "setup", "bin_count", "bin_scan", "bin_scatter", "raster8", "raster16",
          "raster32", "resolve"]


class MeshDesc(C.Structure):
    _fields_ = [("positions", C.c_void_p), ("num_vertices", C.c_uint32),
                ("colors", C.c_void_p), ("indices", C.c_void_p), ("num_triangles", C.c_uint32),
                ("instances", C.c_void_p), ("uvs", C.c_void_p), ("texture", C.c_void_p),
                ("tex_width", C.c_uint32), ("tex_height", C.c_uint32)]


class SensorDesc(C.Structure):
    _fields_ = [("width", C.c_uint32), ("height", C.c_uint32), ("hfov_deg", C.c_float),
                ("near_m", C.c_float), ("outputs", C.c_uint32), ("depth_noise_sigma", C.c_float)]


class Sensor(C.Structure):
    _fields_ = [("width", C.c_uint32), ("height", C.c_uint32), ("outputs", C.c_uint32),
                ("hfov_deg", C.c_float), ("f", C.c_float), ("near_m", C.c_float),
                ("depth_noise_sigma", C.c_float)]


class Pose(C.Structure):
    _fields_ = [("position", C.c_float * 3), ("rotation", C.c_float * 9)]


class ViewStats(C.Structure):
    _fields_ = [("survivors", C.c_uint64), ("bbox_tests", C.c_uint64), ("covered", C.c_uint64)]


class RenderOpts(C.Structure):
    _fields_ = [("tile_size", C.c_uint32), ("bin_factor", C.c_float), ("tile_cap", C.c_uint32),
                ("flags", C.c_uint32), ("stats", C.POINTER(ViewStats))]


class View(C.Structure):
    _fields_ = [("scene", C.c_void_p), ("sensor", C.POINTER(Sensor)), ("pose", Pose),
                ("out_rgb", C.c_void_p), ("out_depth", C.c_void_p), ("out_tri", C.c_void_p),
                ("out_semantic", C.c_void_p), ("noise_seed", C.c_uint64)]


class Actuation(C.Structure):
    _fields_ = [("radius", C.c_double), ("forward_m", C.c_double), ("turn_cos", C.c_double),
                ("turn_sin", C.c_double)]


class ServerCfg(C.Structure):
    _fields_ = [("num_streams", C.c_uint32), ("max_batch", C.c_uint32),
                ("memory_budget", C.c_uint64), ("max_queue", C.c_uint32),
                ("max_wait_us", C.c_uint32)]


class RequestStats(C.Structure):
    _fields_ = [("submit_ns", C.c_uint64), ("launch_ns", C.c_uint64), ("done_ns", C.c_uint64),
                ("batch_size", C.c_uint32), ("batch_id", C.c_uint32)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_uint64), ("completed", C.c_uint64), ("batches", C.c_uint64),
                ("rejected", C.c_uint64), ("peak_inflight_bytes", C.c_uint64),
                ("peak_batch", C.c_uint32), ("pad", C.c_uint32), ("cancelled", C.c_uint64),
                ("expired", C.c_uint64), ("scratch_bytes", C.c_uint64)]


class PhaseTimes(C.Structure):
    _fields_ = [("ms", C.c_double * 9), ("launches", C.c_uint64 * 9), ("sequences", C.c_uint64)]


class HabError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        msg = _status_string(status)
        super().__init__(f"{what}: {msg} ({status})" if what else f"{msg} ({status})")
        self.status = status


_lock = threading.Lock()
_lib = None


def lib_path() -> str:
    return LIB_PATH


def load():
    """Load libhabmi.so (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1904_01201_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, u32, f32 = C.c_void_p, C.c_uint32, C.c_float
        st = C.c_int
        L.hab_status_string.restype = C.c_char_p
        L.hab_status_string.argtypes = [st]
        sig = {
            "hab_init": [C.c_int, C.POINTER(vp)],
            "hab_shutdown": [vp],
            "hab_get_error": [vp],
            "hab_scene_upload": [vp, C.POINTER(MeshDesc), vp, C.POINTER(vp)],
            "hab_scene_release": [vp, vp],
            "hab_scene_info": [vp, C.POINTER(u32), C.POINTER(u32), C.POINTER(C.c_uint64),
                               C.POINTER(f32), C.POINTER(f32)],
            "hab_sensor_spec": [C.POINTER(SensorDesc), C.POINTER(Sensor)],
            "hab_render": [vp, vp, C.POINTER(Sensor), C.POINTER(Pose), u32, vp, vp, vp],
            "hab_render_ex": [vp, vp, C.POINTER(Sensor), C.POINTER(Pose), u32, vp, vp, vp,
                              C.POINTER(RenderOpts), vp],
            "hab_render_batch": [vp, C.POINTER(View), u32, C.POINTER(RenderOpts), vp],
            "hab_render_noalloc": [vp, vp, C.POINTER(Sensor), C.POINTER(Pose), u32, vp, vp, vp],
            "hab_stepper_create": [vp, C.POINTER(View), u32, C.POINTER(RenderOpts), vp,
                                   C.POINTER(vp)],
            "hab_stepper_step": [vp, C.POINTER(Pose), vp],
            "hab_stepper_step_device": [vp, vp, vp],
            "hab_stepper_destroy": [vp],
            "hab_server_create": [vp, C.POINTER(ServerCfg), C.POINTER(vp)],
            "hab_server_submit": [vp, C.POINTER(View), C.POINTER(C.c_uint64)],
            "hab_server_submit_ex": [vp, C.POINTER(View), u32, C.POINTER(C.c_uint64)],
            "hab_server_cancel": [vp, C.c_uint64],
            "hab_test_fail_alloc": [C.c_int64],
            "hab_test_live_allocations": [C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)],
            "hab_server_poll": [vp, C.c_uint64, C.POINTER(RequestStats)],
            "hab_server_wait": [vp, C.c_uint64, C.POINTER(RequestStats)],
            "hab_server_stats_get": [vp, C.POINTER(ServerStats)],
            "hab_server_destroy": [vp],
            "hab_autotune": [vp, C.POINTER(View), u32, vp, C.POINTER(u32), C.POINTER(f32)],
            "hab_profile_enable": [vp, C.c_int],
            "hab_profile_phases": [vp, C.c_uint32],
            "hab_profile_read": [vp, C.POINTER(PhaseTimes)],
            "hab_nav_upload": [vp, vp, u32, C.POINTER(vp)],
            "hab_nav_from_scene": [vp, vp, vp, u32, vp, C.POINTER(vp)],
            "hab_nav_segments": [vp, vp, vp, u32, C.POINTER(u32)],
            "hab_nav_free": [vp, vp, vp, u32, C.c_double, vp, vp],
            "hab_nav_release": [vp, vp],
            "hab_actuate": [vp, C.POINTER(vp), u32, vp, vp, vp, vp, f32, C.POINTER(Actuation), vp],
            "hab_selfcheck_reciprocal": [vp, u32, u32, vp, C.POINTER(C.c_uint64)],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.restype = st
            fn.argtypes = args
        _lib = L
        return L


def _status_string(s: int) -> str:
    try:
        return load().hab_status_string(s).decode()
    except Exception:
        return f"status {s}"


def check(status: int, what: str = ""):
    if status != HAB_OK:
        raise HabError(status, what)


def poses_to_c(poses) -> C.Array:
    """[N, 12] float32 (p[3], R[9]) -> contiguous hab_pose array."""
    p = np.ascontiguousarray(np.asarray(poses, np.float32).reshape(-1, 12))
    arr = (Pose * p.shape[0])()
    C.memmove(arr, p.ctypes.data, p.nbytes)
    return arr


def pose_to_c(pose) -> Pose:
    p = np.ascontiguousarray(np.asarray(pose, np.float32).reshape(12))
    out = Pose()
    C.memmove(C.byref(out), p.ctypes.data, 48)
    return out
