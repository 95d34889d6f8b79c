"""Python front end of the renderer: a context with resident scenes,
sensors, per-view / batched rendering, a graph-captured stepper, a serving
loop and the autotuner.  Thin wrappers over the C ABI (include/hab.h)."""
from __future__ import annotations

import ctypes as C
import math
from dataclasses import dataclass

import numpy as np

from . import binding as B


def _torch():
    import torch
    return torch


def _stream_ptr(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(int(stream.cuda_stream))


def _ptr(t):
    return None if t is None else C.c_void_p(int(t.data_ptr()))


_DT = {"rgb": "uint8", "depth": "float32", "tri": ("int32", "uint32"),
       "semantic": ("int32", "uint32")}


def check_output(name, t, n, sensor):
    """Refuse an output tensor that is not a contiguous CUDA tensor of the
    exact size the library will write ([n, H, W, 3] uint8, [n, H, W] float32
    or [n, H, W] int32)."""
    if t is None:
        return
    torch = _torch()
    H, W = int(sensor.height), int(sensor.width)
    want = n * H * W * (3 if name == "rgb" else 1)
    dt = str(t.dtype).replace("torch.", "")
    ok_dt = _DT[name] if isinstance(_DT[name], tuple) else (_DT[name],)
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name}: expected a CUDA tensor")
    if dt not in ok_dt:
        raise ValueError(f"{name}: dtype {dt}, expected {ok_dt[0]}")
    if not t.is_contiguous() or t.numel() != want:
        raise ValueError(f"{name}: need a contiguous tensor of {want} elements, got {tuple(t.shape)}")


@dataclass
class NavHandle:
    ptr: int
    num_segments: int


@dataclass
class SceneHandle:
    ptr: int
    num_vertices: int
    num_triangles: int
    device_bytes: int
    lo: tuple
    hi: tuple


class Context:
    """One device context (scenes stay resident in HBM until released)."""

    def __init__(self, device: int = 0):
        # torch provides the device memory and streams: bring its runtime up
        # on the device first (initialised after the library, it may not
        # enumerate the GPU)
        torch = _torch()
        if torch.cuda.is_available():
            torch.cuda.set_device(device)
        self.lib = B.load()
        self.device = device
        h = C.c_void_p()
        B.check(self.lib.hab_init(device, C.byref(h)), "hab_init")
        self.h = h
        self._scenes = []

    def close(self):
        if self.h:
            B.check(self.lib.hab_shutdown(self.h), "hab_shutdown")
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # ------------------------------------------------------------ scenes
    def upload(self, positions, colors, indices, instances=None, stream=None, uvs=None,
               texture=None) -> SceneHandle:
        """instances: optional [T] uint32 instance id per triangle (needed
        for the semantic output); uvs [V, 2] float32 with texture [th, tw, 3]
        uint8 (powers of two): textured colour."""
        pos = np.ascontiguousarray(positions, np.float32).reshape(-1, 3)
        idx = np.ascontiguousarray(indices, np.uint32).reshape(-1, 3)
        col = None if colors is None else np.ascontiguousarray(colors, np.uint8).reshape(-1, 3)
        ins = None
        if instances is not None:
            ins = np.ascontiguousarray(instances, np.uint32).reshape(-1)
            if ins.shape[0] != idx.shape[0]:
                raise ValueError(f"instances: {ins.shape[0]} ids for {idx.shape[0]} triangles")
        uv = tex = None
        if (uvs is None) != (texture is None):
            raise ValueError("uvs and texture go together")
        if texture is not None:
            uv = np.ascontiguousarray(uvs, np.float32).reshape(-1, 2)
            tex = np.ascontiguousarray(texture, np.uint8)
            if uv.shape[0] != pos.shape[0] or tex.ndim != 3 or tex.shape[2] != 3:
                raise ValueError("uvs must be [V, 2] and texture [th, tw, 3]")
        d = B.MeshDesc(pos.ctypes.data, pos.shape[0], None if col is None else col.ctypes.data,
                       idx.ctypes.data if idx.size else None, idx.shape[0],
                       ins.ctypes.data if ins is not None and ins.size else None,
                       None if uv is None else uv.ctypes.data,
                       None if tex is None else tex.ctypes.data,
                       0 if tex is None else tex.shape[1], 0 if tex is None else tex.shape[0])
        out = C.c_void_p()
        B.check(self.lib.hab_scene_upload(self.h, C.byref(d), _stream_ptr(stream), C.byref(out)),
                "hab_scene_upload")
        nv, nt, nb = C.c_uint32(), C.c_uint32(), C.c_uint64()
        lo, hi = (C.c_float * 3)(), (C.c_float * 3)()
        B.check(self.lib.hab_scene_info(out, C.byref(nv), C.byref(nt), C.byref(nb), lo, hi))
        s = SceneHandle(out.value, nv.value, nt.value, nb.value, tuple(lo), tuple(hi))
        self._scenes.append(s)
        return s

    def upload_scene(self, scene, stream=None) -> SceneHandle:
        """Upload a generated scene (its instance table, and its texture when
        one is attached)."""
        tex = getattr(scene, "texture", None)
        return self.upload(scene.positions, scene.colors, scene.indices,
                           getattr(scene, "instances", None), stream=stream,
                           uvs=None if tex is None else scene.uvs, texture=tex)

    def release(self, scene: SceneHandle):
        B.check(self.lib.hab_scene_release(self.h, C.c_void_p(scene.ptr)), "hab_scene_release")
        self._scenes.remove(scene)

    # ------------------------------------------------------------ sensors
    @staticmethod
    def sensor(width, height, hfov_deg=90.0, near_m=0.01, outputs=B.OUT_RGB | B.OUT_DEPTH,
               depth_noise_sigma=0.0) -> B.Sensor:
        """depth_noise_sigma: iid Gaussian noise on the inverse depth, in 1/m."""
        lib = B.load()
        d = B.SensorDesc(int(width), int(height), float(hfov_deg), float(near_m), int(outputs),
                         float(depth_noise_sigma))
        s = B.Sensor()
        B.check(lib.hab_sensor_spec(C.byref(d), C.byref(s)), "hab_sensor_spec")
        return s

    # ------------------------------------------------------------ outputs
    @staticmethod
    def alloc(sensor: B.Sensor, n: int, tri: bool = False, device="cuda"):
        torch = _torch()
        H, W = sensor.height, sensor.width
        out = {}
        if sensor.outputs & B.OUT_RGB:
            out["rgb"] = torch.empty((n, H, W, 3), dtype=torch.uint8, device=device)
        if sensor.outputs & B.OUT_DEPTH:
            out["depth"] = torch.empty((n, H, W), dtype=torch.float32, device=device)
        if tri or (sensor.outputs & B.OUT_TRI):
            out["tri"] = torch.empty((n, H, W), dtype=torch.int32, device=device)
        if sensor.outputs & B.OUT_SEMANTIC:
            out["semantic"] = torch.empty((n, H, W), dtype=torch.int32, device=device)
        return out

    @staticmethod
    def _opts(tile_size=0, bin_factor=0.0, tile_cap=0, stats=None, one_sequence=False, lane_owned_z=False):
        flags = (B.RENDER_ONE_SEQUENCE if one_sequence else 0) | (B.RENDER_LANE_OWNED_Z if lane_owned_z else 0)
        o = B.RenderOpts(int(tile_size), float(bin_factor), int(tile_cap), flags, None)
        if stats is not None:
            o.stats = C.cast(stats, C.POINTER(B.ViewStats))
        return o

    # ------------------------------------------------------------ render
    def render(self, scene: SceneHandle, sensor: B.Sensor, poses, rgb=None, depth=None, tri=None,
               tile_size=0, bin_factor=0.0, tile_cap=0, stats=False, stream=None, out=None,
               one_sequence=False, lane_owned_z=False):
        """Render N views of one scene.  Returns dict of output tensors (and
        'stats': list of dicts if requested).  A sensor with the semantic
        output goes through hab_render_batch (one view per pose, noise seed =
        pose index as in hab_render_ex), since hab_render_ex has no semantic
        output."""
        poses = np.asarray(poses, np.float32).reshape(-1, 12)
        n = poses.shape[0]
        if out is None:
            out = {}
        if rgb is not None:
            out["rgb"] = rgb
        if depth is not None:
            out["depth"] = depth
        if tri is not None:
            out["tri"] = tri
        if not out:
            out = self.alloc(sensor, n, tri=False)
        for k in ("rgb", "depth", "tri", "semantic"):
            check_output(k, out.get(k), n, sensor)
        if out.get("semantic") is not None:
            items = [(scene, sensor, poses[k], *[None if out.get(name) is None else out[name][k]
                                                 for name in ("rgb", "depth", "tri", "semantic")], k)
                     for k in range(n)]
            st = self.render_batch(items, tile_size, bin_factor, tile_cap, stats, stream,
                                   one_sequence=one_sequence, lane_owned_z=lane_owned_z)
            if stats:
                out["stats"] = st
            return out
        st = (B.ViewStats * n)() if stats else None
        o = self._opts(tile_size, bin_factor, tile_cap, st, one_sequence, lane_owned_z)
        pc = B.poses_to_c(poses)
        B.check(self.lib.hab_render_ex(self.h, C.c_void_p(scene.ptr), C.byref(sensor), pc, n,
                                       _ptr(out.get("rgb")), _ptr(out.get("depth")),
                                       _ptr(out.get("tri")), C.byref(o), _stream_ptr(stream)),
                "hab_render_ex")
        if stats:
            out["stats"] = [{"survivors": s.survivors, "bbox_tests": s.bbox_tests,
                             "covered": s.covered} for s in st]
        return out

    def render_plain(self, scene, sensor, poses, rgb=None, depth=None, stream=None):
        """hab_render: the minimal entry point."""
        poses = np.asarray(poses, np.float32).reshape(-1, 12)
        check_output("rgb", rgb, poses.shape[0], sensor)
        check_output("depth", depth, poses.shape[0], sensor)
        pc = B.poses_to_c(poses)
        B.check(self.lib.hab_render(self.h, C.c_void_p(scene.ptr), C.byref(sensor), pc,
                                    poses.shape[0], _ptr(rgb), _ptr(depth), _stream_ptr(stream)),
                "hab_render")

    def render_noalloc(self, scene, sensor, poses, rgb=None, depth=None, stream=None):
        """hab_render_noalloc: hab_render on the library's static scratch
        array (no allocation in the call)."""
        poses = np.asarray(poses, np.float32).reshape(-1, 12)
        check_output("rgb", rgb, poses.shape[0], sensor)
        check_output("depth", depth, poses.shape[0], sensor)
        pc = B.poses_to_c(poses)
        B.check(self.lib.hab_render_noalloc(self.h, C.c_void_p(scene.ptr), C.byref(sensor), pc,
                                            poses.shape[0], _ptr(rgb), _ptr(depth), _stream_ptr(stream)),
                "hab_render_noalloc")

    @staticmethod
    def set_poses(views, poses):
        """Write [n, 12] float32 poses (p[3], R[9]) into the n records of a
        View array (from make_views) in place, all at once.  No checks here:
        the library validates every pose when the views are rendered."""
        p = np.ascontiguousarray(np.asarray(poses, np.float32).reshape(-1, 12))
        n = len(views)
        if p.shape[0] != n:
            raise ValueError(f"{p.shape[0]} poses for {n} views")
        raw = np.frombuffer((C.c_char * C.sizeof(views)).from_buffer(views), dtype=np.uint8)
        off = B.View.pose.offset
        raw.reshape(n, C.sizeof(B.View))[:, off:off + C.sizeof(B.Pose)].view(np.float32)[:] = p

    def make_views(self, items):
        """items: iterable of (scene, sensor, pose, rgb, depth, tri[, semantic
        [, noise_seed]]) with tensors or None.  Returns a ctypes View array
        (keeps sensors alive)."""
        items = list(items)
        arr = (B.View * len(items))()
        keep = []
        for k, it in enumerate(items):
            scene, sensor, pose, rgb, depth, tri = it[:6]
            sem = it[6] if len(it) > 6 else None
            seed = int(it[7]) if len(it) > 7 else 0
            check_output("rgb", rgb, 1, sensor)
            check_output("depth", depth, 1, sensor)
            check_output("tri", tri, 1, sensor)
            check_output("semantic", sem, 1, sensor)
            keep.append(sensor)
            arr[k].scene = scene.ptr
            arr[k].sensor = C.pointer(sensor)
            arr[k].pose = B.pose_to_c(pose)
            arr[k].out_rgb = None if rgb is None else int(rgb.data_ptr())
            arr[k].out_depth = None if depth is None else int(depth.data_ptr())
            arr[k].out_tri = None if tri is None else int(tri.data_ptr())
            arr[k].out_semantic = None if sem is None else int(sem.data_ptr())
            arr[k].noise_seed = seed
        arr._keep = keep
        return arr

    def render_batch(self, items, tile_size=0, bin_factor=0.0, tile_cap=0, stats=False, stream=None,
                     views=None, one_sequence=False, lane_owned_z=False):
        """Render a list of views (or prepared hab_view records, `views`).
        32 or more views run as two launch sequences side by side unless
        one_sequence; lane_owned_z selects the atomic-free lane-owned
        z-test (same outputs)."""
        arr = views if views is not None else self.make_views(items)
        n = len(arr)
        st = (B.ViewStats * n)() if stats else None
        o = self._opts(tile_size, bin_factor, tile_cap, st, one_sequence, lane_owned_z)
        B.check(self.lib.hab_render_batch(self.h, arr, n, C.byref(o), _stream_ptr(stream)),
                "hab_render_batch")
        if stats:
            return [{"survivors": s.survivors, "bbox_tests": s.bbox_tests, "covered": s.covered}
                    for s in st]
        return None

    def get_error(self) -> int:
        return int(self.lib.hab_get_error(self.h))

    # ------------------------------------------------------------ profiling
    def profile(self, on: bool = True):
        B.check(self.lib.hab_profile_enable(self.h, 1 if on else 0), "hab_profile_enable")

    def profile_phases(self, names=None):
        """Time only the named phases (None: all)."""
        mask = (1 << len(B.PHASES)) - 1 if names is None else sum(1 << B.PHASES.index(n) for n in names)
        B.check(self.lib.hab_profile_phases(self.h, mask), "hab_profile_phases")

    def profile_read(self):
        """Per-phase summed device ms and launch counts since the last read."""
        t = B.PhaseTimes()
        B.check(self.lib.hab_profile_read(self.h, C.byref(t)), "hab_profile_read")
        return {name: {"ms": t.ms[k], "launches": int(t.launches[k])}
                for k, name in enumerate(B.PHASES) if t.launches[k]}

    # ------------------------------------------------------------ self-check
    def selfcheck_reciprocal(self, lo_bits: int = 0x00800000, hi_bits: int = 0x7E800000, stream=None) -> int:
        """Floats with bits in [lo_bits, hi_bits) whose reciprocal, as the
        setup and raster take it, differs from the IEEE quotient 1/x."""
        n = C.c_uint64()
        B.check(self.lib.hab_selfcheck_reciprocal(self.h, lo_bits, hi_bits, _stream_ptr(stream), C.byref(n)),
                "hab_selfcheck_reciprocal")
        return int(n.value)

    # ------------------------------------------------------------ actuation
    def nav_upload(self, segments) -> "NavHandle":
        """Obstacle segments [n, 4] float32 (x0, z0, x1, z1) of one scene."""
        seg = np.ascontiguousarray(segments, np.float32).reshape(-1, 4)
        out = C.c_void_p()
        B.check(self.lib.hab_nav_upload(self.h, seg.ctypes.data if seg.size else None,
                                        seg.shape[0], C.byref(out)), "hab_nav_upload")
        return NavHandle(out.value, seg.shape[0])

    def nav_from_scene(self, scene: SceneHandle, heights=(0.1, 1.5), stream=None) -> "NavHandle":
        """Obstacles from the scene's own mesh: its cross-sections at the
        given heights, computed on the device."""
        hs = np.ascontiguousarray(heights, np.float64).reshape(-1)
        out = C.c_void_p()
        B.check(self.lib.hab_nav_from_scene(self.h, C.c_void_p(scene.ptr), hs.ctypes.data, hs.shape[0],
                                            _stream_ptr(stream), C.byref(out)), "hab_nav_from_scene")
        n = C.c_uint32()
        B.check(self.lib.hab_nav_segments(self.h, out.value, None, 0, C.byref(n)), "hab_nav_segments")
        return NavHandle(out.value, int(n.value))

    def nav_segments(self, nav: "NavHandle") -> np.ndarray:
        """The obstacle set's segments [n, 4] float32, in order."""
        seg = np.zeros((max(nav.num_segments, 1), 4), np.float32)
        n = C.c_uint32()
        B.check(self.lib.hab_nav_segments(self.h, C.c_void_p(nav.ptr), seg.ctypes.data, nav.num_segments, C.byref(n)),
                "hab_nav_segments")
        return seg[:n.value]

    def nav_free(self, nav: "NavHandle", points, radius=0.1, out=None, stream=None):
        """uint8 [N] device tensor: 1 where a disc of ``radius`` at each (x, z)
        of points (device float64 [N, 2]) is clear of the obstacles."""
        torch = _torch()
        assert points.dtype == torch.float64 and points.is_cuda and points.is_contiguous()
        assert points.dim() == 2 and points.shape[1] == 2
        n = points.shape[0]
        if out is None:
            out = torch.empty(n, dtype=torch.uint8, device=points.device)
        assert out.dtype == torch.uint8 and out.numel() >= n and out.is_contiguous()
        B.check(self.lib.hab_nav_free(self.h, C.c_void_p(nav.ptr), _ptr(points), n, float(radius), _ptr(out),
                                      _stream_ptr(stream)), "hab_nav_free")
        return out

    def nav_release(self, nav: "NavHandle"):
        B.check(self.lib.hab_nav_release(self.h, C.c_void_p(nav.ptr)), "hab_nav_release")

    @staticmethod
    def actuation(radius=0.1, forward_m=0.25, turn_deg=10.0) -> B.Actuation:
        t = math.radians(turn_deg)
        return B.Actuation(float(radius), float(forward_m), math.cos(t), math.sin(t))

    @staticmethod
    def nav_array(navs):
        """A reusable argument for actuate(): the per-agent NavHandles as the
        C array the library takes."""
        return (C.c_void_p * len(navs))(*[nv.ptr for nv in navs])

    def actuate(self, navs, agents, actions, collided=None, poses=None, camera_height=1.5,
                params=None, stream=None):
        """One action per agent.  navs: a NavHandle per agent (or a
        nav_array() of them); agents [n, 4] float64, actions [n] uint8,
        collided [n] uint8, poses [n, 12] float32: contiguous CUDA tensors
        (agents updated in place)."""
        torch = _torch()
        n = len(navs)
        for name, t, dt, per in (("agents", agents, torch.float64, 4), ("actions", actions, torch.uint8, 1),
                                 ("collided", collided, torch.uint8, 1), ("poses", poses, torch.float32, 12)):
            if t is None:
                if name in ("agents", "actions"):
                    raise ValueError(f"{name} is required")
                continue
            if not (isinstance(t, torch.Tensor) and t.is_cuda and t.is_contiguous()
                    and t.dtype == dt and t.numel() == n * per):
                raise ValueError(f"{name}: need a contiguous CUDA {dt} tensor of {n * per} elements")
        arr = navs if isinstance(navs, C.Array) else self.nav_array(navs)
        p = params if params is not None else self.actuation()
        B.check(self.lib.hab_actuate(self.h, arr, n, _ptr(agents), _ptr(actions), _ptr(collided),
                                     _ptr(poses), float(camera_height), C.byref(p),
                                     _stream_ptr(stream)), "hab_actuate")

    # ------------------------------------------------------------ stepper
    def stepper(self, items, tile_size=0, bin_factor=0.0, tile_cap=0, stream=None, one_sequence=False,
                lane_owned_z=False):
        return Stepper(self, items, tile_size, bin_factor, tile_cap, stream, one_sequence, lane_owned_z)

    # ------------------------------------------------------------ autotune
    def autotune(self, items, stream=None):
        arr = self.make_views(items)
        ts, bf = C.c_uint32(), C.c_float()
        B.check(self.lib.hab_autotune(self.h, arr, len(arr), _stream_ptr(stream), C.byref(ts),
                                      C.byref(bf)), "hab_autotune")
        return int(ts.value), float(bf.value)


class Stepper:
    """A fixed batch composition captured as a HIP graph; step(poses)."""

    def __init__(self, ctx: Context, items, tile_size=0, bin_factor=0.0, tile_cap=0, stream=None,
                 one_sequence=False, lane_owned_z=False):
        self.ctx = ctx
        self.views = ctx.make_views(items)
        o = Context._opts(tile_size, bin_factor, tile_cap, one_sequence=one_sequence,
                          lane_owned_z=lane_owned_z)
        h = C.c_void_p()
        B.check(ctx.lib.hab_stepper_create(ctx.h, self.views, len(self.views), C.byref(o),
                                           _stream_ptr(stream), C.byref(h)), "hab_stepper_create")
        self.h = h

    def step(self, poses, stream=None):
        pc = B.poses_to_c(poses)
        if len(pc) != len(self.views):
            raise ValueError("one pose per view")
        B.check(self.ctx.lib.hab_stepper_step(self.h, pc, _stream_ptr(stream)), "hab_stepper_step")

    def step_device(self, poses, stream=None):
        """A step whose poses are already on the device: a contiguous CUDA
        float32 tensor [n, 12] in the views' order (e.g. actuate()'s poses
        output)."""
        torch = _torch()
        n = len(self.views)
        if not (isinstance(poses, torch.Tensor) and poses.is_cuda and poses.is_contiguous()
                and poses.dtype == torch.float32 and poses.numel() == 12 * n):
            raise ValueError(f"poses: need a contiguous CUDA float32 tensor of {12 * n} elements")
        B.check(self.ctx.lib.hab_stepper_step_device(self.h, _ptr(poses), _stream_ptr(stream)),
                "hab_stepper_step_device")

    def close(self):
        if self.h:
            B.check(self.ctx.lib.hab_stepper_destroy(self.h), "hab_stepper_destroy")
            self.h = None


class Server:
    """Continuous-batching request loop over the context's resident scenes.

    submit() is non-blocking and returns a ticket; the request's output
    tensors must stay alive until poll()/wait() reports it complete.  While
    a server runs, the context is used only through it."""

    def __init__(self, ctx: Context, num_streams=2, max_batch=256, memory_budget=8 << 30,
                 max_queue=65536, max_wait_us=0):
        self.ctx = ctx
        self.lib = ctx.lib
        cfg = B.ServerCfg(int(num_streams), int(max_batch), int(memory_budget), int(max_queue),
                          int(max_wait_us))
        h = C.c_void_p()
        B.check(self.lib.hab_server_create(ctx.h, C.byref(cfg), C.byref(h)), "hab_server_create")
        self.h = h
        self._keep = {}

    def submit(self, scene, sensor, pose, rgb=None, depth=None, tri=None, semantic=None,
               noise_seed=0, timeout_us=0) -> int:
        check_output("rgb", rgb, 1, sensor)
        check_output("depth", depth, 1, sensor)
        check_output("tri", tri, 1, sensor)
        check_output("semantic", semantic, 1, sensor)
        v = B.View()
        v.scene = scene.ptr
        v.sensor = C.pointer(sensor)
        v.pose = B.pose_to_c(pose)
        v.out_rgb = None if rgb is None else int(rgb.data_ptr())
        v.out_depth = None if depth is None else int(depth.data_ptr())
        v.out_tri = None if tri is None else int(tri.data_ptr())
        v.out_semantic = None if semantic is None else int(semantic.data_ptr())
        v.noise_seed = int(noise_seed)
        t = C.c_uint64()
        B.check(self.lib.hab_server_submit_ex(self.h, C.byref(v), int(timeout_us), C.byref(t)),
                "hab_server_submit_ex")
        self._keep[t.value] = (rgb, depth, tri, semantic)
        return t.value

    @staticmethod
    def _stats(rs):
        return {"submit_ns": rs.submit_ns, "launch_ns": rs.launch_ns, "done_ns": rs.done_ns,
                "batch_size": rs.batch_size, "batch_id": rs.batch_id}

    def cancel(self, ticket: int) -> bool:
        """True if the request was still queued and is now cancelled (its
        poll/wait then raise with HAB_ERR_CANCELLED); False if it was
        already launched (it completes)."""
        s = self.lib.hab_server_cancel(self.h, C.c_uint64(ticket))
        if s == B.HAB_ERR_NOT_READY:
            return False
        B.check(s, "hab_server_cancel")
        return True

    def poll(self, ticket: int):
        rs = B.RequestStats()
        s = self.lib.hab_server_poll(self.h, C.c_uint64(ticket), C.byref(rs))
        if s == B.HAB_ERR_NOT_READY:
            return None
        self._keep.pop(ticket, None)
        B.check(s, "hab_server_poll")
        return self._stats(rs)

    def wait(self, ticket: int):
        rs = B.RequestStats()
        s = self.lib.hab_server_wait(self.h, C.c_uint64(ticket), C.byref(rs))
        self._keep.pop(ticket, None)
        B.check(s, "hab_server_wait")
        return self._stats(rs)

    def stats(self):
        st = B.ServerStats()
        B.check(self.lib.hab_server_stats_get(self.h, C.byref(st)), "hab_server_stats_get")
        return {k: getattr(st, k) for k, _ in B.ServerStats._fields_ if k != "pad"}

    def close(self):
        if self.h:
            B.check(self.lib.hab_server_destroy(self.h), "hab_server_destroy")
            self.h = None
            self._keep.clear()
