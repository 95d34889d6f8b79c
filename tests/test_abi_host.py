"""Host-only checks of the C ABI (no GPU needed): the built library loads,
exports every function include/hab.h declares, validates sensor requests
and reports status strings."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_1904_01201_amd as P
from paper_1904_01201_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "hab.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:hab_status|const char \*)\s*(hab_\w+)\s*\(", src, re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(P.lib_path()):
        pytest.fail("libhabmi.so is not built (run __graft_entry__.build())")
    return B.load()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(B.EXPORTED) == set(names)


def test_status_strings(lib):
    for s in range(7):
        assert lib.hab_status_string(s)
    assert lib.hab_status_string(99) == b"unknown status"


def spec(w, h, hfov=90.0, near=0.0, outputs=0, noise=0.0):
    d = B.SensorDesc(w, h, hfov, near, outputs, noise)
    s = B.Sensor()
    rc = B.load().hab_sensor_spec(C.byref(d), C.byref(s))
    return rc, s


def test_sensor_spec_paper_defaults(lib):
    """256^2 at 90 degrees: f = 128 exactly; defaults near 0.01 and RGB+D."""
    rc, s = spec(256, 256)
    assert rc == B.HAB_OK
    assert s.f == 128.0 and abs(s.near_m - 0.01) < 1e-9 and s.outputs == 3


@pytest.mark.parametrize("args", [(0, 16), (16, 0), (4097, 16), (16, 16, 0.0), (16, 16, 180.0),
                                  (16, 16, 90.0, -1.0), (16, 16, 90.0, 0.0, 16),
                                  (16, 16, float("nan")), (16, 16, 90.0, 0.0, 3, -0.1),
                                  (16, 16, 90.0, 0.0, 3, float("nan")),
                                  (16, 16, 90.0, 0.0, 3, float("inf"))])
def test_sensor_spec_rejects(lib, args):
    rc, _ = spec(*args)
    assert rc == B.HAB_ERR_INVALID_ARG


def test_sensor_spec_semantic(lib):
    """The semantic output bit (8) is accepted alone or with the others."""
    for outputs in (B.OUT_SEMANTIC, B.OUT_RGB | B.OUT_DEPTH | B.OUT_SEMANTIC, 15):
        rc, s = spec(64, 48, 90.0, 0.01, outputs)
        assert rc == B.HAB_OK and s.outputs == outputs


def test_sensor_spec_depth_noise(lib):
    """The noise sigma is carried through unchanged (0 = ideal depth)."""
    rc, s = spec(64, 48, 90.0, 0.01, 3, 0.4)
    assert rc == B.HAB_OK and s.depth_noise_sigma == np.float32(0.4)
    rc, s = spec(64, 48)
    assert rc == B.HAB_OK and s.depth_noise_sigma == 0.0


def test_null_arguments(lib):
    assert lib.hab_init(0, None) == B.HAB_ERR_INVALID_ARG
    assert lib.hab_shutdown(None) == B.HAB_ERR_INVALID_ARG
    assert lib.hab_get_error(None) == B.HAB_ERR_INVALID_ARG
    assert lib.hab_render(None, None, None, None, 0, None, None, None) == B.HAB_ERR_INVALID_ARG
    assert lib.hab_render_batch(None, None, 0, None, None) == B.HAB_ERR_INVALID_ARG
    assert lib.hab_render_noalloc(None, None, None, None, 0, None, None, None) == B.HAB_ERR_INVALID_ARG
    assert lib.hab_stepper_step(None, None, None) == B.HAB_ERR_INVALID_ARG
    assert lib.hab_profile_phases(None, 1) == B.HAB_ERR_INVALID_ARG
    assert lib.hab_stepper_step_device(None, None, None) == B.HAB_ERR_INVALID_ARG
    assert lib.hab_nav_upload(None, None, 0, None) == B.HAB_ERR_INVALID_ARG
    assert lib.hab_nav_release(None, None) == B.HAB_ERR_INVALID_ARG
    p = B.Actuation(0.1, 0.25, 1.0, 0.0)
    assert lib.hab_actuate(None, None, 0, None, None, None, None, 1.5, C.byref(p), None) == B.HAB_ERR_INVALID_ARG
    assert lib.hab_server_submit(None, None, None) == B.HAB_ERR_INVALID_ARG
    n = C.c_uint64()
    assert lib.hab_selfcheck_reciprocal(None, 0x00800000, 0x7E800000, None, C.byref(n)) == B.HAB_ERR_INVALID_ARG


def test_output_tensor_checks():
    """The binding refuses output buffers of the wrong size before calling
    into the library (a short buffer would be written out of bounds)."""
    torch = pytest.importorskip("torch")
    from paper_1904_01201_amd.renderer import check_output
    s = B.Sensor(8, 4, 3, 90.0, 4.0, 0.01)
    with pytest.raises(ValueError):
        check_output("depth", torch.empty(31), 1, s)      # CPU tensor / wrong size


def test_set_poses_writes_each_record():
    """Context.set_poses writes pose k into View record k and nothing else."""
    n = 5
    views = (B.View * n)()
    for k in range(n):
        views[k].noise_seed = 1000 + k
    poses = np.arange(12 * n, dtype=np.float32).reshape(n, 12) * 0.5
    P.Context.set_poses(views, poses)
    for k in range(n):
        assert list(views[k].pose.position) == list(poses[k, :3])
        assert list(views[k].pose.rotation) == list(poses[k, 3:])
        assert views[k].noise_seed == 1000 + k and not views[k].scene
    with pytest.raises(ValueError):
        P.Context.set_poses(views, poses[:4])

