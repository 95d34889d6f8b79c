"""Persistent autotune table (HABMI_AUTOTUNE_CACHE): hab_autotune writes
the context's choices, a new context loads those saved for its GPU
architecture and uses them, and a file for another architecture or with
malformed lines changes nothing.  The choice never changes an output."""
import json
import os

import pytest

from scenegen import configs
from tests.gpu_common import gpu_ctx, note

pytestmark = pytest.mark.gpu


def _items(c, w, out, sn, hs):
    return [(hs[w.env_scene[e]], sn, w.poses[0, e], out["rgb"][e], out["depth"][e], None)
            for e in range(w.num_envs)]


def _raster_phases(c, items):
    c.profile(True)
    c.render_batch(items)
    c.profile(False)
    return sorted(k for k in c.profile_read() if k.startswith("raster"))


def test_autotune_table_persists(tmp_path, monkeypatch):
    import torch
    path = str(tmp_path / "tune.json")
    monkeypatch.setenv("HABMI_AUTOTUNE_CACHE", path)
    w = configs.batch64_4scenes_256(steps=1, scene_T=(20_000, 40_000))
    note("autotune cache: tune and save")
    c1 = gpu_ctx()
    try:
        hs = [c1.upload_scene(s) for s in w.scenes]
        sn = c1.sensor(256, 256)
        out = c1.alloc(sn, w.num_envs)
        ts, bf = c1.autotune(_items(c1, w, out, sn, hs))
    finally:
        c1.close()
    doc = json.load(open(path))
    assert doc["arch"].startswith("gfx")
    classes = {e["class"]: (e["tile"], e["bin_factor"]) for e in doc["entries"]}
    assert len(classes) >= 1 and (ts, bf) in classes.values()
    # force a distinguishable choice (32-pixel tiles) for every class
    for e in doc["entries"]:
        e["tile"] = 32
    with open(path, "w") as f:
        f.write('{"arch": "%s", "entries": [\n' % doc["arch"])
        f.write(",\n".join('  {"class": %d, "tile": %d, "bin_factor": %g}' % (e["class"], e["tile"], e["bin_factor"])
                           for e in doc["entries"]))
        f.write("\n]}\n")
    note("autotune cache: load in a new context")
    c2 = gpu_ctx()
    try:
        hs = [c2.upload_scene(s) for s in w.scenes]
        sn = c2.sensor(256, 256)
        out = c2.alloc(sn, w.num_envs)
        assert _raster_phases(c2, _items(c2, w, out, sn, hs)) == ["raster32"]
        ref = c2.alloc(sn, w.num_envs)
        c2.render_batch(_items(c2, w, ref, sn, hs), tile_size=16)
        torch.cuda.synchronize()
        for k in out:
            assert torch.equal(out[k], ref[k]), k
    finally:
        c2.close()
    # another architecture's table, and garbage, are ignored
    with open(path, "w") as f:
        f.write('{"arch": "gfx000", "entries": [\n')
        f.write(",\n".join('  {"class": %d, "tile": 8, "bin_factor": 1}' % k for k in classes))
        f.write("\n]}\n")
    for text in (None, '{"arch": "%s", "entries": [\n  {"class": "x", "tile": 8}\n]}\n' % doc["arch"]):
        if text is not None:
            with open(path, "w") as f:
                f.write(text)
        c3 = gpu_ctx()
        try:
            hs = [c3.upload_scene(s) for s in w.scenes]
            sn = c3.sensor(256, 256)
            out = c3.alloc(sn, w.num_envs)
            assert _raster_phases(c3, _items(c3, w, out, sn, hs)) == ["raster16"]
        finally:
            c3.close()
