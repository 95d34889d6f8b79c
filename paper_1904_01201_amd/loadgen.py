"""Open-loop load generator for the serving loop (Server).

Agents submit single-view step requests (fixed scene and sensor per agent,
poses from the agent's own random walk).  Arrivals are Poisson at a total
rate lambda split evenly over the agents; an agent has at most one request
in flight, so an arrival that falls while its previous request is still
being served waits for that completion.  Two latencies are kept: the
server's own submit -> completion stamp, and arrival -> completion (which
adds the wait for the agent's previous request).  `saturate()` measures
the closed-loop throughput (every agent of the first `num` resubmits on
completion) that the open-loop sweep is scaled by.  Arrival times are
CLOCK_MONOTONIC, the clock of the server's stamps.
"""
from __future__ import annotations

import collections
import ctypes as C
import heapq
import time

import numpy as np

from . import binding as B


class Agents:
    def __init__(self, ctx, scenes, scene_of, sensors, poses, device="cuda"):
        """scenes: SceneHandles; scene_of[a]: scene index; sensors[a]: Sensor;
        poses: [steps, agents, 12]."""
        self.ctx = ctx
        self.n = len(scene_of)
        self.poses = np.ascontiguousarray(poses, np.float32)
        self.views = []
        self.outs = []
        for a in range(self.n):
            sn = sensors[a]
            out = ctx.alloc(sn, 1)
            v = B.View()
            v.scene = scenes[scene_of[a]].ptr
            v.sensor = C.pointer(sn)
            v.out_rgb = int(out["rgb"].data_ptr()) if "rgb" in out else None
            v.out_depth = int(out["depth"].data_ptr()) if "depth" in out else None
            v.out_tri = None
            v.out_semantic = int(out["semantic"].data_ptr()) if "semantic" in out else None
            self.views.append(v)
            self.outs.append((sn, out))
        self.step = np.zeros(self.n, np.int64)

    def submit(self, srv, a):
        v = self.views[a]
        p = self.poses[self.step[a] % self.poses.shape[0], a]
        C.memmove(C.byref(v, B.View.pose.offset), p.ctypes.data, 48)
        self.step[a] += 1
        t = C.c_uint64()
        B.check(srv.lib.hab_server_submit(srv.h, C.byref(v), C.byref(t)), "submit")
        return t.value


def _drain(srv, inflight, done_cb, limit=64):
    """Poll up to `limit` in-flight tickets (oldest first)."""
    rs = B.RequestStats()
    finished = []
    for t in list(inflight.keys())[:limit]:
        s = srv.lib.hab_server_poll(srv.h, C.c_uint64(t), C.byref(rs))
        if s == B.HAB_ERR_NOT_READY:
            continue
        B.check(s, "poll")
        finished.append(t)
        done_cb(inflight.pop(t), rs.submit_ns, rs.done_ns, rs.batch_size)
    return finished


def saturate(srv, agents: Agents, seconds=1.0, num=None):
    """Closed loop: each of the first `num` agents keeps one request in
    flight.  Returns requests/s and submit -> completion latencies (ms)."""
    inflight = {}
    lat = []
    for a in range(agents.n if num is None else min(num, agents.n)):
        inflight[agents.submit(srv, a)] = a
    t0 = time.perf_counter()
    done = 0

    def cb(a, s_ns, d_ns, bs):
        nonlocal done
        done += 1
        lat.append((d_ns - s_ns) * 1e-6)
        if time.perf_counter() - t0 < seconds:
            inflight[agents.submit(srv, a)] = a

    while inflight:
        _drain(srv, inflight, cb, limit=len(inflight))
    el = time.perf_counter() - t0
    return done / el, np.array(lat)


def open_loop(srv, agents: Agents, rate, seconds=1.0, seed=0):
    """Poisson arrivals at `rate` requests/s in total over `seconds`.
    Returns the throughput (requests completed inside the window per
    second), submit -> completion and arrival -> completion latencies (ms)
    of every request that arrived inside the window (those still waiting
    when it ends are served and counted), and the batch size each request
    rode in."""
    rng = np.random.default_rng(seed)
    per = rate / agents.n
    heap = [(float(rng.exponential(1.0 / per)), a) for a in range(agents.n)]
    heapq.heapify(heap)
    busy = np.zeros(agents.n, bool)
    backlog = [collections.deque() for _ in range(agents.n)]   # arrivals while busy
    nback = 0
    inflight = {}
    lat, e2e, bsz = [], [], []
    t0 = time.monotonic()
    t0_ns = int(t0 * 1e9)
    end_ns = t0_ns + int(seconds * 1e9)
    done = 0

    def cb(item, s_ns, d_ns, bs):
        nonlocal done, nback
        a, ta = item
        done += d_ns <= end_ns
        lat.append((d_ns - s_ns) * 1e-6)
        e2e.append((d_ns - t0_ns) * 1e-6 - ta * 1e3)
        bsz.append(bs)
        if backlog[a]:
            nback -= 1
            inflight[agents.submit(srv, a)] = (a, backlog[a].popleft())
        else:
            busy[a] = False

    while True:
        now = time.monotonic() - t0
        if now >= seconds and not inflight and not nback:
            break
        while heap and heap[0][0] <= now and now < seconds:
            ta, a = heapq.heappop(heap)
            if busy[a]:
                backlog[a].append(ta)
                nback += 1
            else:
                inflight[agents.submit(srv, a)] = (a, ta)
                busy[a] = True
            heapq.heappush(heap, (ta + float(rng.exponential(1.0 / per)), a))
        if inflight:
            _drain(srv, inflight, cb)
    return done / seconds, np.array(lat), np.array(e2e), np.array(bsz)
