"""Request loop around the libvr.so server (vr_server_* in include/vr.h).

The server itself (admission against the memory budget, continuous batching
into persistent frame launches, completion tracking) is native code; this
module only registers resident meshes, submits a timed request stream and
collects completions, as a client would.
"""
from __future__ import annotations

import time

import numpy as np

from . import vr


class Server:
    """Owns a vr_server and the device tensors of its meshes."""

    def __init__(self, budget_bytes, max_inflight=2, max_tick_draws=1024, max_tick_tris=0, device=0):
        self.cfg = vr.make_server_config(budget_bytes, max_inflight, max_tick_draws, max_tick_tris)
        self.h = vr.vr_server_create(device, self.cfg)
        self.keep = []

    def close(self):
        if self.h is not None:
            vr.vr_server_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def check(self, st):
        if st != vr.VR_OK:
            raise vr.VrError(st, vr.vr_server_last_error(self.h))

    def add_mesh(self, indices, vertices):
        st, m = vr.vr_server_add_mesh(self.h, indices, vertices)
        self.check(st)
        self.keep.append((indices, vertices))
        return m

    def submit(self, request):
        st, t = vr.vr_server_submit(self.h, request)
        self.check(st)
        return t

    def submit_many(self, requests):
        """Queues all requests under one lock (the scheduler sees them together)."""
        st, tickets = vr.vr_server_submit_many(self.h, requests)
        self.check(st)
        return tickets

    def poll(self, cap=256, timeout_ms=0):
        st, out = vr.vr_server_poll(self.h, cap, timeout_ms)
        self.check(st)
        return out

    def fetch(self, ticket, num_tris):
        st, arr = vr.vr_server_fetch(self.h, ticket, num_tris)
        self.check(st)
        return arr

    def release(self, ticket):
        self.check(vr.vr_server_release(self.h, ticket))

    def stats(self):
        st, s = vr.vr_server_stats_get(self.h)
        self.check(st)
        return s

    def drain(self, n, timeout_s=60.0, release=True):
        """Collects n completions (releasing each unless told otherwise)."""
        got = []
        t_end = time.perf_counter() + timeout_s
        while len(got) < n:
            if time.perf_counter() > t_end:
                raise TimeoutError(f"{len(got)} of {n} requests finished")
            for c in self.poll(timeout_ms=50):
                got.append(c)
                if release:
                    self.release(c["ticket"])
        return got


def replay(server: Server, requests, arrivals, timeout_s=120.0, rejected=None):
    """Submits requests[i] at arrivals[i] seconds after the start (a Poisson
    stream), releasing results as they finish.  Returns (completions,
    submit lateness in seconds, wall seconds).  With a list for `rejected`,
    requests the budget can never hold are recorded there by index instead
    of raising."""
    n = len(requests)
    got, late = [], np.zeros(n)
    t0 = time.perf_counter()
    i = 0
    expect = n
    while len(got) < expect:
        now = time.perf_counter() - t0
        if now > timeout_s:
            raise TimeoutError(f"{len(got)} of {expect} requests finished")
        while i < n and arrivals[i] <= now:
            st, _ = vr.vr_server_submit(server.h, requests[i])
            if st == vr.VR_ERR_CAPACITY and rejected is not None:
                rejected.append(i)
                expect -= 1
            else:
                server.check(st)
            late[i] = now - arrivals[i]
            i += 1
            now = time.perf_counter() - t0
        for c in server.poll(timeout_ms=0):
            got.append(c)
            server.release(c["ticket"])
        if i < n:
            gap = arrivals[i] - (time.perf_counter() - t0)
            if gap > 2e-4:
                time.sleep(min(gap - 1e-4, 1e-3))
        else:
            time.sleep(5e-5)
    return got, late, time.perf_counter() - t0


def summarize(completions, wall_s):
    """Latency (finish - submit) percentiles in ms and throughput."""
    lat = np.array([c["t_done"] - c["t_submit"] for c in completions]) * 1e3
    queue = np.array([c["t_launch"] - c["t_submit"] for c in completions]) * 1e3
    tris = sum(c["num_tris"] for c in completions)
    ticks = len({c["tick"] for c in completions})
    return {"requests": len(completions), "triangles": int(tris), "wall_s": wall_s,
            "tri_per_s": tris / wall_s if wall_s > 0 else 0.0, "req_per_s": len(completions) / wall_s,
            "latency_ms_p50": float(np.percentile(lat, 50)), "latency_ms_p99": float(np.percentile(lat, 99)),
            "latency_ms_mean": float(lat.mean()), "queue_ms_p99": float(np.percentile(queue, 99)),
            "ticks": ticks, "requests_per_tick": len(completions) / max(1, ticks),
            "errors": int(sum(1 for c in completions if c["status"] != vr.VR_OK))}
