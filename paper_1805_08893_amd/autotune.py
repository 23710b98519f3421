"""Per-mesh-class choice of strategy, batch size and unique budget.

The paper reports the best batch configuration per application after a
search (Sections 4.2 and 5).  Here the search is automated: a draw is put in
a mesh class (size bucket, shader cost bucket, index-locality bucket), and
the first draw of each class is timed through vr_autotune (libvr.so) over
a candidate list; the winner is kept for the class and can be persisted as
JSON.  The search measures throughput, the quantity that counts once draws
share a persistent launch: a draw smaller than `min_tris` is timed as its
index buffer repeated until it reaches that size (same vertices, same
locality), so launch latency does not decide the choice.  The choice changes how a draw is batched, never what a given
configuration computes: every candidate is a configuration the oracle
parity tests cover.
"""
from __future__ import annotations

import ctypes as C
import json
import math
import os

import numpy as np

from . import vr

DEFAULT_CANDIDATES = [
    (vr.VR_NAIVE, 1, 0),
    (vr.VR_STATIC_BALLOT, 64, 0), (vr.VR_STATIC_BALLOT, 128, 0),
    (vr.VR_STATIC_HASH, 64, 0), (vr.VR_STATIC_HASH, 128, 0), (vr.VR_STATIC_SORT, 64, 0),
    (vr.VR_DYN_HASH, 64, 64), (vr.VR_DYN_HASH, 128, 128), (vr.VR_DYN_HASH, 256, 256), (vr.VR_DYN_HASH, 341, 256),
    (vr.VR_DYN_PHASH, 256, 256), (vr.VR_DYN_PHASH, 341, 256), (vr.VR_DYN_SORT, 256, 256),
    (vr.VR_DYN_BALLOT, 85, 64),
]


class vr_tune_candidate(C.Structure):
    _fields_ = [("strategy", C.c_int), ("batch_tris", C.c_uint32), ("max_unique", C.c_uint32),
                ("wg_size", C.c_uint32), ("kernel_ms", C.c_float), ("plan_ms", C.c_float),
                ("invocations", C.c_uint64)]


def _lib():
    L = vr.lib()
    if not getattr(L, "_tune_bound", False):
        L.vr_autotune.argtypes = [C.c_void_p, C.c_void_p, C.c_uint64, C.c_void_p, C.c_uint32,
                                  C.POINTER(vr.vr_shader_params), C.POINTER(vr_tune_candidate), C.c_uint32,
                                  C.c_uint32, C.POINTER(C.c_uint32)]
        L.vr_autotune.restype = C.c_int
        L._tune_bound = True
    return L


def vr_autotune(ctx, indices, vertices, shader, candidates=DEFAULT_CANDIDATES, reps=5):
    """Times every candidate on this draw; returns (best index, list of dicts)."""
    sh = shader if isinstance(shader, vr.vr_shader_params) else vr.make_shader(shader)
    arr = (vr_tune_candidate * len(candidates))(*[vr_tune_candidate(s, bt, nu, 0, 0.0, 0.0, 0)
                                                  for s, bt, nu in candidates])
    best = C.c_uint32(0)
    V = vertices.shape[0] if vertices.dim() == 2 else vertices.numel() // 8
    st = _lib().vr_autotune(ctx, indices.data_ptr(), indices.numel(), vertices.data_ptr(), V, C.byref(sh), arr,
                            len(candidates), reps, C.byref(best))
    if st != vr.VR_OK:
        raise vr.VrError(st, vr.vr_last_error(ctx))
    rows = [dict(strategy=a.strategy, batch_tris=a.batch_tris, max_unique=a.max_unique, kernel_ms=a.kernel_ms,
                 plan_ms=a.plan_ms, invocations=int(a.invocations)) for a in arr]
    return int(best.value), rows


def shader_flops(sp):
    mvp = 49
    if sp.kind == 1:
        return mvp + 31 + 48 * sp.num_lights
    if sp.kind == 2:
        return mvp + 11 + 9 * sp.iterations
    return mvp


def locality(indices_host: np.ndarray, windows=16, window_tris=256) -> float:
    """Mean fraction of distinct indices in a few windows of 256 triangles
    (0.33 for a perfectly strip-like order, 1.0 when nothing repeats)."""
    T = len(indices_host) // 3
    if T == 0:
        return 1.0
    w = min(window_tris, T)
    starts = np.linspace(0, T - w, num=min(windows, max(1, T // w)), dtype=np.int64)
    fr = [len(np.unique(indices_host[3 * s:3 * (s + w)])) / (3.0 * w) for s in starts]
    return float(np.mean(fr))


def mesh_class(num_tris: int, sp, loc: float) -> str:
    size = min(5, max(0, int(math.log2(max(1, num_tris)) // 3) - 2))   # buckets of 8x
    cost = 0 if shader_flops(sp) < 100 else 1 if shader_flops(sp) < 400 else 2 if shader_flops(sp) < 900 else 3
    order = 0 if loc < 0.45 else 1 if loc < 0.7 else 2
    return f"s{size}-c{cost}-o{order}"


class Autotuner:
    """Chooses a configuration per mesh class, timing the first draw of each
    class; `table` maps class -> {strategy, batch_tris, max_unique, ...}."""

    def __init__(self, ctx, candidates=DEFAULT_CANDIDATES, path=None, sample_tris=1 << 20, min_tris=1 << 20):
        self.ctx = ctx
        self.candidates = candidates
        self.path = path
        self.sample_tris = sample_tris
        self.min_tris = min(min_tris, sample_tris)
        self.table = {}
        if path and os.path.exists(path):
            with open(path) as f:
                self.table = json.load(f)

    def choose(self, indices_dev, indices_host, vertices, shader):
        T = indices_dev.numel() // 3
        key = mesh_class(T, shader, locality(indices_host))
        if key not in self.table and T > 0:
            sample = indices_dev[:3 * min(T, self.sample_tris)]
            if T < self.min_tris:
                sample = sample.repeat((self.min_tris + T - 1) // T)
            best, rows = vr_autotune(self.ctx, sample, vertices, shader, self.candidates)
            self.table[key] = dict(rows[best], key=key, sample_tris=sample.numel() // 3,
                                   candidates=[{k: r[k] for k in ("strategy", "batch_tris", "max_unique",
                                                                  "kernel_ms", "plan_ms")} for r in rows])
        if key not in self.table:
            return key, (vr.VR_NAIVE, 1, 0)
        e = self.table[key]
        return key, (e["strategy"], e["batch_tris"], e["max_unique"])

    def save(self, path=None):
        path = path or self.path
        if path:
            with open(path, "w") as f:
                json.dump(self.table, f, indent=1)
