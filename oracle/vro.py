"""ctypes wrapper of the CPU oracle (oracle/libvro.so).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
benchmark's CPU-baseline leg use it; the GPU product path never does.
Arrays are numpy, host memory, and every call is synchronous.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvro.so")

OK, ERR_ARG, ERR_INDEX_RANGE, ERR_CAPACITY = 0, 1, 2, 3
NAIVE, STATIC_BALLOT, STATIC_SORT, STATIC_HASH, DYN_SORT, DYN_HASH, DYN_PHASH, DYN_BALLOT, MULTI = range(9)
STRATEGY_NAMES = ["naive", "static_ballot", "static_sort", "static_hash", "dyn_sort", "dyn_hash",
                  "dyn_phash", "dyn_ballot", "multi"]
OUT_FLOATS = 12


class Opts(C.Structure):
    _fields_ = [("max_unique", C.c_uint32), ("wg_size", C.c_uint32),
                ("hash_slots", C.c_uint32), ("hash_probes", C.c_uint32)]


class Shader(C.Structure):
    _fields_ = [("kind", C.c_uint32), ("num_lights", C.c_uint32), ("iterations", C.c_uint32),
                ("spec_squarings", C.c_uint32), ("mvp", C.c_float * 16), ("model", C.c_float * 12),
                ("normal", C.c_float * 9), ("eye", C.c_float * 3), ("ambient", C.c_float * 3),
                ("kd", C.c_float), ("ks", C.c_float), ("katt", C.c_float), ("coef", C.c_float * 8),
                ("lights", (C.c_float * 6) * 16)]


class Outputs(C.Structure):
    _fields_ = [("corners", C.c_void_p), ("tris", C.c_void_p), ("verts", C.c_void_p),
                ("verts_cap", C.c_uint64), ("local_idx", C.c_void_p), ("unit_offsets", C.c_void_p),
                ("unit_invocations", C.c_void_p), ("units_cap", C.c_uint64),
                ("counters", C.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build_oracle  # noqa: WPS433
            build_oracle.build()
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.vro_units_bound.argtypes = [C.c_int, C.c_uint64, C.c_uint32]
        L.vro_units_bound.restype = C.c_uint64
        L.vro_check_args.argtypes = [C.c_uint64, C.c_uint32, C.POINTER(Shader), C.c_int, C.c_uint32,
                                     C.POINTER(Opts), C.POINTER(Outputs), C.POINTER(C.c_uint32)]
        L.vro_check_args.restype = C.c_int
        L.vro_plan_dynamic.argtypes = [P, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, P, C.c_uint64]
        L.vro_plan_dynamic.restype = C.c_int64
        L.vro_process_draw.argtypes = [P, C.c_uint64, P, C.c_uint32, C.POINTER(Shader), C.c_int,
                                       C.c_uint32, C.POINTER(Opts), C.POINTER(Outputs)]
        L.vro_process_draw.restype = C.c_int
        L.vro_shade.argtypes = [C.POINTER(Shader), P, P]
        L.vro_shade.restype = None
        L.vro_shade_f64.argtypes = [C.POINTER(Shader), P, P]
        L.vro_shade_f64.restype = None
        L.vro_count_unique.argtypes = [P, C.c_uint64, C.c_uint32]
        L.vro_count_unique.restype = C.c_int64
        L.vro_fifo_misses.argtypes = [P, C.c_uint64, C.c_uint32, C.c_uint32]
        L.vro_fifo_misses.restype = C.c_int64
        L.vro_parallel_cache_hits.argtypes = [P, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, C.c_int]
        L.vro_parallel_cache_hits.restype = C.c_int64
        L.vro_walk_step.argtypes = [P, C.c_uint32, P, C.c_uint32, P, P, C.c_uint32, P, C.c_int, C.c_uint32, P, P]
        L.vro_walk_step.restype = C.c_int
        L.vro_setup.argtypes = [P, C.c_uint64, C.c_uint32, C.c_uint32, P]
        L.vro_setup.restype = C.c_uint64
        L.vro_walk_options.argtypes = [C.c_uint32, C.c_uint32, P, C.c_uint32, P, P, C.c_uint32, P, P]
        L.vro_walk_options.restype = C.c_uint32
        L.vro_walk_choose.argtypes = [C.c_uint32, C.c_float, P, P, C.c_uint32, P]
        L.vro_walk_choose.restype = C.c_uint32
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def make_shader(sp) -> Shader:
    """Marshal a workloads.ShaderParams (or any object with the same fields)."""
    s = Shader()
    s.kind, s.num_lights, s.iterations, s.spec_squarings = (int(sp.kind), int(sp.num_lights),
                                                             int(sp.iterations), int(sp.spec_squarings))
    for name, n in (("mvp", 16), ("model", 12), ("normal", 9), ("eye", 3), ("ambient", 3), ("coef", 8)):
        arr = np.asarray(getattr(sp, name), dtype=np.float32).ravel()
        assert arr.size == n, name
        C.memmove(C.addressof(getattr(s, name)), arr.ctypes.data, 4 * n)
    s.kd, s.ks, s.katt = float(np.float32(sp.kd)), float(np.float32(sp.ks)), float(np.float32(sp.katt))
    lights = np.ascontiguousarray(np.asarray(sp.lights, dtype=np.float32).reshape(16, 6))
    C.memmove(C.addressof(s.lights), lights.ctypes.data, 4 * 96)
    return s


def make_opts(max_unique=0, wg_size=0, hash_slots=0, hash_probes=0) -> Opts:
    return Opts(max_unique, wg_size, hash_slots, hash_probes)


def units_bound(strategy, num_tris, batch_tris):
    return int(lib().vro_units_bound(strategy, num_tris, batch_tris))


def process_draw(indices, vertices, shader, strategy, batch_tris, opts=None, *,
                 corners=True, tris=True, verts=True, local_idx=True, units=True):
    """Run one draw; returns (status, dict of outputs)."""
    indices = np.ascontiguousarray(indices, dtype=np.uint32)
    vertices = np.ascontiguousarray(vertices, dtype=np.float32)
    n = len(indices)
    T = n // 3
    V = vertices.shape[0] if vertices.ndim == 2 else len(vertices) // 8
    res = {}
    if corners:
        res["corners"] = np.zeros((n, OUT_FLOATS), dtype=np.float32)
    if tris:
        res["tris"] = np.zeros(n, dtype=np.uint32)
    vcap = max(n, V) if strategy == MULTI else n
    if verts:
        res["verts"] = np.zeros((max(vcap, 1), OUT_FLOATS), dtype=np.float32)
    if local_idx and strategy == MULTI:
        local_idx = False   # not defined for the single vertex-buffer unit
    if local_idx:
        res["local_idx"] = np.zeros(n, dtype=np.uint16)
    ucap = units_bound(strategy, T, batch_tris) if batch_tris else T
    if units:
        res["unit_offsets"] = np.zeros(ucap + 1, dtype=np.uint32)
        res["unit_invocations"] = np.zeros(max(ucap, 1), dtype=np.uint32)
    res["counters"] = np.zeros(4, dtype=np.uint64)
    out = Outputs(_ptr(res.get("corners")), _ptr(res.get("tris")), _ptr(res.get("verts")),
                  vcap if verts else 0, _ptr(res.get("local_idx")), _ptr(res.get("unit_offsets")),
                  _ptr(res.get("unit_invocations")), ucap if units else 0, _ptr(res["counters"]))
    sh = shader if isinstance(shader, Shader) else make_shader(shader)
    op = opts if (opts is None or isinstance(opts, Opts)) else make_opts(**opts)
    rc = lib().vro_process_draw(_ptr(indices), n, _ptr(vertices), V, C.byref(sh), strategy, batch_tris,
                                C.byref(op) if op is not None else None, C.byref(out))
    if rc == OK:
        inv, nunits = int(res["counters"][0]), int(res["counters"][1])
        if verts:
            res["verts"] = res["verts"][:inv]
        if units:
            res["unit_offsets"] = res["unit_offsets"][:nunits + 1]
            res["unit_invocations"] = res["unit_invocations"][:nunits]
    return rc, res


def plan_dynamic(indices, num_vertices, max_unique, max_tris):
    indices = np.ascontiguousarray(indices, dtype=np.uint32)
    T = len(indices) // 3
    offs = np.zeros(T + 1, dtype=np.uint32)
    B = lib().vro_plan_dynamic(_ptr(indices), T, num_vertices, max_unique, max_tris, _ptr(offs), T + 1)
    if B < 0:
        return None
    return offs[:B + 1]


def shade(shader, vin, f64=False):
    """Shade an array of input vertices [n, 8] one at a time."""
    vin = np.ascontiguousarray(vin, dtype=np.float32).reshape(-1, 8)
    sh = shader if isinstance(shader, Shader) else make_shader(shader)
    out = np.zeros((len(vin), OUT_FLOATS), dtype=np.float64 if f64 else np.float32)
    fn = lib().vro_shade_f64 if f64 else lib().vro_shade
    for i in range(len(vin)):
        fn(C.byref(sh), vin[i].ctypes.data, out[i].ctypes.data)
    return out


def count_unique(indices, num_vertices):
    indices = np.ascontiguousarray(indices, dtype=np.uint32)
    return int(lib().vro_count_unique(_ptr(indices), len(indices), num_vertices))


def parallel_cache_hits(indices, num_vertices, procs, per_cycle, entries, contiguous=True):
    """Hits of parallel per-processor LRU caches (Section 4.1, Table 1)."""
    indices = np.ascontiguousarray(indices, dtype=np.uint32)
    return int(lib().vro_parallel_cache_hits(_ptr(indices), len(indices), num_vertices, procs, per_cycle, entries,
                                             1 if contiguous else 0))


def setup(corners, width, height):
    """Triangle setup of assembled corners [3T, 12]: (records float32[T, 8],
    visible count); records[:, 5] holds the uint32 flags."""
    corners = np.ascontiguousarray(corners, dtype=np.float32)
    T = len(corners) // 3
    rec = np.zeros((T, 8), np.float32)
    vis = int(lib().vro_setup(_ptr(corners), T, width, height, _ptr(rec)))
    return rec, vis


def walk_step(keys, setup, uniforms, strategy, batch=0):
    """One random-walk step (Section 5); returns (status, new keys, counters)."""
    keys = np.ascontiguousarray(keys, dtype=np.uint32)
    out = np.zeros_like(keys)
    cnt = np.zeros(4, dtype=np.uint64)
    act = np.ascontiguousarray(setup.activity, dtype=np.float32)
    mv = np.ascontiguousarray(setup.moves, dtype=np.int8)
    w = np.ascontiguousarray(setup.weights, dtype=np.float32)
    u = np.ascontiguousarray(uniforms, dtype=np.float32)
    rc = lib().vro_walk_step(_ptr(keys), len(keys), _ptr(act), setup.grid, _ptr(mv), _ptr(w), len(w), _ptr(u),
                             strategy, batch, _ptr(out), _ptr(cnt))
    return rc, out, cnt


def walk_options(x, y, setup):
    """A cell's kept options: (likelihoods float32[k], move indices[k])."""
    L = np.zeros(8, np.float32)
    mi = np.zeros(8, np.uint32)
    act = np.ascontiguousarray(setup.activity, dtype=np.float32)
    mv = np.ascontiguousarray(setup.moves, dtype=np.int8)
    w = np.ascontiguousarray(setup.weights, dtype=np.float32)
    k = lib().vro_walk_options(x, y, _ptr(act), setup.grid, _ptr(mv), _ptr(w), len(w), _ptr(L), _ptr(mi))
    return L[:k], mi[:k]


def walk_choose(key, u, L, mi, moves):
    L = np.ascontiguousarray(L, dtype=np.float32)
    mi = np.ascontiguousarray(mi, dtype=np.uint32)
    mv = np.ascontiguousarray(moves, dtype=np.int8)
    return int(lib().vro_walk_choose(key, float(u), _ptr(L), _ptr(mi), len(L), _ptr(mv)))


def fifo_misses(indices, num_vertices, k):
    indices = np.ascontiguousarray(indices, dtype=np.uint32)
    return int(lib().vro_fifo_misses(_ptr(indices), len(indices), num_vertices, k))
