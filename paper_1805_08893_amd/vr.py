"""Python binding of libvr.so (the C ABI in include/vr.h).

Argument marshalling only: every step of the geometry stage runs in the
HIP kernels of libvr.so.  The functions keep the C names; tensors are
torch CUDA (HIP) tensors whose data pointers are handed to the library.
If libvr.so is missing this module raises on first use; there is no
fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvr.so")

(VR_OK, VR_ERR_ARG, VR_ERR_INDEX_RANGE, VR_ERR_CAPACITY, VR_ERR_OOM, VR_ERR_DEVICE, VR_ERR_BUSY,
 VR_CANCELLED) = range(8)
(VR_NAIVE, VR_STATIC_BALLOT, VR_STATIC_SORT, VR_STATIC_HASH, VR_DYN_SORT, VR_DYN_HASH, VR_DYN_PHASH,
 VR_DYN_BALLOT, VR_MULTI) = range(9)
STRATEGIES = {"naive": VR_NAIVE, "static_ballot": VR_STATIC_BALLOT, "static_sort": VR_STATIC_SORT,
              "static_hash": VR_STATIC_HASH, "dyn_sort": VR_DYN_SORT, "dyn_hash": VR_DYN_HASH,
              "dyn_phash": VR_DYN_PHASH, "dyn_ballot": VR_DYN_BALLOT, "multi": VR_MULTI}
STRATEGY_NAMES = {v: k for k, v in STRATEGIES.items()}
DYNAMIC = (VR_DYN_SORT, VR_DYN_HASH, VR_DYN_PHASH, VR_DYN_BALLOT)
OUT_FLOATS = 12
# limits of include/vr.h
VR_MAX_BATCH_STATIC, VR_MAX_BATCH_BALLOT, VR_MAX_BATCH_DYNAMIC, VR_MAX_UNIQUE = 256, 1024, 4096, 4096
VR_MAX_HASH_SLOTS = 8192

EXPORTS = ["vr_create", "vr_destroy", "vr_set_stream", "vr_check_args", "vr_plan_dynamic", "vr_process_draw",
           "vr_process_draw_noalloc",
           "vr_sync", "vr_walk_step", "vr_stream_create", "vr_stream_push", "vr_stream_finish",
           "vr_stream_destroy", "vr_frame_create", "vr_frame_run", "vr_frame_destroy", "vr_process_draws", "vr_autotune",
           "vr_set_kernel_timing", "vr_kernel_times", "vr_math_selftest", "vr_last_error", "vr_server_create", "vr_server_add_mesh",
           "vr_server_submit", "vr_server_submit_many", "vr_server_poll", "vr_server_release", "vr_server_fetch", "vr_server_cancel", "vr_server_stats_get",
           "vr_server_destroy", "vr_server_last_error", "vr_server_simulate"]


class vr_opts(C.Structure):
    _fields_ = [("max_unique", C.c_uint32), ("wg_size", C.c_uint32), ("hash_slots", C.c_uint32),
                ("hash_probes", C.c_uint32), ("d_plan", C.c_void_p)]


class vr_shader_params(C.Structure):
    _fields_ = [("kind", C.c_uint32), ("num_lights", C.c_uint32), ("iterations", C.c_uint32),
                ("spec_squarings", C.c_uint32), ("mvp", C.c_float * 16), ("model", C.c_float * 12),
                ("normal", C.c_float * 9), ("eye", C.c_float * 3), ("ambient", C.c_float * 3),
                ("kd", C.c_float), ("ks", C.c_float), ("katt", C.c_float), ("coef", C.c_float * 8),
                ("lights", (C.c_float * 6) * 16)]


class vr_outputs(C.Structure):
    _fields_ = [("corners", C.c_void_p), ("tris", C.c_void_p), ("verts", C.c_void_p),
                ("verts_cap", C.c_uint64), ("local_idx", C.c_void_p), ("unit_offsets", C.c_void_p),
                ("unit_invocations", C.c_void_p), ("units_cap", C.c_uint64), ("counters", C.c_void_p)]


class vr_draw(C.Structure):
    _fields_ = [("d_indices", C.c_void_p), ("num_indices", C.c_uint64), ("d_vertices", C.c_void_p),
                ("num_vertices", C.c_uint32), ("shader", C.c_uint32), ("strategy", C.c_int),
                ("batch_tris", C.c_uint32), ("max_unique", C.c_uint32), ("d_plan", C.c_void_p),
                ("d_corners", C.c_void_p), ("d_counters", C.c_void_p)]


class vr_server_config(C.Structure):
    _fields_ = [("budget_bytes", C.c_uint64), ("max_inflight", C.c_uint32), ("max_tick_draws", C.c_uint32),
                ("max_tick_tris", C.c_uint64)]


class vr_request(C.Structure):
    _fields_ = [("mesh", C.c_uint32), ("num_tris", C.c_uint32), ("strategy", C.c_int), ("batch_tris", C.c_uint32),
                ("max_unique", C.c_uint32), ("pad", C.c_uint32), ("user", C.c_uint64),
                ("shader", vr_shader_params)]


class vr_completion(C.Structure):
    _fields_ = [("ticket", C.c_uint64), ("user", C.c_uint64), ("status", C.c_int32), ("tick", C.c_uint32),
                ("num_tris", C.c_uint64), ("invocations", C.c_uint64), ("units", C.c_uint64),
                ("d_corners", C.c_void_p), ("t_submit", C.c_double), ("t_admit", C.c_double),
                ("t_launch", C.c_double), ("t_done", C.c_double)]


class vr_server_stats(C.Structure):
    _fields_ = [(k, C.c_uint64) for k in (
        "submitted", "completed", "cancelled", "rejected", "ticks", "budget_bytes", "reserved_bytes",
        "peak_reserved_bytes", "pending", "admitted", "inflight_ticks", "max_pending", "max_tick_draws",
        "admission_blocked", "plan_bytes")]


class vr_sim_request(C.Structure):
    _fields_ = [("arrival", C.c_double), ("cancel_at", C.c_double), ("hold", C.c_double),
                ("num_tris", C.c_uint64), ("bytes", C.c_uint64)]


class vr_sim_result(C.Structure):
    _fields_ = [("status", C.c_int32), ("tick", C.c_uint32), ("t_admit", C.c_double), ("t_launch", C.c_double),
                ("t_done", C.c_double), ("t_release", C.c_double), ("offset", C.c_uint64)]


def _struct_dict(x):
    return {k: getattr(x, k) for k, _ in x._fields_}


class VrError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"vr status {status}: {message}")
        self.status = status


_lib = None


def lib():
    """The loaded libvr.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.vr_create.argtypes = [C.POINTER(C.c_void_p), C.c_int, P]
        L.vr_create.restype = C.c_int
        L.vr_destroy.argtypes = [P]
        L.vr_destroy.restype = None
        L.vr_set_stream.argtypes = [P, P]
        L.vr_set_stream.restype = C.c_int
        L.vr_check_args.argtypes = [C.c_uint64, C.c_uint32, C.POINTER(vr_shader_params), C.c_int, C.c_uint32,
                                    C.POINTER(vr_opts), C.POINTER(vr_outputs)]
        L.vr_check_args.restype = C.c_int
        L.vr_plan_dynamic.argtypes = [P, P, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, P, C.c_uint64]
        L.vr_plan_dynamic.restype = C.c_int
        L.vr_process_draw.argtypes = [P, P, C.c_uint64, P, C.c_uint32, C.POINTER(vr_shader_params), C.c_int,
                                      C.c_uint32, C.POINTER(vr_opts), C.POINTER(vr_outputs)]
        L.vr_process_draw.restype = C.c_int
        L.vr_process_draw_noalloc.argtypes = L.vr_process_draw.argtypes
        L.vr_process_draw_noalloc.restype = C.c_int
        L.vr_walk_step.argtypes = [P, P, C.c_uint32, P, C.c_uint32, P, P, C.c_uint32, P, C.c_int, C.c_uint32, P, P]
        L.vr_walk_step.restype = C.c_int
        L.vr_stream_create.argtypes = [P, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, P, C.c_uint64,
                                       C.POINTER(C.c_void_p)]
        L.vr_stream_create.restype = C.c_int
        L.vr_stream_push.argtypes = [P, P, C.c_uint64, P, C.c_uint32, C.POINTER(vr_shader_params), C.c_int,
                                     C.c_uint32]
        L.vr_stream_push.restype = C.c_int
        L.vr_stream_finish.argtypes = [P, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]
        L.vr_stream_finish.restype = C.c_int
        L.vr_stream_destroy.argtypes = [P]
        L.vr_stream_destroy.restype = None
        L.vr_sync.argtypes = [P, C.POINTER(C.c_uint64)]
        L.vr_sync.restype = C.c_int
        L.vr_frame_create.argtypes = [P, C.POINTER(vr_draw), C.c_uint32, C.POINTER(vr_shader_params), C.c_uint32,
                                      C.c_int, C.POINTER(C.c_void_p)]
        L.vr_frame_create.restype = C.c_int
        L.vr_frame_run.argtypes = [P]
        L.vr_frame_run.restype = C.c_int
        L.vr_frame_destroy.argtypes = [P]
        L.vr_frame_destroy.restype = None
        L.vr_process_draws.argtypes = [P, C.POINTER(vr_draw), C.c_uint32, C.POINTER(vr_shader_params), C.c_uint32]
        L.vr_process_draws.restype = C.c_int
        L.vr_set_kernel_timing.argtypes = [P, C.c_int]
        L.vr_set_kernel_timing.restype = C.c_int
        L.vr_kernel_times.argtypes = [P, C.POINTER(C.c_float), C.c_uint32, C.POINTER(C.c_uint32)]
        L.vr_kernel_times.restype = C.c_int
        L.vr_math_selftest.argtypes = [P, C.c_uint32, C.c_uint64, C.c_uint64, P, C.POINTER(C.c_uint64)]
        L.vr_math_selftest.restype = C.c_int
        L.vr_last_error.argtypes = [P]
        L.vr_last_error.restype = C.c_char_p
        L.vr_server_create.argtypes = [C.c_int, C.POINTER(vr_server_config), C.POINTER(C.c_void_p)]
        L.vr_server_add_mesh.argtypes = [P, P, C.c_uint64, P, C.c_uint32, C.POINTER(C.c_uint32)]
        L.vr_server_submit.argtypes = [P, C.POINTER(vr_request), C.POINTER(C.c_uint64)]
        L.vr_server_submit_many.argtypes = [P, C.POINTER(vr_request), C.c_uint32, C.POINTER(C.c_uint64),
                                            C.POINTER(C.c_uint32)]
        L.vr_server_poll.argtypes = [P, C.POINTER(vr_completion), C.c_uint32, C.POINTER(C.c_uint32), C.c_uint32]
        L.vr_server_release.argtypes = [P, C.c_uint64]
        L.vr_server_cancel.argtypes = [P, C.c_uint64]
        L.vr_server_fetch.argtypes = [P, C.c_uint64, P, C.c_uint64]
        L.vr_server_stats_get.argtypes = [P, C.POINTER(vr_server_stats)]
        L.vr_server_simulate.argtypes = [C.POINTER(vr_server_config), C.POINTER(vr_sim_request), C.c_uint32,
                                         C.c_double, C.c_double, C.POINTER(vr_sim_result),
                                         C.POINTER(vr_server_stats)]
        for f in ("vr_server_create", "vr_server_add_mesh", "vr_server_submit", "vr_server_submit_many", "vr_server_poll",
                  "vr_server_release", "vr_server_fetch", "vr_server_cancel", "vr_server_stats_get", "vr_server_simulate"):
            getattr(L, f).restype = C.c_int
        L.vr_server_destroy.argtypes = [P]
        L.vr_server_destroy.restype = None
        L.vr_server_last_error.argtypes = [P]
        L.vr_server_last_error.restype = C.c_char_p
        _lib = L
    return _lib


# ---------------------------------------------------------------- marshalling
def make_shader(sp) -> vr_shader_params:
    """From a workloads.ShaderParams (or an object with the same fields)."""
    s = vr_shader_params()
    s.kind, s.num_lights, s.iterations, s.spec_squarings = (int(sp.kind), int(sp.num_lights),
                                                             int(sp.iterations), int(sp.spec_squarings))
    for name, n in (("mvp", 16), ("model", 12), ("normal", 9), ("eye", 3), ("ambient", 3), ("coef", 8)):
        arr = np.ascontiguousarray(np.asarray(getattr(sp, name), dtype=np.float32).ravel())
        assert arr.size == n, name
        C.memmove(C.addressof(getattr(s, name)), arr.ctypes.data, 4 * n)
    s.kd, s.ks, s.katt = float(np.float32(sp.kd)), float(np.float32(sp.ks)), float(np.float32(sp.katt))
    lights = np.ascontiguousarray(np.asarray(sp.lights, dtype=np.float32).reshape(16, 6))
    C.memmove(C.addressof(s.lights), lights.ctypes.data, 4 * 96)
    return s


def make_opts(max_unique=0, wg_size=0, hash_slots=0, hash_probes=0, plan=None) -> vr_opts:
    return vr_opts(max_unique, wg_size, hash_slots, hash_probes, None if plan is None else plan.data_ptr())


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream_handle(stream):
    if stream is None:
        return None
    return C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


# ---------------------------------------------------------------- C names
def vr_create(device=0, stream=None):
    h = C.c_void_p()
    st = lib().vr_create(C.byref(h), int(device), _stream_handle(stream))
    if st != VR_OK:
        raise VrError(st, lib().vr_last_error(None).decode())
    return h


def vr_destroy(ctx):
    lib().vr_destroy(ctx)


def vr_set_stream(ctx, stream):
    return lib().vr_set_stream(ctx, _stream_handle(stream))


def vr_last_error(ctx=None):
    return lib().vr_last_error(ctx).decode()


def vr_check_args(num_indices, num_vertices, shader, strategy, batch_tris, opts=None, outputs=None):
    sh = shader if isinstance(shader, vr_shader_params) else make_shader(shader)
    out = outputs if outputs is not None else vr_outputs()
    return lib().vr_check_args(num_indices, num_vertices, C.byref(sh), strategy, batch_tris,
                               C.byref(opts) if opts is not None else None, C.byref(out))


def vr_plan_dynamic(ctx, indices, num_vertices, max_unique, max_tris, plan):
    return lib().vr_plan_dynamic(ctx, _ptr(indices), indices.numel(), num_vertices, max_unique, max_tris,
                                 _ptr(plan), plan.numel())


def vr_stream_create(ctx, slots, chunk_tris, width, height, records):
    """records: float32 device tensor [capacity, 8]."""
    h = C.c_void_p()
    st = lib().vr_stream_create(ctx, slots, chunk_tris, width, height, _ptr(records), records.shape[0], C.byref(h))
    return st, h


def vr_stream_push(stream, indices, vertices, shader, strategy, batch_tris):
    sh = shader if isinstance(shader, vr_shader_params) else make_shader(shader)
    V = vertices.shape[0] if vertices.dim() == 2 else vertices.numel() // 8
    return lib().vr_stream_push(stream, _ptr(indices), indices.numel(), _ptr(vertices), V, C.byref(sh), strategy,
                                batch_tris)


def vr_stream_finish(stream):
    t, v, i = C.c_uint64(0), C.c_uint64(0), C.c_uint64(0)
    st = lib().vr_stream_finish(stream, C.byref(t), C.byref(v), C.byref(i))
    return st, int(t.value), int(v.value), int(i.value)


def vr_stream_destroy(stream):
    lib().vr_stream_destroy(stream)


def vr_walk_step(ctx, keys_in, activity, grid, moves, weights, uniforms, strategy, batch_agents, keys_out,
                 counters=None):
    """One random-walk step (device tensors; moves as int8 (dx, dy) pairs)."""
    return lib().vr_walk_step(ctx, _ptr(keys_in), keys_in.numel(), _ptr(activity), grid, _ptr(moves), _ptr(weights),
                              weights.numel(), _ptr(uniforms), strategy, batch_agents, _ptr(keys_out),
                              None if counters is None else counters.data_ptr())


def vr_process_draw(ctx, indices, vertices, shader, strategy, batch_tris, opts=None, outputs=None):
    sh = shader if isinstance(shader, vr_shader_params) else make_shader(shader)
    out = outputs if outputs is not None else vr_outputs()
    V = vertices.shape[0] if vertices.dim() == 2 else vertices.numel() // 8
    return lib().vr_process_draw(ctx, _ptr(indices), indices.numel(), _ptr(vertices), V, C.byref(sh),
                                 strategy, batch_tris, C.byref(opts) if opts is not None else None,
                                 C.byref(out))


def vr_process_draw_noalloc(ctx, indices, vertices, shader, strategy, batch_tris, opts=None, outputs=None):
    """As vr_process_draw, with the library's static scratch (no allocation)."""
    sh = shader if isinstance(shader, vr_shader_params) else make_shader(shader)
    out = outputs if outputs is not None else vr_outputs()
    V = vertices.shape[0] if vertices.dim() == 2 else vertices.numel() // 8
    return lib().vr_process_draw_noalloc(ctx, _ptr(indices), indices.numel(), _ptr(vertices), V, C.byref(sh),
                                         strategy, batch_tris, C.byref(opts) if opts is not None else None,
                                         C.byref(out))


def vr_sync(ctx):
    inv = C.c_uint64(0)
    st = lib().vr_sync(ctx, C.byref(inv))
    return st, int(inv.value)


def make_draw(indices, vertices, shader_index, strategy, batch_tris, corners, counters=None, max_unique=0,
              plan=None) -> vr_draw:
    """A frame entry from torch tensors (device memory)."""
    V = vertices.shape[0] if vertices.dim() == 2 else vertices.numel() // 8
    return vr_draw(indices.data_ptr() if indices.numel() else None, indices.numel(),
                   vertices.data_ptr(), V, shader_index, strategy, batch_tris, max_unique,
                   None if plan is None else plan.data_ptr(), corners.data_ptr() if corners.numel() else None,
                   None if counters is None else counters.data_ptr())


def _tables(draws, shaders):
    dr = (vr_draw * max(1, len(draws)))(*draws)
    sh = [x if isinstance(x, vr_shader_params) else make_shader(x) for x in shaders]
    st = (vr_shader_params * max(1, len(sh)))(*sh)
    return dr, st


def vr_frame_create(ctx, draws, shaders, capture_graph=False):
    dr, st = _tables(draws, shaders)
    h = C.c_void_p()
    rc = lib().vr_frame_create(ctx, dr, len(draws), st, len(shaders), 1 if capture_graph else 0, C.byref(h))
    return rc, h


def vr_frame_run(frame):
    return lib().vr_frame_run(frame)


def vr_frame_destroy(frame):
    lib().vr_frame_destroy(frame)


def vr_process_draws(ctx, draws, shaders):
    dr, st = _tables(draws, shaders)
    return lib().vr_process_draws(ctx, dr, len(draws), st, len(shaders))


def vr_set_kernel_timing(ctx, enable):
    return lib().vr_set_kernel_timing(ctx, 1 if enable else 0)


def vr_kernel_times(ctx, cap=4096):
    """Milliseconds of the timed launches since the previous call, in order."""
    buf = (C.c_float * cap)()
    n = C.c_uint32(0)
    st = lib().vr_kernel_times(ctx, buf, cap, C.byref(n))
    if st != VR_OK:
        raise VrError(st, vr_last_error(ctx))
    return [buf[i] for i in range(min(n.value, cap))]


def vr_math_selftest(ctx, fn, first=0, count=1 << 32, out=None):
    """Rounded-arithmetic self-test (fn 0 = 1/x, 1 = sqrt, 2 = 1/sqrt) over the
    float32 bit patterns [first, first + count); returns (status, mismatches).
    `out`, a device tensor of `count` floats, receives the results."""
    m = C.c_uint64(0)
    st = lib().vr_math_selftest(ctx, fn, first, count, None if out is None else out.data_ptr(), C.byref(m))
    return st, int(m.value)


# ---------------------------------------------------------------- convenience
class GeometryStage:
    """A context plus output allocation with torch (device memory only)."""

    def __init__(self, device=0, stream=None):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        self.ctx = vr_create(device, stream if stream is not None else torch.cuda.current_stream(device))

    def close(self):
        if self.ctx is not None:
            vr_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, st):
        if st != VR_OK:
            raise VrError(st, vr_last_error(self.ctx))

    def alloc_outputs(self, num_tris, strategy, batch_tris, corners=True, tris=False, verts=False,
                      local_idx=False, units=False, num_vertices=0):
        """Output tensors for a draw; MULTI's verts hold all num_vertices."""
        torch = self.torch
        n = 3 * num_tris
        res = {"counters": torch.zeros(4, dtype=torch.int64, device=self.device)}
        if corners:
            res["corners"] = torch.empty((n, OUT_FLOATS), dtype=torch.float32, device=self.device)
        if tris:
            res["tris"] = torch.empty(n, dtype=torch.int32, device=self.device)
        if verts:
            rows = max(n, num_vertices) if strategy == VR_MULTI else n
            res["verts"] = torch.empty((max(rows, 1), OUT_FLOATS), dtype=torch.float32, device=self.device)
        if local_idx:
            res["local_idx"] = torch.empty(n, dtype=torch.int16, device=self.device)
        if units:
            ucap = units_bound(strategy, num_tris, batch_tris)
            res["unit_offsets"] = torch.empty(ucap + 1, dtype=torch.int32, device=self.device)
            res["unit_invocations"] = torch.empty(max(ucap, 1), dtype=torch.int32, device=self.device)
        return res

    @staticmethod
    def describe(res):
        def p(k):
            t = res.get(k)
            return None if t is None else t.data_ptr()
        ucap = res["unit_invocations"].numel() if res.get("unit_invocations") is not None else 0
        vcap = res["verts"].shape[0] if res.get("verts") is not None else 0
        return vr_outputs(p("corners"), p("tris"), p("verts"), vcap, p("local_idx"), p("unit_offsets"),
                          p("unit_invocations"), ucap, p("counters"))

    def draw(self, indices, vertices, shader, strategy, batch_tris, opts=None, res=None, **want):
        if res is None:
            res = self.alloc_outputs(indices.numel() // 3, strategy, batch_tris, **want)
        o = opts if (opts is None or isinstance(opts, vr_opts)) else make_opts(**opts)
        st = vr_process_draw(self.ctx, indices, vertices, shader, strategy, batch_tris, o, self.describe(res))
        self.check(st)
        return res

    def sync(self):
        st, inv = vr_sync(self.ctx)
        return st, inv


def units_bound(strategy, num_tris, batch_tris):
    if strategy == VR_MULTI:
        return 1
    if strategy in (VR_STATIC_SORT, VR_STATIC_HASH):
        return (num_tris + batch_tris - 1) // batch_tris
    return num_tris


# ------------------------------------------------------------- request server
def make_server_config(budget_bytes, max_inflight=0, max_tick_draws=0, max_tick_tris=0) -> vr_server_config:
    return vr_server_config(int(budget_bytes), int(max_inflight), int(max_tick_draws), int(max_tick_tris))


def vr_server_create(device, cfg):
    h = C.c_void_p()
    st = lib().vr_server_create(device, C.byref(cfg), C.byref(h))
    if st != VR_OK:
        raise VrError(st, vr_last_error(None))
    return h


def vr_server_last_error(server):
    msg = lib().vr_server_last_error(server)
    return msg.decode() if msg else ""


def vr_server_add_mesh(server, indices, vertices):
    """Registers a resident mesh (torch device tensors kept alive by the caller)."""
    m = C.c_uint32()
    V = vertices.shape[0] if vertices.dim() == 2 else vertices.numel() // 8
    st = lib().vr_server_add_mesh(server, _ptr(indices), indices.numel(), _ptr(vertices), V, C.byref(m))
    return st, m.value


def make_request(mesh, num_tris, shader, strategy, batch_tris, max_unique=0, user=0) -> vr_request:
    sh = shader if isinstance(shader, vr_shader_params) else make_shader(shader)
    return vr_request(mesh, num_tris, strategy, batch_tris, max_unique, 0, user, sh)


def vr_server_submit(server, request):
    t = C.c_uint64()
    st = lib().vr_server_submit(server, C.byref(request), C.byref(t))
    return st, t.value


def vr_server_submit_many(server, requests):
    """(status, tickets of the requests queued: all of them when status is VR_OK)."""
    n = len(requests)
    arr = (vr_request * n)(*requests)
    tickets = (C.c_uint64 * max(n, 1))()
    acc = C.c_uint32()
    st = lib().vr_server_submit_many(server, arr, n, tickets, C.byref(acc))
    return st, [int(tickets[i]) for i in range(acc.value)]


def vr_server_poll(server, cap=256, timeout_ms=0):
    """(status, list of completion dicts)."""
    buf = (vr_completion * cap)()
    n = C.c_uint32()
    st = lib().vr_server_poll(server, buf, cap, C.byref(n), timeout_ms)
    return st, [_struct_dict(buf[i]) for i in range(n.value)]


def vr_server_release(server, ticket):
    return lib().vr_server_release(server, ticket)


def vr_server_fetch(server, ticket, num_tris):
    """(status, float32[3 num_tris][12] numpy array) of a finished request."""
    out = np.empty((3 * num_tris, OUT_FLOATS), dtype=np.float32)
    st = lib().vr_server_fetch(server, ticket, out.ctypes.data, out.nbytes)
    return st, out


def vr_server_cancel(server, ticket):
    return lib().vr_server_cancel(server, ticket)


def vr_server_stats_get(server):
    o = vr_server_stats()
    st = lib().vr_server_stats_get(server, C.byref(o))
    return st, _struct_dict(o)


def vr_server_destroy(server):
    lib().vr_server_destroy(server)


def vr_server_simulate(cfg, requests, tick_fixed_s, tick_s_per_tri):
    """requests: list of (arrival, num_tris, bytes, cancel_at, hold), sorted by
    arrival.  Returns (status, list of result dicts, stats dict)."""
    n = len(requests)
    rq = (vr_sim_request * max(1, n))(*[vr_sim_request(a, c, h, t, b) for a, t, b, c, h in requests])
    res = (vr_sim_result * max(1, n))()
    stats = vr_server_stats()
    st = lib().vr_server_simulate(C.byref(cfg), rq, n, tick_fixed_s, tick_s_per_tri, res, C.byref(stats))
    return st, [_struct_dict(res[i]) for i in range(n)], _struct_dict(stats)
