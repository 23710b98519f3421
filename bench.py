"""Benchmark of the geometry stage on one MI355X.

Workload: icosphere subdivided 8 times (655,362 vertices, 1,310,720
triangles), Hilbert order with 5% local swaps in windows of 256, FP32
attributes, Phong shading with 8 point lights.  One step runs the whole hot
path once over this draw for every strategy, each producing the per-corner
shaded output and the invocation count:
    dynamic batch plan (N_u = 256, N_pmax = 341, the paper's setting, where
    the unique budget closes most batches), shared by the dynamic
    strategies; naive; static wave64 ballot (64 triangles); dynamic sort,
    hash and parallel hash (256 / 341).
value = triangles processed per second over the whole step (all strategies,
inputs resident in HBM).  Per-strategy throughput and shading rate are
reported beside it, with the roofline of the dominant kernel and the CPU
oracle timed on a bounded sample.
"""
import argparse
import glob
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP32_VECTOR_PEAK_TFLOPS = 157.3

METRIC = "triangles/s & shading rate per strategy vs no-reuse; p50/p99 draw latency"

# main kernel of each draw in the step (Phong shading instantiation; the
# step's dedup units fit the LDS of the occupancy-bound kernels, which they take)
KERNEL_NAMES = {"naive": "k_naive<1>", "static_ballot": "k_ballot<1>", "dyn_sort": "k_dedup<256, 0, 1, true>",
                "dyn_hash": "k_dedup<256, 1, 1, true>", "dyn_phash": "k_dedup<256, 2, 1, true>"}


def shader_flops(sp):
    """FP32 operations of one vertex-program evaluation (fma = 2, sqrt and
    divide = 1 each), counted from the written program."""
    mvp = 4 * 6 + 3 * 5 + 10
    if sp.kind == 1:
        return mvp + 18 + 13 + 48 * sp.num_lights
    if sp.kind == 2:
        return mvp + 11 + 9 * sp.iterations
    return mvp


def host_cpu_model():
    """The host CPU's model name (Linux), or None."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def strip_c_comments(text):
    """C/C++ source without its // and /* */ comments; string and character
    literals (which may hold those markers) are kept as they are."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c in "\"'":                       # a literal, up to its unescaped closing quote
            j = i + 1
            while j < n and text[j] != c and text[j] != "\n":
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            while i < n and text[i] != "\n":
                i += 1
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        else:
            out.append(c)
            i += 1
    return "".join(out)


def kernel_source_sha():
    """Hash of the kernel sources with comments and blank lines removed:
    HBM-traffic counters are used only when they were taken on exactly this
    code (a comment edit does not make them stale)."""
    h = hashlib.sha256()
    files = sorted(glob.glob(os.path.join(ROOT, "paper_1805_08893_amd", "csrc", "*"))) + \
        [os.path.join(ROOT, "include", "vr.h")]
    for f in files:
        with open(f, encoding="utf-8") as fh:
            text = strip_c_comments(fh.read())
        code = "\n".join(line.rstrip() for line in text.splitlines() if line.strip())
        h.update(os.path.basename(f).encode())
        h.update(code.encode())
    return h.hexdigest()[:16]


def committed_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary, or
    None when it is missing or was taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_source_sha") != kernel_source_sha():
        return None
    k = d.get("kernels", {}).get(kernel)
    return None if k is None else k.get("hbm_bytes_per_launch")


def scene_benchmark(stage, seed=3, num_draws=2000, replays=10, table=None):
    """Many draws in one persistent launch (a hipGraph frame) against one
    launch per draw, with autotuned per-class configurations.  Draw sizes are
    log-normal in [100, 200000] triangles (mean about 5,000), each draw the
    first T_d triangles of a grid or icosphere base mesh in Hilbert or scan
    order, shaders MVP, Phong-4 or Phong-16.  With `table` (a JSON path) the
    autotuner's choices are read from it when it exists and written to it
    otherwise, so that separate runs (profiler passes) use the same ones."""
    import torch
    from paper_1805_08893_amd import vr
    from paper_1805_08893_amd import workloads as W
    from paper_1805_08893_amd.autotune import Autotuner

    bases = [W.grid_mesh(318, 318, seed, "hilbert"), W.grid_mesh(318, 318, seed, "scan"),
             W.icosphere_mesh(7, seed, "hilbert"), W.icosphere_mesh(7, seed, "scan")]
    dev = [(torch.from_numpy(m.indices.view(np.int32)).cuda(), torch.from_numpy(m.vertices).cuda()) for m in bases]
    shaders = [W.shader_for_mesh(bases[2], W.SHADER_MVP, seed),
               W.shader_for_mesh(bases[2], W.SHADER_PHONG, seed, num_lights=4),
               W.shader_for_mesh(bases[2], W.SHADER_PHONG, seed, num_lights=16)]
    rng = np.random.default_rng(seed)
    Ts = np.clip(np.exp(rng.normal(np.log(5000.0) - 0.72, 1.2, num_draws)), 100, 200000).astype(np.int64)
    which = rng.integers(0, len(bases), num_draws)
    shade = rng.integers(0, len(shaders), num_draws)
    tuner = Autotuner(stage.ctx, path=table)
    total_T = int(Ts.sum())
    corners = torch.empty((3 * total_T, 12), dtype=torch.float32, device="cuda")
    counters = torch.zeros((num_draws, 4), dtype=torch.int64, device="cuda")
    draws, cfgs, plans = [], [], []
    off = 0
    t_tune = time.perf_counter()
    for d in range(num_draws):
        m = bases[which[d]]
        T = int(min(Ts[d], m.num_tris))
        idx, vtx = dev[which[d]][0][:3 * T], dev[which[d]][1]
        key, (s, bt, nu) = tuner.choose(idx, m.indices[:3 * T], vtx, shaders[shade[d]])
        plan = None
        if s in vr.DYNAMIC:
            plan = torch.empty(T + 2, dtype=torch.int32, device="cuda")
            stage.check(vr.vr_plan_dynamic(stage.ctx, idx, m.num_verts, nu, bt, plan))
        c = corners[3 * off:3 * (off + T)]
        draws.append(vr.make_draw(idx, vtx, int(shade[d]), s, bt, c, counters[d], nu, plan))
        cfgs.append((idx, vtx, int(shade[d]), s, bt, nu, plan, c, counters[d]))
        plans.append(plan)
        off += T
    stage.check(stage.sync()[0])
    t_tune = time.perf_counter() - t_tune
    if table:
        tuner.save()
    # one launch per draw
    sh = [vr.make_shader(x) for x in shaders]
    outs = [vr.vr_outputs(c.data_ptr(), None, None, 0, None, None, None, 0, cnt.data_ptr())
            for (_, _, _, _, _, _, _, c, cnt) in cfgs]
    opts = [vr.make_opts(max_unique=nu, plan=plan) for (_, _, _, _, _, nu, plan, _, _) in cfgs]

    def per_draw():
        for k, (idx, vtx, si, s, bt, nu, plan, c, cnt) in enumerate(cfgs):
            stage.check(vr.vr_process_draw(stage.ctx, idx, vtx, sh[si], s, bt, opts[k], outs[k]))

    per_draw()
    stage.check(stage.sync()[0])
    inv_loop = int(counters[:, 0].sum().item())
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(3):
        per_draw()
    e1.record()
    torch.cuda.synchronize()
    loop_ms = e0.elapsed_time(e1) / 3
    stage.check(stage.sync()[0])
    rc, frame = vr.vr_frame_create(stage.ctx, draws, shaders, capture_graph=True)
    stage.check(rc)
    try:
        counters.zero_()
        for _ in range(2):
            stage.check(vr.vr_frame_run(frame))
        stage.check(stage.sync()[0])
        inv_frame = int(counters[:, 0].sum().item())
        e0.record()
        for _ in range(replays):
            stage.check(vr.vr_frame_run(frame))
        e1.record()
        torch.cuda.synchronize()
        frame_ms = e0.elapsed_time(e1) / replays
        stage.check(stage.sync()[0])
    finally:
        vr.vr_frame_destroy(frame)
    classes = {k: {"strategy": vr.STRATEGY_NAMES[v["strategy"]], "batch_tris": v["batch_tris"],
                   "max_unique": v["max_unique"]} for k, v in tuner.table.items()}
    # roofs of the frame: per draw 12 B/triangle of indices, 32 B per
    # referenced vertex, 144 B/triangle of corners; FP32 work = invocations x
    # the program's operations
    inv_d = counters[:, 0].cpu().numpy()
    alg_bytes = alg_flops = 0
    for d in range(num_draws):
        m = bases[which[d]]
        T = int(min(Ts[d], m.num_tris))
        alg_bytes += 156 * T + 32 * len(np.unique(m.indices[:3 * T]))
        alg_flops += int(inv_d[d]) * shader_flops(shaders[shade[d]])
    return {"draws": num_draws, "triangles": total_T, "frame_ms": frame_ms, "per_draw_launch_ms": loop_ms,
            "frame_tri_per_s": total_T / (frame_ms * 1e-3), "per_draw_tri_per_s": total_T / (loop_ms * 1e-3),
            "speedup_frame_vs_per_draw": loop_ms / frame_ms, "invocations_frame": inv_frame,
            "invocations_per_draw": inv_loop, "autotune_and_plan_s": t_tune,
            "algorithmic_bytes": alg_bytes, "hbm_frac": alg_bytes / (frame_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "alu_frac": alg_flops / (frame_ms * 1e-3) / 1e12 / FP32_VECTOR_PEAK_TFLOPS, "classes": classes}


def sweep(mesh, sp, reps=10):
    """Batch-size sweep of every strategy (one JSON line per configuration):
    main-kernel time, plan time and invocations."""
    import torch
    from paper_1805_08893_amd import vr
    T, V = mesh.num_tris, mesh.num_verts
    idx = torch.from_numpy(mesh.indices.view(np.int32)).cuda()
    vtx = torch.from_numpy(mesh.vertices).cuda()
    stage = vr.GeometryStage(0)
    shader = vr.make_shader(sp)
    plan = torch.empty(T + 2, dtype=torch.int32, device="cuda")
    out = stage.alloc_outputs(T, vr.VR_NAIVE, 1, corners=True)
    configs = [("naive", vr.VR_NAIVE, 1, 0)]
    for bt in (21, 32, 64, 128, 256, 512, 1024):
        configs.append(("static_ballot", vr.VR_STATIC_BALLOT, bt, 0))
    for bt in (32, 64, 128, 256):
        configs += [("static_sort", vr.VR_STATIC_SORT, bt, 0), ("static_hash", vr.VR_STATIC_HASH, bt, 0)]
    for nu, bt in ((64, 64), (128, 128), (256, 128), (256, 256), (256, 341), (512, 512)):
        for name, s in (("dyn_ballot", vr.VR_DYN_BALLOT), ("dyn_sort", vr.VR_DYN_SORT), ("dyn_hash", vr.VR_DYN_HASH),
                        ("dyn_phash", vr.VR_DYN_PHASH)):
            configs.append((name, s, bt, nu))
    for name, s, bt, nu in configs:
        plan_ms = None
        if s in vr.DYNAMIC:
            vr.vr_set_kernel_timing(stage.ctx, True)
            vr.vr_kernel_times(stage.ctx)
            for _ in range(reps):
                stage.check(vr.vr_plan_dynamic(stage.ctx, idx, V, nu, bt, plan))
            plan_ms = float(np.mean(vr.vr_kernel_times(stage.ctx)))
        o = vr.make_opts(max_unique=nu, plan=plan if s in vr.DYNAMIC else None)
        rc = vr.vr_check_args(3 * T, V, shader, s, bt, o, stage.describe(out))
        if rc != vr.VR_OK:
            print(json.dumps({"strategy": name, "batch_tris": bt, "max_unique": nu, "error": rc}), flush=True)
            continue
        for _ in range(2):
            stage.check(vr.vr_process_draw(stage.ctx, idx, vtx, shader, s, bt, o, stage.describe(out)))
        vr.vr_set_kernel_timing(stage.ctx, True)
        vr.vr_kernel_times(stage.ctx)
        for _ in range(reps):
            stage.check(vr.vr_process_draw(stage.ctx, idx, vtx, shader, s, bt, o, stage.describe(out)))
        ms = float(np.mean(vr.vr_kernel_times(stage.ctx)))
        vr.vr_set_kernel_timing(stage.ctx, False)
        st, inv = stage.sync()
        stage.check(st)
        inv //= reps + 2
        print(json.dumps({"strategy": name, "batch_tris": bt, "max_unique": nu, "kernel_us": round(ms * 1e3, 1),
                          "plan_us": None if plan_ms is None else round(plan_ms * 1e3, 1), "invocations": inv,
                          "reuse": round(1 - inv / (3 * T), 4), "tri_per_s": T / (ms * 1e-3)}), flush=True)
    stage.close()


def unit_chunks(T, cuts, parts):
    """Split triangles [0, T) into at most `parts` contiguous chunks whose
    bounds are unit starts (`cuts`, ascending, from 0): each chunk is a draw
    of its own whose units are exactly the units of the whole draw in it
    (static batches restart at multiples of the batch size, and greedy
    dynamic batching restarts at every batch start)."""
    cuts = np.asarray(cuts, dtype=np.int64)
    want = [T * k // parts for k in range(1, parts)]
    pos = np.searchsorted(cuts, want)
    inner = sorted({int(cuts[p]) for p in pos if p < len(cuts) and 0 < cuts[p] < T})
    b = [0] + inner + [T]
    return [(b[i], b[i + 1]) for i in range(len(b) - 1) if b[i + 1] > b[i]]


def strategy_cuts(vro, mesh, s, bt, nu):
    """Unit starts usable as chunk bounds: every triangle (naive), multiples
    of the batch size (static), the dynamic plan's batch starts (dynamic)."""
    from paper_1805_08893_amd import vr
    T = mesh.num_tris
    if s == vr.VR_NAIVE:
        return np.arange(T, dtype=np.int64)
    if s in vr.DYNAMIC:
        assert nu >= 3, "dynamic strategies name their unique budget"
        return vro.plan_dynamic(mesh.indices, mesh.num_verts, nu, bt)[:-1]
    return np.arange(0, T, bt, dtype=np.int64)


def cpu_oracle_baseline(mesh, sp, strategies, st_passes, mt_passes):
    """The C oracle timed on the host: (i) one thread over whole draws, and
    (ii) all host threads, each running the oracle on a contiguous chunk of
    whole units (the dynamic plan is made first, sequentially, and timed
    apart; each chunk then plans its own part again, inside the parallel
    time).  The chunks' invocation counts must add up to the whole draw's.
    Beside it, the k-entry FIFO post-transform cache (k = 16, 32) as the
    classic comparison point for the invocations of each strategy."""
    from concurrent.futures import ThreadPoolExecutor
    from oracle import vro
    T, V = mesh.num_tris, mesh.num_verts
    U = int(len(np.unique(mesh.indices)))
    threads = len(os.sched_getaffinity(0))
    vsh = vro.make_shader(sp)
    whole = {}
    t_st, tris_st = 0.0, 0
    for _ in range(st_passes):
        for name, s, bt, nu in strategies:
            c0 = time.perf_counter()
            rc, r = vro.process_draw(mesh.indices, mesh.vertices, vsh, s, bt, {"max_unique": nu}, tris=False,
                                     verts=False, local_idx=False, units=False)
            t_st += time.perf_counter() - c0
            tris_st += T
            assert rc == vro.OK, (name, rc)
            whole[name] = int(r["counters"][0])
    # plans (sequential), then the chunks of every strategy on all threads
    plan_s, chunks = {}, {}
    for name, s, bt, nu in strategies:
        c0 = time.perf_counter()
        cuts = strategy_cuts(vro, mesh, s, bt, nu)
        plan_s[name] = time.perf_counter() - c0
        chunks[name] = unit_chunks(T, cuts, threads)

    def run(name, s, bt, nu, a, b):
        rc, r = vro.process_draw(mesh.indices[3 * a:3 * b], mesh.vertices, vsh, s, bt, {"max_unique": nu},
                                 tris=False, verts=False, local_idx=False, units=False)
        assert rc == vro.OK, (name, rc)
        return int(r["counters"][0])

    t_mt, tris_mt, per = 0.0, 0, {}
    with ThreadPoolExecutor(threads) as pool:
        for _ in range(mt_passes):
            for name, s, bt, nu in strategies:
                c0 = time.perf_counter()
                inv = sum(pool.map(lambda ab: run(name, s, bt, nu, *ab), chunks[name]))
                dt = time.perf_counter() - c0
                t_mt += dt
                tris_mt += T
                per[name] = per.get(name, 0.0) + dt
                if inv != whole[name]:
                    raise RuntimeError(f"{name}: chunked oracle invocations {inv} != whole draw {whole[name]}")
    fifo = {}
    for k in (16, 32):
        m = vro.fifo_misses(mesh.indices, V, k)
        fifo[f"fifo{k}"] = {"invocations": m, "shading_rate": m / U, "reuse": 1.0 - m / (3.0 * T)}
    from paper_1805_08893_amd import vr
    plan_total = sum(plan_s[n] for n, s, *_ in strategies if s in vr.DYNAMIC)
    return {"value": tris_mt / t_mt, "unit": "triangles/s", "cores": threads, "kind": "oracle",
            "sample": f"{mt_passes} pass(es) of the full step ({len(strategies)} draws x {T} triangles) on "
                      f"{threads} threads, each thread the C oracle on a contiguous chunk of whole units, "
                      f"{t_mt:.1f} s wall; dynamic plans made beforehand on one thread ({plan_total:.2f} s, "
                      f"not in the value)",
            "single_thread": {"value": tris_st / t_st, "cores": 1,
                              "sample": f"{st_passes} pass(es) of the full step, one thread, {t_st:.1f} s"},
            "per_strategy_ms_all_cores": {n: 1e3 * v / mt_passes for n, v in per.items()},
            "plan_ms_one_thread": {n: 1e3 * plan_s[n] for n, s, *_ in strategies if s in vr.DYNAMIC},
            "fifo_post_transform_cache": fifo,
            "host_cpu": host_cpu_model(), "host_threads": threads}



def measure_draw(stage, idx, vtx, V, sp, strategy, bt, nu=0, reps=20, flush=None, output="corners", U=None):
    """One configuration: plan time (dynamic), main-kernel time from the
    library's HIP events, draw time (events around the whole call) p50/p99,
    invocations and the roofline fractions.  output = "corners" (per-corner
    shaded vertices, 144 B per triangle) or "indexed" (the shaded vertices of
    every unit once plus the assembled index triangles: 48 B per invocation
    and 12 B per triangle).  U = distinct indices of the draw (default V).
    With `flush` (a device tensor) the caches are overwritten before every
    timed draw (cold runs)."""
    import torch
    from paper_1805_08893_amd import vr
    T = idx.numel() // 3
    sh = vr.make_shader(sp)
    plan = None
    plan_ms = None
    if strategy in vr.DYNAMIC:
        plan = torch.empty(T + 2, dtype=torch.int32, device="cuda")
        vr.vr_set_kernel_timing(stage.ctx, True)
        vr.vr_kernel_times(stage.ctx)
        for _ in range(max(3, reps // 4)):
            stage.check(vr.vr_plan_dynamic(stage.ctx, idx, V, nu, bt, plan))
        plan_ms = float(np.median(vr.vr_kernel_times(stage.ctx)))
        vr.vr_set_kernel_timing(stage.ctx, False)
    indexed = output == "indexed"
    out = stage.alloc_outputs(T, strategy, bt, corners=not indexed, tris=indexed, verts=indexed, num_vertices=V)
    o = vr.make_opts(max_unique=nu, plan=plan)
    for _ in range(3):
        stage.check(vr.vr_process_draw(stage.ctx, idx, vtx, sh, strategy, bt, o, stage.describe(out)))
    st, _ = stage.sync()
    stage.check(st)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    vr.vr_set_kernel_timing(stage.ctx, True)
    vr.vr_kernel_times(stage.ctx)
    for e0, e1 in ev:
        if flush is not None:
            flush.fill_(1.0)
        e0.record()
        stage.check(vr.vr_process_draw(stage.ctx, idx, vtx, sh, strategy, bt, o, stage.describe(out)))
        e1.record()
    torch.cuda.synchronize()
    kms = np.array(vr.vr_kernel_times(stage.ctx), dtype=np.float64)
    vr.vr_set_kernel_timing(stage.ctx, False)
    st, _ = stage.sync()
    stage.check(st)
    ms = np.array([a.elapsed_time(b) for a, b in ev])
    inv = int(out["counters"][0].item())
    units = int(out["counters"][1].item())
    U = int(V) if U is None else int(U)
    k = float(np.median(kms))
    alg = algorithmic_bytes(T, U, inv, output, multi=strategy == vr.VR_MULTI)
    return {"output": output, "batch_tris": bt, "max_unique": nu, "kernel_ms_p50": k,
            "draw_ms_p50": float(np.percentile(ms, 50)), "draw_ms_p99": float(np.percentile(ms, 99)),
            "plan_ms_p50": plan_ms, "invocations": inv, "units": units, "shading_rate": inv / U,
            "reuse": 1.0 - inv / (3.0 * T), "tri_per_s": T / (k * 1e-3),
            "tri_per_s_with_plan": T / ((k + (plan_ms or 0.0)) * 1e-3), "algorithmic_bytes": alg,
            "hbm_frac": alg / (k * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "alu_frac": inv * shader_flops(sp) / (k * 1e-3) / 1e12 / FP32_VECTOR_PEAK_TFLOPS}


def algorithmic_bytes(T, U, inv, output="corners", multi=False):
    """Bytes a draw must move at least: its indices (12 B per triangle),
    every referenced vertex once (32 B), and its outputs: 144 B per triangle
    of per-corner vertices, or 48 B per invocation of shaded vertices plus
    12 B per triangle of assembled indices.  The two-pass reference also
    writes its shaded buffer (48 B per vertex) and reads it back once."""
    if multi:   # indexed: the shaded buffer is the output
        return 12 * T + 32 * U + (96 * U + 144 * T if output == "corners" else 48 * U + 12 * T)
    base = 12 * T + 32 * min(U, inv)
    return base + (144 * T if output == "corners" else 48 * inv + 12 * T)


def batch_sweep(stage, idx, vtx, V, U, sp, reps=10):
    """The bench workload over batch sizes {32, 64, 128, 256}: static ballot,
    sort and hash with N_p = B, and the dynamic strategies with N_pmax = B and
    N_u = 64 ceil(B / 64); then the paper's point (N_u 256, N_pmax 341) and
    the shading rate against the unique budget N_u with N_pmax = 4 N_u / 3
    (dynamic hash).  Main-kernel time, plan time, invocations, shading rate."""
    from paper_1805_08893_amd import vr
    rows = []

    def add(name, s, bt, nu):
        r = measure_draw(stage, idx, vtx, V, sp, s, bt, nu, reps=reps, U=U)
        rows.append({"strategy": name, "batch_tris": bt, "max_unique": nu,
                     "kernel_us": round(r["kernel_ms_p50"] * 1e3, 1),
                     "plan_us": None if r["plan_ms_p50"] is None else round(r["plan_ms_p50"] * 1e3, 1),
                     "invocations": r["invocations"], "shading_rate": round(r["shading_rate"], 4),
                     "tri_per_s": r["tri_per_s"], "hbm_frac": round(r["hbm_frac"], 4)})

    for B in (32, 64, 128, 256):
        nu = 64 * -(-B // 64)
        for name, s in (("static_ballot", vr.VR_STATIC_BALLOT), ("static_sort", vr.VR_STATIC_SORT),
                        ("static_hash", vr.VR_STATIC_HASH)):
            add(name, s, B, 0)
        for name, s in (("dyn_ballot", vr.VR_DYN_BALLOT), ("dyn_sort", vr.VR_DYN_SORT),
                        ("dyn_hash", vr.VR_DYN_HASH), ("dyn_phash", vr.VR_DYN_PHASH)):
            add(name, s, B, nu)
    for name, s in (("dyn_sort", vr.VR_DYN_SORT), ("dyn_hash", vr.VR_DYN_HASH), ("dyn_phash", vr.VR_DYN_PHASH)):
        add(name, s, 341, 256)
    curve = []
    # per-corner outputs keep every unique vertex of a unit in LDS (48 B
    # each): up to N_u = 2048; indexed outputs stream them out: up to 4096
    for output, budgets in (("corners", (64, 128, 256, 512, 1024, 2048)), ("indexed", (1024, 2048, 3072, 4096))):
        for nu in budgets:
            bt = min(vr.VR_MAX_BATCH_DYNAMIC, 4 * nu // 3)
            r = measure_draw(stage, idx, vtx, V, sp, vr.VR_DYN_HASH, bt, nu, reps=reps, U=U, output=output)
            curve.append({"output": output, "max_unique": nu, "batch_tris": bt,
                          "shading_rate": round(r["shading_rate"], 4), "kernel_us": round(r["kernel_ms_p50"] * 1e3, 1),
                          "plan_us": round(r["plan_ms_p50"] * 1e3, 1), "tri_per_s": r["tri_per_s"],
                          "hbm_frac": round(r["hbm_frac"], 4)})
    return {"rows": rows, "shading_rate_vs_max_unique": curve}


def indexed_outputs(stage, idx, vtx, V, U, sp, configs, reps=10):
    """Each strategy with the indexed outputs (the shaded vertices of every
    unit once and the assembled index triangles), where reuse cuts the bytes
    written, against the per-corner form."""
    out = {}
    for name, s, bt, nu in configs:
        out[name] = measure_draw(stage, idx, vtx, V, sp, s, bt, nu, reps=reps, output="indexed", U=U)
    naive = out.get("naive")
    if naive:
        for r in out.values():
            r["speedup_vs_naive"] = naive["kernel_ms_p50"] / r["kernel_ms_p50"]
    return out


def plain_latency(stage, reps=50):
    """The small grid (64 x 64 vertices, 7,938 triangles, row-major, MVP):
    launch-latency bound, so the latency of one draw is reported: GPU time
    between events, and the host's time from the call to the completed draw."""
    import torch
    from paper_1805_08893_amd import vr
    from paper_1805_08893_amd import workloads as W
    mesh, sp = W.grid64_scan_mvp()
    idx = torch.from_numpy(mesh.indices.view(np.int32)).cuda()
    vtx = torch.from_numpy(mesh.vertices).cuda()
    out = {}
    for name, s, bt in (("naive", vr.VR_NAIVE, 1), ("static_sort_64", vr.VR_STATIC_SORT, 64)):
        r = measure_draw(stage, idx, vtx, mesh.num_verts, sp, s, bt, reps=reps)
        res = stage.alloc_outputs(mesh.num_tris, s, bt, corners=True)
        sh = vr.make_shader(sp)
        wall = []
        for _ in range(reps):
            t0 = time.perf_counter()
            stage.check(vr.vr_process_draw(stage.ctx, idx, vtx, sh, s, bt, None, stage.describe(res)))
            torch.cuda.synchronize()
            wall.append((time.perf_counter() - t0) * 1e3)
        r.update({"host_ms_p50": float(np.percentile(wall, 50)), "host_ms_p99": float(np.percentile(wall, 99))})
        out[name] = r
    stage.check(stage.sync()[0])
    return {"workload": "grid64_scan_mvp", "triangles": mesh.num_tris, "draws": out}


def heavy_orders(stage, reps=10):
    """The heavy shader on a large grid (2048 x 2048 vertices, 8,380,418
    triangles, normal offset with 64 iterations) in Hilbert and in fully
    random triangle order: naive, dynamic ballot (N_u 64 / N_pmax 85) and
    dynamic hash (256 / 341), with per-corner and with indexed outputs."""
    import torch
    from paper_1805_08893_amd import vr
    from paper_1805_08893_amd import workloads as W
    out = {}
    for order in ("hilbert", "random"):
        mesh, sp = W.grid2048_offset64(order)
        idx = torch.from_numpy(mesh.indices.view(np.int32)).cuda()
        vtx = torch.from_numpy(mesh.vertices).cuda()
        cfgs = (("naive", vr.VR_NAIVE, 1, 0), ("dyn_ballot", vr.VR_DYN_BALLOT, 85, 64),
                ("dyn_hash", vr.VR_DYN_HASH, 341, 256))
        out[order] = {name: measure_draw(stage, idx, vtx, mesh.num_verts, sp, s, bt, nu, reps=reps)
                      for name, s, bt, nu in cfgs}
        out[order]["indexed"] = {name: measure_draw(stage, idx, vtx, mesh.num_verts, sp, s, bt, nu, reps=reps,
                                                    output="indexed")
                                 for name, s, bt, nu in cfgs}
        del idx, vtx
        torch.cuda.empty_cache()
        progress(f"heavy {order} done")
    return {"workload": "grid2048_offset64", "triangles": 2 * 2047 * 2047, "orders": out}


def walk_benchmark(stage, steps=10, batch=512):
    """The parallel random walk (300,000 agents on 256 x 256, moves within
    16 cells, 8 options kept): 10 steps searching every agent's cell, and 10
    searching each distinct cell of 512-agent batches once; both must end
    with the same agents' cells."""
    import torch
    from paper_1805_08893_amd import vr
    from paper_1805_08893_amd import workloads as W
    s = W.walk_setup()
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a.view(np.int32) if a.dtype == np.uint32 else a)).cuda()
    act, mv, w = dev(s.activity), dev(s.moves), dev(s.weights)
    us = [dev(W.walk_uniforms(s.seed, k, len(s.keys))) for k in range(steps)]
    out, final = {}, {}
    for name, strat, b in (("naive", vr.VR_NAIVE, 0), (f"hash_{batch}", vr.VR_STATIC_HASH, batch)):
        keys = dev(s.keys)
        nxt = torch.empty_like(keys)
        cnt = torch.zeros((steps, 4), dtype=torch.int64, device="cuda")
        for k in range(2):   # warm-up
            stage.check(vr.vr_walk_step(stage.ctx, keys, act, s.grid, mv, w, us[k], strat, b, nxt))
        torch.cuda.synchronize()
        keys = dev(s.keys)
        vr.vr_set_kernel_timing(stage.ctx, True)
        vr.vr_kernel_times(stage.ctx)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for k in range(steps):
            stage.check(vr.vr_walk_step(stage.ctx, keys, act, s.grid, mv, w, us[k], strat, b, nxt, cnt[k]))
            keys, nxt = nxt, keys
        e1.record()
        torch.cuda.synchronize()
        kms = np.array(vr.vr_kernel_times(stage.ctx), dtype=np.float64)
        vr.vr_set_kernel_timing(stage.ctx, False)
        stage.check(stage.sync()[0])
        ev = cnt[:, 0].cpu().numpy()
        out[name] = {"ms_per_step": e0.elapsed_time(e1) / steps, "kernel_ms_per_step": float(kms.mean()),
                     "searches_per_step": ev.tolist(), "reuse_per_step": (1.0 - ev / len(s.keys)).round(4).tolist()}
        final[name] = keys.cpu().numpy()
    names = list(out)
    out["same_final_cells"] = bool(np.array_equal(final[names[0]], final[names[1]]))
    out["speedup"] = out["naive"]["ms_per_step"] / out[names[1]]["ms_per_step"]
    out.update(agents=len(s.keys), grid=s.grid, moves=int(len(s.weights)), steps=steps)
    return out


def stream_benchmark(stage, idx, vtx, sp, T, chunk=65536, reps=5):
    """The bench mesh streamed in 64K-triangle chunks with static ballot
    rounds (no analysis of the index buffer) through a ring of 1, 2 or 4
    corner buffers, triangle setup (1920 x 1080) consuming each buffer on a
    second HIP stream; against the whole mesh as one chunk.  Host wall time
    from the first push to both stages finished."""
    import torch
    from paper_1805_08893_amd import vr
    rec = torch.empty((T, 8), dtype=torch.float32, device="cuda")
    sh = vr.make_shader(sp)
    out = {}
    for name, slots, ch in (("whole", 1, T), ("ring1", 1, chunk), ("ring2", 2, chunk), ("ring4", 4, chunk)):
        times, vis = [], 0
        for _ in range(reps + 1):
            st, h = vr.vr_stream_create(stage.ctx, slots, ch, 1920, 1080, rec)
            stage.check(st)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for c0 in range(0, T, ch):
                c1 = min(T, c0 + ch)
                stage.check(vr.vr_stream_push(h, idx[3 * c0:3 * c1], vtx, sh, vr.VR_STATIC_BALLOT, 64))
            st, tris, vis, inv = vr.vr_stream_finish(h)
            times.append(time.perf_counter() - t0)
            vr.vr_stream_destroy(h)
            stage.check(st)
        t = float(np.median(times[1:]))
        out[name] = {"slots": slots, "chunk_tris": ch, "ms": t * 1e3, "tri_per_s": T / t, "visible": vis,
                     "invocations": inv}
    stage.check(stage.sync()[0])
    return out


def plan_probe(reps=20):
    """The dynamic planner alone (vr_plan_dynamic), timed by HIP events on the
    large icosphere (1,310,720 triangles) and the large grid (8,380,418
    triangles, Hilbert and random order) at the budgets the draws use."""
    import torch
    from paper_1805_08893_amd import vr
    from paper_1805_08893_amd import workloads as W
    stage = vr.GeometryStage(0)
    out = {}
    cases = [("icosphere8", None, [(256, 341), (256, 256), (64, 85), (1024, 1365), (4096, 4096)]),
             ("grid2048_hilbert", "hilbert", [(64, 85), (256, 341)]),
             ("grid2048_random", "random", [(256, 341), (64, 85), (2048, 2730)])]
    for name, order, budgets in cases:
        mesh = W.icosphere8_hilbert_phong8()[0] if order is None else W.grid2048_offset64(order)[0]
        idx = torch.from_numpy(mesh.indices.view(np.int32)).cuda()
        plan = torch.empty(mesh.num_tris + 2, dtype=torch.int32, device="cuda")
        for nu, npm in budgets:
            def run():
                stage.check(vr.vr_plan_dynamic(stage.ctx, idx, mesh.num_verts, nu, npm, plan))
            run()
            ms = []
            for _ in range(reps):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                run()
                e1.record()
                torch.cuda.synchronize()
                ms.append(e0.elapsed_time(e1))
            st, _ = stage.sync()
            stage.check(st)
            out[f"{name}_{nu}_{npm}"] = {"ms_p50": float(np.median(ms)), "batches": int(plan[0].item()),
                                         "triangles": mesh.num_tris}
            progress(f"plan probe {name} {nu}/{npm}: {np.median(ms):.4f} ms")
        del idx, plan
        torch.cuda.empty_cache()
    stage.close()
    return out


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


RATE_SWEEP = (4000.0, 16000.0, 64000.0)


def serving_benchmark(stage, seed=11, n=2000, rate=500.0, budget=64 << 30, small_budget=256 << 20):
    """A Poisson stream of draw requests against 200 resident meshes (sizes
    log-normal around 20k triangles, clamped to [1k, 2M]; a request draws a
    whole mesh with Phong lighting of 1..16 lights), served by the
    continuous-batching server and by the same server launching every
    request alone, at 500 requests/s and at the higher rates of RATE_SWEEP;
    a burst of the same requests for peak throughput; and the stream again
    under a 256 MB result budget (queueing and rejections)."""
    import torch
    from paper_1805_08893_amd import vr, serve
    from paper_1805_08893_amd import workloads as W
    from paper_1805_08893_amd.autotune import Autotuner

    bases = W.serving_bases(seed)
    pool = W.serving_pool(bases, seed + 1)
    tr = W.serving_trace(pool, seed + 2, n=n, rate=rate)
    dev = [(torch.from_numpy(m.indices.view(np.int32)).cuda(), torch.from_numpy(m.vertices).cuda()) for m in bases]
    shaders = {}
    tuner = Autotuner(stage.ctx)
    cfg_of = {}
    for i in range(n):
        m, L = int(tr["mesh"][i]), int(tr["lights"][i])
        b, start, size = pool[m]
        if (b, L) not in shaders:
            sp = W.shader_for_mesh(bases[b], W.SHADER_PHONG, seed + b, num_lights=L)
            shaders[(b, L)] = (sp, vr.make_shader(sp))
        if (m, L) not in cfg_of:
            idx = dev[b][0][3 * start:3 * (start + size)]
            host = bases[b].indices[3 * start:3 * (start + size)]
            cfg_of[(m, L)] = tuner.choose(idx, host, dev[b][1], shaders[(b, L)][0])[1]
    stage.check(stage.sync()[0])

    def requests(ids):
        out = []
        for i in range(n):
            m, L = int(tr["mesh"][i]), int(tr["lights"][i])
            s, bt, nu = cfg_of[(m, L)]
            out.append(vr.make_request(ids[m], pool[m][2], shaders[(pool[m][0], L)][1], s, bt, nu, user=i))
        return out

    def keep(srv):
        return {k: v for k, v in srv.stats().items()
                if k in ("ticks", "peak_reserved_bytes", "admission_blocked", "max_tick_draws", "max_pending",
                         "plan_bytes", "rejected")}

    def run(max_tick_draws):
        with serve.Server(budget, max_inflight=2, max_tick_draws=max_tick_draws) as srv:
            ids = [srv.add_mesh(dev[b][0][3 * start:3 * (start + size)], dev[b][1]) for b, start, size in pool]
            reqs = requests(ids)
            for r in reqs:                      # warm-up: builds and caches every plan
                srv.submit(r)
            srv.drain(n)
            t0 = time.perf_counter()
            srv.submit_many(reqs)               # burst: everything at once, in one call
            got = srv.drain(n)
            burst = serve.summarize(got, time.perf_counter() - t0)
            got, late, wall = serve.replay(srv, reqs, tr["arrival"])
            out = serve.summarize(got, wall)
            out["submit_late_ms_p99"] = float(np.percentile(late, 99) * 1e3)
            # the same stream at higher mean rates (arrival times scaled), up to
            # past what one launch per request sustains
            sweep = []
            for r in RATE_SWEEP:
                got, late, wall = serve.replay(srv, reqs, tr["arrival"] * (rate / r))
                sv = serve.summarize(got, wall)
                sweep.append({"rate_req_per_s": r, **{k: sv[k] for k in (
                    "tri_per_s", "req_per_s", "latency_ms_p50", "latency_ms_p99", "requests_per_tick")},
                    "submit_late_ms_p99": float(np.percentile(late, 99) * 1e3)})
            out["rate_sweep"] = sweep
            out["burst_tri_per_s"] = burst["tri_per_s"]
            out["burst_wall_s"] = burst["wall_s"]
            out["burst_requests_per_tick"] = burst["requests_per_tick"]
            out["stats"] = keep(srv)
            return out

    def run_small():
        with serve.Server(small_budget, max_inflight=2) as srv:
            ids = [srv.add_mesh(dev[b][0][3 * start:3 * (start + size)], dev[b][1]) for b, start, size in pool]
            reqs = requests(ids)
            rejected = []
            got, _, wall = serve.replay(srv, reqs, tr["arrival"], rejected=rejected)
            out = serve.summarize(got, wall)
            out["rejected_requests"] = len(rejected)
            # burst: admission waits for released results
            rej = []
            got, _, wall = serve.replay(srv, reqs, np.zeros(n), rejected=rej)
            b = serve.summarize(got, wall)
            out.update(burst_tri_per_s=b["tri_per_s"], burst_wall_s=b["wall_s"],
                       burst_queue_ms_p99=b["queue_ms_p99"], burst_latency_ms_p99=b["latency_ms_p99"])
            out["stats"] = keep(srv)
            return out

    progress("serving: configurations chosen")
    batched = run(1024)
    progress("serving: batched server done")
    single = run(1)
    progress("serving: per-request launches done")
    small = run_small()
    progress("serving: 256 MB budget done")
    sizes = np.array([p[2] for p in pool])
    return {"requests": n, "rate_req_per_s": rate, "mean_tris": float(tr["size"].mean()),
            "meshes": len(pool), "mesh_tris_p50": float(np.median(sizes)), "mesh_tris_max": int(sizes.max()),
            "budget_bytes": budget, "batched": batched, "per_request_launch": single,
            "budget_256MB": small}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-passes", type=int, default=3,
                    help="passes of the full step the one-thread CPU oracle times (about 5 s)")
    ap.add_argument("--cpu-mt-passes", type=int, default=12,
                    help="passes of the full step the all-threads CPU oracle times")
    ap.add_argument("--level", type=int, default=8, help="icosphere subdivision level")
    ap.add_argument("--only", default=None, help="run only this strategy in each step (profiling)")
    ap.add_argument("--no-scene", action="store_true", help="skip the many-draw frame measurement")
    ap.add_argument("--no-serve", action="store_true", help="skip the request-server measurement")
    ap.add_argument("--serve-requests", type=int, default=2000, metavar="N",
                    help="requests of the serving stream (30000 is the full 60 s at 500 requests/s)")
    ap.add_argument("--autotune-table", default=None, metavar="JSON",
                    help="scene: read the autotuner's choices from this file if it exists, else write them")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the cold-cache runs, the small-grid latency and the heavy-shader orders")
    ap.add_argument("--sweep", action="store_true",
                    help="time every strategy over batch sizes 32..1024 on the workload and exit")
    ap.add_argument("--plan-probe", action="store_true",
                    help="time the dynamic planner alone on the large icosphere and the large grid and exit")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="time a plain device-to-device copy of BYTES (counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: the geometry stage has no cross-GPU path "
              f"(asked for --gpus {args.gpus})", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1805_08893_amd import vr
    from paper_1805_08893_amd import workloads as W

    torch.cuda.set_device(0)
    if args.copy_probe:
        n = args.copy_probe // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        out = {"copy_bytes": args.copy_probe}
        for name, fn in (("copy", lambda: dst.copy_(src)), ("fill", lambda: dst.fill_(2.0))):
            for _ in range(args.warmup):
                fn()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(args.steps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / args.steps
            moved = (2 if name == "copy" else 1) * args.copy_probe
            out[name] = {"ms": ms, "GBps": moved / (ms * 1e-3) / 1e9}
        print(json.dumps(out), flush=True)
        return
    if args.plan_probe:
        print(json.dumps(plan_probe(reps=max(3, min(args.steps, 50)))), flush=True)
        return
    mesh, sp = W.icosphere8_hilbert_phong8(level=args.level)
    T, V = mesh.num_tris, mesh.num_verts
    if args.sweep:
        sweep(mesh, sp, reps=max(3, min(args.steps, 20)))
        return
    U = int(len(np.unique(mesh.indices)))
    idx = torch.from_numpy(mesh.indices.view(np.int32)).cuda()
    vtx = torch.from_numpy(mesh.vertices).cuda()
    stage = vr.GeometryStage(0)
    plan = torch.empty(T + 2, dtype=torch.int32, device="cuda")
    NU, NP = 256, 341   # the paper's dynamic setting: N_u = 256 binds before N_pmax = 341
    strategies = [("naive", vr.VR_NAIVE, 1, {}),
                  ("static_ballot", vr.VR_STATIC_BALLOT, 64, {}),
                  ("dyn_sort", vr.VR_DYN_SORT, NP, dict(max_unique=NU, plan=plan)),
                  ("dyn_hash", vr.VR_DYN_HASH, NP, dict(max_unique=NU, plan=plan)),
                  ("dyn_phash", vr.VR_DYN_PHASH, NP, dict(max_unique=NU, plan=plan))]
    if args.only:
        strategies = [s for s in strategies if s[0] == args.only]
        assert strategies, f"unknown strategy {args.only}"
    res = {name: stage.alloc_outputs(T, s, bt, corners=True) for name, s, bt, _ in strategies}
    opts = {name: vr.make_opts(**o) for name, _, _, o in strategies}
    shader = vr.make_shader(sp)
    stream = torch.cuda.current_stream()

    def step(events=None):
        if events is not None:
            events["plan"][0].record(stream)
        st = vr.vr_plan_dynamic(stage.ctx, idx, V, NU, NP, plan)
        stage.check(st)
        if events is not None:
            events["plan"][1].record(stream)
        for name, s, bt, _ in strategies:
            if events is not None:
                events[name][0].record(stream)
            stage.check(vr.vr_process_draw(stage.ctx, idx, vtx, shader, s, bt, opts[name],
                                           stage.describe(res[name])))
            if events is not None:
                events[name][1].record(stream)

    for _ in range(args.warmup):
        step()
    st, _ = stage.sync()
    stage.check(st)

    # the timed steps: nothing but the work of the step on the stream
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st, inv_total = stage.sync()
    stage.check(st)

    # the same steps again, instrumented: HIP events around every draw and
    # around every main kernel (breakdown and roofline only)
    names = ["plan"] + [s[0] for s in strategies]
    ev = [{n: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for n in names}
          for _ in range(args.steps)]
    vr.vr_set_kernel_timing(stage.ctx, True)
    vr.vr_kernel_times(stage.ctx)           # start from an empty record
    for k in range(args.steps):
        step(ev[k])
    torch.cuda.synchronize()
    ktimes = np.array(vr.vr_kernel_times(stage.ctx, cap=len(names) * args.steps + 16),
                      dtype=np.float64).reshape(args.steps, len(names))
    vr.vr_set_kernel_timing(stage.ctx, False)
    st, _ = stage.sync()
    stage.check(st)

    ms_step = (t1 - t0) * 1e3 / args.steps
    tris_step = T * len(strategies)
    value = tris_step / (ms_step * 1e-3)
    per = {}
    for j, n in enumerate(names):
        ms = [ev[k][n][0].elapsed_time(ev[k][n][1]) for k in range(args.steps)]
        per[n] = {"ms_mean": float(np.mean(ms)), "ms_p50": float(np.percentile(ms, 50)),
                  "ms_p99": float(np.percentile(ms, 99)), "kernel_ms_mean": float(ktimes[:, j].mean())}
    for name, s, bt, _ in strategies:
        inv = int(res[name]["counters"][0].item())
        p = per[name]
        p.update({"tri_per_s": T / (p["ms_mean"] * 1e-3), "invocations": inv, "shading_rate": inv / U,
                  "reuse": 1.0 - inv / (3.0 * T), "speedup_vs_naive": None})
    for name, *_ in strategies:
        per[name]["speedup_vs_naive"] = (per["naive"]["ms_mean"] / per[name]["ms_mean"]) if "naive" in per else None
        kms = per[name]["kernel_ms_mean"]
        per[name]["hbm_frac"] = (12 * T + 32 * U + 144 * T) / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS
        per[name]["alu_frac"] = per[name]["invocations"] * shader_flops(sp) / (kms * 1e-3) / 1e12 / FP32_VECTOR_PEAK_TFLOPS

    # dominant kernel: the main kernel of the slowest draw of the step, timed
    # with HIP events around its launch on the library's stream
    dom = max((s[0] for s in strategies), key=lambda n: per[n]["kernel_ms_mean"])
    dom_ms = per[dom]["kernel_ms_mean"]
    alg_bytes = 12 * T + 32 * U + 144 * T            # indices + each referenced vertex once + corners
    alg_flops = per[dom]["invocations"] * shader_flops(sp)
    gbs = alg_bytes / (dom_ms * 1e-3) / 1e9
    tfl = alg_flops / (dom_ms * 1e-3) / 1e12
    if gbs / HBM_PEAK_GBS >= tfl / FP32_VECTOR_PEAK_TFLOPS:
        roof = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS}
    else:
        roof = {"bound": "alu", "achieved": tfl, "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": tfl / FP32_VECTOR_PEAK_TFLOPS}
    roof.update({"traffic": committed_traffic(KERNEL_NAMES[dom]), "kernel": KERNEL_NAMES[dom], "draw": dom,
                 "bytes_per_launch": alg_bytes, "flops_per_launch": alg_flops, "ms_per_launch": dom_ms,
                 "hbm_frac": gbs / HBM_PEAK_GBS, "alu_frac": tfl / FP32_VECTOR_PEAK_TFLOPS,
                 "kernel_source_sha": kernel_source_sha()})

    cpu = None
    if not args.no_cpu:
        cpu = cpu_oracle_baseline(mesh, sp, [(n, s, bt, o.get("max_unique", 0)) for n, s, bt, o in strategies],
                                  args.cpu_passes, args.cpu_mt_passes)
        progress("CPU oracle done")

    cold = None
    if not args.only and not args.no_extra:
        # the same draws with the caches overwritten (1 GiB) before each one
        flush = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        cold = {name: measure_draw(stage, idx, vtx, V, sp, s, bt, o.get("max_unique", 0), reps=5, flush=flush)
                for name, s, bt, o in strategies}
        del flush
        torch.cuda.empty_cache()
        progress("cold runs done")
    indexed = sweep_rows = None
    if not args.only and not args.no_extra:
        try:
            indexed = indexed_outputs(stage, idx, vtx, V, U, sp,
                                      [("naive", vr.VR_NAIVE, 1, 0), ("static_ballot", vr.VR_STATIC_BALLOT, 64, 0),
                                       ("dyn_ballot", vr.VR_DYN_BALLOT, 85, 64), ("dyn_sort", vr.VR_DYN_SORT, NP, NU),
                                       ("dyn_hash", vr.VR_DYN_HASH, NP, NU), ("dyn_phash", vr.VR_DYN_PHASH, NP, NU),
                                       ("dyn_hash_4096", vr.VR_DYN_HASH, 4096, 4096),
                                       ("dyn_phash_4096", vr.VR_DYN_PHASH, 4096, 4096)])
            progress("indexed outputs done")
            sweep_rows = batch_sweep(stage, idx, vtx, V, U, sp)
            progress("batch sweep done")
        except Exception as exc:   # the headline line must still be printed
            indexed = {"error": repr(exc)}
    multi = None
    if not args.only and not args.no_extra:
        # the two-pass reference (shade the vertex buffer, then gather)
        multi = measure_draw(stage, idx, vtx, V, sp, vr.VR_MULTI, 1, reps=20)
        multi["speedup_vs_naive"] = per["naive"]["kernel_ms_mean"] / multi["kernel_ms_p50"]
        multi["dyn_hash_speedup"] = multi["kernel_ms_p50"] / per["dyn_hash"]["kernel_ms_mean"]
        progress("two-pass reference done")
    plain = heavy = None
    if not args.only and not args.no_extra:
        try:
            plain = plain_latency(stage)
            heavy = heavy_orders(stage)
        except Exception as exc:   # the headline line must still be printed
            heavy = {"error": repr(exc)}
    stream = None
    if not args.only and not args.no_extra:
        try:
            stream = stream_benchmark(stage, idx, vtx, sp, T)
            progress("streaming done")
        except Exception as exc:   # the headline line must still be printed
            stream = {"error": repr(exc)}
    walk = None
    if not args.only and not args.no_extra:
        try:
            walk = walk_benchmark(stage)
            progress("random walk done")
        except Exception as exc:   # the headline line must still be printed
            walk = {"error": repr(exc)}
    scene = None
    if not args.no_scene and not args.only:
        try:
            scene = scene_benchmark(stage, table=args.autotune_table)
            progress("scene done")
        except Exception as exc:   # the headline line must still be printed
            scene = {"error": repr(exc)}
    serving = None
    if not args.no_serve and not args.only:
        try:
            serving = serving_benchmark(stage, n=args.serve_requests)
        except Exception as exc:
            serving = {"error": repr(exc)}

    line = {"metric": METRIC, "value": value, "unit": "triangles/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"icosphere{args.level}_hilbert_swap5_phong8", "triangles": T, "vertices": V,
                       "unique_vertices": U, "strategies": [s[0] for s in strategies],
                       "static_batch_tris": 64, "dynamic_max_unique": NU, "dynamic_max_tris": NP,
                       "output": "per-corner shaded vertices + invocation counters"},
            "roofline": roof, "cpu_baseline": cpu, "per_strategy": per, "indexed": indexed, "sweep": sweep_rows,
            "multi": multi, "cold": cold, "plain": plain, "heavy": heavy, "stream": stream, "walk": walk, "scene": scene,
            "serving": serving}
    print(json.dumps(line), flush=True)
    stage.close()


if __name__ == "__main__":
    main()
