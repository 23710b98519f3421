"""Reuse of parallel per-processor caches against batching (the analogue of
the paper's Table 1, Section 4.1) on the synthetic meshes, from the CPU
oracle only.  Test infrastructure like the rest of oracle/: it prints a
markdown table and touches no GPU.

    python -m oracle.reuse_table

Parallel caches: 256 processors (MI355X compute units), 2,048 vertex
invocations per processor and cycle (32 resident wave64 wavefronts), LRU
caches of 16, 32 and 64 KB holding 48-byte shaded vertices (341, 682 and
1,365 entries), chunks dealt in consecutive runs.  Batching: static ballot
rounds with 32-triangle batches (96 indices, the paper's warp setting) and
64-triangle batches, and dynamic batches with N_u = 256, N_pmax = 341.
"""
import numpy as np

from oracle import vro
from paper_1805_08893_amd import workloads as W

PROCS, PER_CYCLE = 256, 2048
ENTRIES = {"16KB": 16384 // 48, "32KB": 32768 // 48, "64KB": 65536 // 48}


def meshes():
    yield "icosphere k=8, Hilbert + 5% swaps", W.icosphere8_hilbert_phong8()[0]
    yield "icosphere k=8, scan", W.icosphere_mesh(8, 3, "scan")
    yield "grid 1024x1024, scan", W.grid_mesh(1024, 1024, 11, "scan")
    yield "grid 2048x2048, Hilbert", W.grid2048_offset64("hilbert")[0]
    yield "grid 2048x2048, random", W.grid2048_offset64("random")[0]
    yield "grid 64x64, scan", W.grid64_scan_mvp()[0]


def reuse(m, strategy, bt, nu=0):
    sp = W.make_shader(W.SHADER_MVP, 0)
    rc, o = vro.process_draw(m.indices, m.vertices, sp, strategy, bt, vro.make_opts(max_unique=nu), corners=False,
                             tris=False, verts=False, local_idx=False, units=False)
    assert rc == vro.OK
    return 1.0 - int(o["counters"][0]) / len(m.indices)


def main():
    print("| mesh | vert | tris | ideal | cache 16KB | cache 32KB | cache 64KB | ballot 32 | ballot 64 | dyn 256/341 |")
    print("|---|---|---|---|---|---|---|---|---|---|")
    for name, m in meshes():
        n = len(m.indices)
        ideal = 1.0 - len(np.unique(m.indices)) / n
        cache = [vro.parallel_cache_hits(m.indices, m.num_verts, PROCS, PER_CYCLE, e) / n for e in ENTRIES.values()]
        row = [ideal, *cache, reuse(m, vro.STATIC_BALLOT, 32), reuse(m, vro.STATIC_BALLOT, 64),
               reuse(m, vro.DYN_HASH, 341, 256)]
        print(f"| {name} | {m.num_verts:,} | {m.num_tris:,} | " + " | ".join(f"{x:.3f}" for x in row) + " |",
              flush=True)


if __name__ == "__main__":
    main()
