"""Colliding keys through the LDS hash tables, against the oracle.

Algorithm 3 probes linearly from h(k) = (k * 0x9E3779B1 mod 2^32) >> (32 - b)
in a table of 2^b slots; parallel hashing (Section 3.4) gives each lane a
few probes and hands the rest to the whole wavefront.  These streams use
only vertex indices whose top 10 hash bits agree, so every key of a unit
starts probing at the same slot for any table of up to 1024 slots: each
insertion walks the chain of all earlier keys, the tables run at load factor
up to 1 (hash_slots = the smallest power of two the unit allows), and the
cooperative path, including its retry after a lost slot, carries most keys.
Hash-table slots never show in the outputs: corners, assembled indices,
local ids, unit offsets and per-unit invocation counts must equal the
oracle's bit for bit.
"""
import numpy as np
import pytest

from oracle import vro
from paper_1805_08893_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from test_gpu_parity import compare, gpu_draw  # noqa: E402


@pytest.fixture(scope="module")
def stage():
    from paper_1805_08893_amd import vr
    s = vr.GeometryStage(0)
    yield s
    s.close()


def _colliding(V, bits=10, target=37):
    k = np.arange(V, dtype=np.uint64)
    top = ((k * np.uint64(0x9E3779B1)) & np.uint64(0xFFFFFFFF)) >> np.uint64(32 - bits)
    return np.nonzero(top == target)[0].astype(np.uint32)


@pytest.fixture(scope="module")
def streams():
    V = 1 << 20
    pool = _colliding(V)
    assert len(pool) >= 900
    rng = np.random.default_rng(91)
    verts = np.zeros((V, 8), np.float32)
    verts[:, :3] = rng.uniform(-1, 1, (V, 3)).astype(np.float32)
    verts[:, 3:6] = np.float32([0.0, 0.6, 0.8])
    verts[:, 6:] = rng.uniform(0, 1, (V, 2)).astype(np.float32)
    T = 4000
    # sliding window over the pool: about two new keys per triangle, so a
    # dynamic batch fills its unique budget exactly (a full table) and static
    # batches hold distinct keys with repeats
    slide = 2 * np.arange(T)[:, None] + rng.integers(0, 8, (T, 3))
    sliding = pool[slide % len(pool)].ravel()
    # every key distinct: static batches at 3 N_p distinct keys
    distinct = pool[np.arange(3 * 300) % len(pool)]
    return {"sliding": W.Mesh("colliding_sliding", sliding.astype(np.uint32), verts),
            "distinct": W.Mesh("colliding_distinct", distinct.astype(np.uint32), verts)}


def _pow2(x):
    p = 1
    while p < x:
        p *= 2
    return p


CASES = [
    # (strategy, batch_tris, max_unique); the table is the smallest power of
    # two >= N_u (dynamic) or >= 3 N_p (static)
    (vro.STATIC_HASH, 64, 0),
    (vro.STATIC_HASH, 85, 0),
    (vro.STATIC_HASH, 256, 0),
    (vro.DYN_HASH, 341, 256),
    (vro.DYN_HASH, 512, 512),
    (vro.DYN_HASH, 100, 64),
    (vro.DYN_PHASH, 341, 256),
    (vro.DYN_PHASH, 512, 512),
    (vro.DYN_PHASH, 100, 64),
]


@pytest.mark.parametrize("strategy,bt,nu", CASES, ids=[f"{vro.STRATEGY_NAMES[s]}_{b}_{u}" for s, b, u in CASES])
@pytest.mark.parametrize("which", ["sliding", "distinct"])
def test_colliding_keys_match_oracle(stage, streams, strategy, bt, nu, which):
    mesh = streams[which]
    sp = W.shader_for_mesh(W.grid_mesh(8, 8, 3), W.SHADER_PHONG, 5, num_lights=2)
    rc, ora = vro.process_draw(mesh.indices, mesh.vertices, sp, strategy, bt, {"max_unique": nu})
    assert rc == vro.OK
    need = nu if strategy != vro.STATIC_HASH else 3 * bt
    full = _pow2(need)
    if strategy != vro.STATIC_HASH and which == "sliding":
        # the budget binds: units hold exactly N_u keys (a full table)
        assert int(ora["unit_invocations"].max()) == nu
    for slots in (full, 0):
        for probes in ((1, 0) if strategy == vro.DYN_PHASH else (0,)):
            print(f"case colliding {which} s={vro.STRATEGY_NAMES[strategy]} bt={bt} nu={nu} "
                  f"slots={slots} probes={probes}", flush=True)
            gpu = gpu_draw(stage, mesh, sp, strategy, bt, nu, hash_slots=slots, hash_probes=probes)
            compare(gpu, ora)
