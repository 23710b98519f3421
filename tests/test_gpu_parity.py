"""Parity of the HIP geometry stage (through the C ABI) with the CPU oracle.

Integer outputs (batch plans, unit offsets, per-unit invocations, local
ids, assembled indices, counters) must match bit for bit.  The FP32 shaded
vertices are compared bitwise as well: both sides evaluate the same FP32
operation sequence with contraction disabled, so the tolerance is zero; a
second, looser check (|a-b| <= 1e-6 * max(|a|, |b|, 1)) is reported in the
failure message to separate rounding slips from wrong results.
"""
import numpy as np
import pytest

from oracle import vro
from paper_1805_08893_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def stage():
    from paper_1805_08893_amd import vr
    s = vr.GeometryStage(0)
    yield s
    s.close()


def _log(msg):
    print(msg, flush=True)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _bits(a):
    return np.ascontiguousarray(a).view(np.uint32)


def _assert_float_bits(name, got, exp):
    if np.array_equal(_bits(got), _bits(exp)):
        return
    bad = np.argwhere(_bits(got) != _bits(exp))
    rel = np.abs(got.astype(np.float64) - exp) / np.maximum(1.0, np.maximum(np.abs(got), np.abs(exp)))
    raise AssertionError(f"{name}: {len(bad)} float words differ (first {bad[:4].tolist()}), "
                         f"max rel {rel.max():.3e}")


def gpu_draw(stage, mesh, shader, strategy, bt, nu=0, want_all=True, **opts):
    from paper_1805_08893_amd import vr
    idx, vtx = _dev(mesh.indices), _dev(mesh.vertices)
    res = stage.draw(idx, vtx, shader, strategy, bt, dict(max_unique=nu, **opts), corners=True, tris=want_all,
                     verts=want_all, local_idx=want_all, units=want_all)
    st, inv = stage.sync()
    assert st == vr.VR_OK, vr.vr_last_error(stage.ctx)
    out = {k: v.cpu().numpy() for k, v in res.items()}
    out["inv_total"] = inv
    return out


def compare(gpu, ora, check_floats=True):
    oc = ora["counters"]
    inv, units = int(oc[0]), int(oc[1])
    assert int(gpu["counters"][0]) == inv, (int(gpu["counters"][0]), inv)
    assert int(gpu["counters"][1]) == units, (int(gpu["counters"][1]), units)
    assert gpu["inv_total"] == inv
    if "unit_offsets" in gpu:
        np.testing.assert_array_equal(gpu["unit_offsets"][:units + 1].view(np.uint32), ora["unit_offsets"])
        np.testing.assert_array_equal(gpu["unit_invocations"][:units].view(np.uint32), ora["unit_invocations"])
    if "local_idx" in gpu:
        np.testing.assert_array_equal(gpu["local_idx"].view(np.uint16), ora["local_idx"])
    if "tris" in gpu:
        np.testing.assert_array_equal(gpu["tris"].view(np.uint32), ora["tris"])
    if check_floats:
        _assert_float_bits("corners", gpu["corners"], ora["corners"])
        if "verts" in gpu:
            _assert_float_bits("verts", gpu["verts"][:inv], ora["verts"])


def _meshes_small():
    rng = np.random.default_rng(17)
    out = [W.grid_mesh(23, 19, 5, "hilbert"), W.icosphere_mesh(4, 6, "hilbert", swap_frac=0.05),
           W.icosphere_mesh(3, 6, "random")]
    V = 500
    out.append(W.Mesh("random_v500", rng.integers(0, V, 3 * 3001).astype(np.uint32),
                      W.grid_mesh(25, 20, 9).vertices))
    out.append(W.Mesh("all_equal", np.full(3 * 777, 7, np.uint32), W.grid_mesh(4, 4, 9).vertices))
    out.append(W.Mesh("all_distinct", np.arange(3 * 1000, dtype=np.uint32) % 3000,
                      W.grid_mesh(60, 50, 9).vertices))
    out.append(W.Mesh("one_tri_last_vertex", np.array([0, 15, 15], np.uint32), W.grid_mesh(4, 4, 9).vertices))
    return out


STRATS = [
    ("naive", vro.NAIVE, 1, 0),
    ("static_ballot_64", vro.STATIC_BALLOT, 64, 0),
    ("static_ballot_7", vro.STATIC_BALLOT, 7, 0),
    ("static_ballot_1024", vro.STATIC_BALLOT, 1024, 0),
    ("static_sort_64", vro.STATIC_SORT, 64, 0),
    ("static_sort_256", vro.STATIC_SORT, 256, 0),
    ("static_sort_5", vro.STATIC_SORT, 5, 0),
    ("static_hash_64", vro.STATIC_HASH, 64, 0),
    ("static_hash_200", vro.STATIC_HASH, 200, 0),
    ("dyn_sort_341_256", vro.DYN_SORT, 341, 256),
    ("dyn_sort_5_3", vro.DYN_SORT, 5, 3),
    ("dyn_hash_341_256", vro.DYN_HASH, 341, 256),
    ("dyn_hash_512_512", vro.DYN_HASH, 512, 512),
    ("dyn_hash_33_100", vro.DYN_HASH, 33, 100),
    ("dyn_phash_341_256", vro.DYN_PHASH, 341, 256),
    ("dyn_phash_128_128", vro.DYN_PHASH, 128, 128),
    ("dyn_ballot_85_64", vro.DYN_BALLOT, 85, 64),
    ("dyn_ballot_200_150", vro.DYN_BALLOT, 200, 150),
    # the largest configurations each strategy accepts
    ("static_hash_256", vro.STATIC_HASH, 256, 0),
    ("dyn_sort_512_512", vro.DYN_SORT, 512, 512),
    ("dyn_phash_512_512", vro.DYN_PHASH, 512, 512),
    ("dyn_ballot_512_64", vro.DYN_BALLOT, 512, 64),
]


@pytest.mark.parametrize("sname,strategy,bt,nu", STRATS, ids=[s[0] for s in STRATS])
def test_parity_small_meshes(stage, sname, strategy, bt, nu):
    for mi, mesh in enumerate(_meshes_small()):
        kind = [W.SHADER_MVP, W.SHADER_PHONG, W.SHADER_OFFSET][mi % 3]
        sp = W.shader_for_mesh(mesh, kind, 40 + mi, num_lights=8 if kind == W.SHADER_PHONG else 0,
                               iterations=64)
        _log(f"case {sname} mesh={mesh.name} T={mesh.num_tris} kind={kind}")
        rc, ora = vro.process_draw(mesh.indices, mesh.vertices, sp, strategy, bt, {"max_unique": nu})
        assert rc == vro.OK
        gpu = gpu_draw(stage, mesh, sp, strategy, bt, nu)
        compare(gpu, ora)


def test_parity_corners_only_mode(stage):
    """Without indexed outputs the kernels skip the prefix pass."""
    mesh = W.icosphere_mesh(4, 3, "hilbert", swap_frac=0.05)
    sp = W.shader_for_mesh(mesh, W.SHADER_PHONG, 3, num_lights=8)
    for sname, strategy, bt, nu in STRATS:
        _log(f"case corners-only {sname}")
        rc, ora = vro.process_draw(mesh.indices, mesh.vertices, sp, strategy, bt, {"max_unique": nu})
        gpu = gpu_draw(stage, mesh, sp, strategy, bt, nu, want_all=False)
        compare(gpu, ora)


@pytest.mark.parametrize("nu,tmax", [(3, 5), (64, 85), (256, 341), (512, 512), (100, 33), (7, 512)])
def test_plan_parity(stage, nu, tmax):
    from paper_1805_08893_amd import vr
    ordered = W.grid_mesh(120, 90, 8, "hilbert")
    mixed = W.Mesh("hilbert_then_random",
                   np.concatenate([ordered.indices, W.grid_mesh(120, 90, 8, "random").indices]), ordered.vertices)
    for mesh in (W.icosphere_mesh(6, 8, "hilbert", swap_frac=0.05), W.grid_mesh(160, 150, 8, "random"),
                 W.grid_mesh(97, 31, 8, "scan"), mixed):
        _log(f"case plan nu={nu} tmax={tmax} mesh={mesh.name} T={mesh.num_tris}")
        exp = vro.plan_dynamic(mesh.indices, mesh.num_verts, nu, tmax)
        idx = _dev(mesh.indices)
        plan = torch.empty(mesh.num_tris + 2, dtype=torch.int32, device="cuda")
        st = vr.vr_plan_dynamic(stage.ctx, idx, mesh.num_verts, nu, tmax, plan)
        assert st == vr.VR_OK
        st, _ = stage.sync()
        assert st == vr.VR_OK
        got = plan.cpu().numpy().view(np.uint32)
        B = int(got[0])
        assert B == len(exp) - 1, (B, len(exp) - 1)
        np.testing.assert_array_equal(got[1:B + 2], exp)


def test_plan_reuse_matches_inline_plan(stage):
    from paper_1805_08893_amd import vr
    mesh = W.icosphere_mesh(5, 3, "hilbert", swap_frac=0.05)
    sp = W.shader_for_mesh(mesh, W.SHADER_MVP, 3)
    idx, vtx = _dev(mesh.indices), _dev(mesh.vertices)
    plan = torch.empty(mesh.num_tris + 2, dtype=torch.int32, device="cuda")
    assert vr.vr_plan_dynamic(stage.ctx, idx, mesh.num_verts, 256, 341, plan) == vr.VR_OK
    a = stage.draw(idx, vtx, sp, vr.VR_DYN_HASH, 341, dict(max_unique=256, plan=plan), corners=True, tris=True)
    b = stage.draw(idx, vtx, sp, vr.VR_DYN_HASH, 341, dict(max_unique=256), corners=True, tris=True)
    assert stage.sync()[0] == vr.VR_OK
    assert torch.equal(a["corners"], b["corners"]) and torch.equal(a["tris"], b["tris"])


def test_launch_shape_never_changes_results(stage):
    """Workgroup size, hash-table size and probe count change the launch
    only: every shape gives the oracle's outputs bit for bit, and hash and
    parallel hash give the same ids."""
    mesh = W.icosphere_mesh(4, 12, "random")
    sp = W.shader_for_mesh(mesh, W.SHADER_MVP, 12)
    ref = None
    for strategy in (vro.DYN_HASH, vro.DYN_PHASH, vro.DYN_SORT):
        rc, ora = vro.process_draw(mesh.indices, mesh.vertices, sp, strategy, 341, {"max_unique": 256})
        assert rc == vro.OK
        for wg, slots, probes in ((0, 0, 0), (64, 256, 1), (512, 4096, 64), (128, 256, 0)):
            _log(f"case shape s={strategy} wg={wg} slots={slots} probes={probes}")
            g = gpu_draw(stage, mesh, sp, strategy, 341, 256, wg_size=wg, hash_slots=slots, hash_probes=probes)
            compare(g, ora)
            if strategy == vro.DYN_SORT:
                continue
            if ref is None:
                ref = g
            for k in ("corners", "tris", "local_idx", "unit_offsets", "unit_invocations"):
                np.testing.assert_array_equal(g[k], ref[k])


def test_repeat_runs_bitwise_identical(stage):
    mesh = W.icosphere_mesh(5, 14, "hilbert", swap_frac=0.05)
    sp = W.shader_for_mesh(mesh, W.SHADER_PHONG, 14, num_lights=4)
    for strategy, bt, nu in ((vro.DYN_PHASH, 341, 256), (vro.STATIC_BALLOT, 256, 0)):
        a = gpu_draw(stage, mesh, sp, strategy, bt, nu)
        for _ in range(3):
            b = gpu_draw(stage, mesh, sp, strategy, bt, nu)
            for k in ("corners", "tris", "verts", "unit_offsets"):
                np.testing.assert_array_equal(a[k], b[k])


def test_index_out_of_range_reported(stage):
    from paper_1805_08893_amd import vr
    mesh = W.grid_mesh(10, 10, 1, "scan")
    bad = mesh.indices.copy()
    bad[100] = mesh.num_verts          # one past the end
    sp = W.shader_for_mesh(mesh, W.SHADER_MVP, 1)
    for strategy, bt, nu in ((vro.NAIVE, 1, 0), (vro.STATIC_SORT, 64, 0), (vro.DYN_HASH, 64, 64),
                             (vro.STATIC_BALLOT, 64, 0)):
        stage.draw(_dev(bad), _dev(mesh.vertices), sp, strategy, bt, dict(max_unique=nu), corners=True)
        st, _ = stage.sync()
        assert st == vr.VR_ERR_INDEX_RANGE
        # the error is cleared: a valid draw after it succeeds
        gpu_draw(stage, mesh, sp, strategy, bt, nu)


def test_empty_draw(stage):
    from paper_1805_08893_amd import vr
    idx = torch.zeros(0, dtype=torch.int32, device="cuda")
    vtx = _dev(W.grid_mesh(3, 3, 1).vertices)
    sp = W.make_shader(W.SHADER_MVP, 1)
    res = stage.draw(idx, vtx, sp, vr.VR_DYN_SORT, 64, corners=True, units=True)
    res["counters"].fill_(5)
    stage.draw(idx, vtx, sp, vr.VR_DYN_SORT, 64, res=res)
    st, inv = stage.sync()
    assert st == vr.VR_OK and inv == 0
    assert res["counters"].cpu().tolist() == [0, 0, 0, 0]
    assert int(res["unit_offsets"][0]) == 0


FULL = [("naive", vro.NAIVE, 1, 0), ("static_ballot_64", vro.STATIC_BALLOT, 64, 0),
        ("static_sort_64", vro.STATIC_SORT, 64, 0), ("static_hash_128", vro.STATIC_HASH, 128, 0),
        ("dyn_sort_256_256", vro.DYN_SORT, 256, 256), ("dyn_hash_341_256", vro.DYN_HASH, 341, 256),
        ("dyn_phash_341_256", vro.DYN_PHASH, 341, 256), ("dyn_ballot_85_64", vro.DYN_BALLOT, 85, 64)]


@pytest.fixture(scope="module")
def ico8():
    return W.icosphere8_hilbert_phong8()


@pytest.mark.parametrize("sname,strategy,bt,nu", FULL, ids=[s[0] for s in FULL])
def test_parity_full_icosphere8_phong8(stage, ico8, sname, strategy, bt, nu):
    """The full 1,310,720-triangle draw: every output compared bitwise."""
    mesh, sp = ico8
    _log(f"case full icosphere8 {sname}")
    rc, ora = vro.process_draw(mesh.indices, mesh.vertices, sp, strategy, bt, {"max_unique": nu})
    gpu = gpu_draw(stage, mesh, sp, strategy, bt, nu)
    compare(gpu, ora)


BENCH = [("naive", vro.NAIVE, 1, 0), ("static_ballot_64", vro.STATIC_BALLOT, 64, 0),
         ("dyn_sort_256_256", vro.DYN_SORT, 256, 256), ("dyn_hash_256_256", vro.DYN_HASH, 256, 256),
         ("dyn_phash_256_256", vro.DYN_PHASH, 256, 256)]


@pytest.mark.parametrize("sname,strategy,bt,nu", BENCH, ids=[s[0] for s in BENCH])
def test_parity_bench_launch_configuration(stage, ico8, sname, strategy, bt, nu):
    """The draws exactly as bench.py times them: corners and counters only,
    dynamic draws with a plan built by vr_plan_dynamic (their units come from
    the context's counters), twice in a row; corners bitwise."""
    from paper_1805_08893_amd import vr
    mesh, sp = ico8
    _log(f"case bench configuration {sname}")
    rc, ora = vro.process_draw(mesh.indices, mesh.vertices, sp, strategy, bt, {"max_unique": nu},
                               tris=False, verts=False, local_idx=False, units=False)
    assert rc == vro.OK
    idx, vtx = _dev(mesh.indices), _dev(mesh.vertices)
    plan = None
    if strategy >= vro.DYN_SORT:
        plan = torch.empty(mesh.num_tris + 2, dtype=torch.int32, device="cuda")
        assert vr.vr_plan_dynamic(stage.ctx, idx, mesh.num_verts, nu, bt, plan) == vr.VR_OK
    for rep in range(2):
        res = stage.draw(idx, vtx, sp, strategy, bt, vr.make_opts(max_unique=nu, plan=plan), corners=True)
        st, inv = stage.sync()
        assert st == vr.VR_OK, vr.vr_last_error(stage.ctx)
        assert inv == int(ora["counters"][0]) and int(res["counters"][0].item()) == inv
        assert int(res["counters"][1].item()) == int(ora["counters"][1])
        np.testing.assert_array_equal(res["corners"].cpu().numpy().view(np.uint32),
                                      ora["corners"].view(np.uint32))


def test_sort_wide_and_narrow_index_spans(stage):
    """The sort's radix passes depend on each batch's index span (one pass
    per 8 bits).  A stream of uniform random indices over 3M vertices (spans
    of 22 bits: three passes), followed by a grid in Hilbert order (one or
    two passes), has both kinds in one draw."""
    V = 3_000_000
    rng = np.random.default_rng(17)
    wide = rng.integers(0, V, 3 * 6000, dtype=np.uint32)
    grid = W.grid_mesh(60, 50, 5, "hilbert")
    verts = np.zeros((V, 8), dtype=np.float32)
    verts[:, :3] = rng.uniform(-1, 1, (V, 3)).astype(np.float32)
    verts[:, 3:6] = np.float32(0.57735026)
    verts[:grid.num_verts] = grid.vertices
    mesh = W.Mesh("wide_then_narrow", np.concatenate([wide, grid.indices]), verts)
    sp = W.shader_for_mesh(grid, W.SHADER_MVP, 5)
    for sname, strategy, bt, nu in (("static_sort_64", vro.STATIC_SORT, 64, 0),
                                    ("static_sort_256", vro.STATIC_SORT, 256, 0),
                                    ("dyn_sort_341_256", vro.DYN_SORT, 341, 256)):
        _log(f"case sort spans {sname}")
        rc, ora = vro.process_draw(mesh.indices, mesh.vertices, sp, strategy, bt, {"max_unique": nu})
        assert rc == vro.OK
        compare(gpu_draw(stage, mesh, sp, strategy, bt, nu), ora)
