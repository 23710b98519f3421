"""Large dynamic batches (unique budgets and primitive caps up to 4096)
through the C ABI against the CPU oracle: the device planner's classes for
caps above 512, per-corner draws whose shaded vertices fill most of the LDS,
draws with indexed outputs only (the shaded vertices stream out through a
one-row-per-thread stage), and the configurations that do not fit one
workgroup, which are argument errors raised before any launch."""
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


def _plan_meshes():
    ordered = W.grid_mesh(150, 120, 8, "hilbert")
    mixed = W.Mesh("hilbert_then_random",
                   np.concatenate([ordered.indices, W.grid_mesh(150, 120, 8, "random").indices]), ordered.vertices)
    return (W.icosphere_mesh(6, 8, "hilbert", swap_frac=0.05), W.grid_mesh(200, 180, 8, "random"), mixed)


@pytest.mark.parametrize("nu,tmax", [(1024, 1365), (700, 1000), (2048, 2048), (64, 2048), (2730, 3640),
                                     (4096, 4096), (3, 4096), (1000, 600)])
def test_plan_parity_large_caps(stage, nu, tmax):
    """Plans of every primitive-cap class above 512 equal the sequential
    greedy chain, on an ordered, a random and a half-ordered stream (several
    segments, composition levels and the aligned check failing part way)."""
    from paper_1805_08893_amd import vr
    for mesh in _plan_meshes():
        _log(f"case plan nu={nu} tmax={tmax} mesh={mesh.name} T={mesh.num_tris}")
        exp = vro.plan_dynamic(mesh.indices, mesh.num_verts, nu, tmax)
        idx = _dev(mesh.indices)
        plan = torch.empty(mesh.num_tris + 2, dtype=torch.int32, device="cuda")
        assert vr.vr_plan_dynamic(stage.ctx, idx, mesh.num_verts, nu, tmax, plan) == vr.VR_OK
        st, _ = stage.sync()
        assert st == vr.VR_OK, vr.vr_last_error(stage.ctx)
        got = plan.cpu().numpy().view(np.uint32)
        B = int(got[0])
        assert B == len(exp) - 1, (B, len(exp) - 1)
        np.testing.assert_array_equal(got[1:B + 2], exp)


def _draw_meshes():
    return (W.icosphere_mesh(5, 21, "hilbert", swap_frac=0.05), W.grid_mesh(90, 70, 21, "random"))


def _compare(g, o, want):
    n_inv, n_units = int(o["counters"][0]), int(o["counters"][1])
    assert int(g["counters"][0]) == n_inv and int(g["counters"][1]) == n_units
    if "corners" in want:
        assert np.array_equal(g["corners"].view(np.uint32), o["corners"].view(np.uint32))
    if "tris" in want:
        assert np.array_equal(g["tris"].view(np.uint32), o["tris"])
    if "verts" in want:
        assert np.array_equal(g["verts"][:n_inv].view(np.uint32), o["verts"].view(np.uint32))
    if "local_idx" in want:
        assert np.array_equal(g["local_idx"].view(np.uint16), o["local_idx"])
    if "units" in want:
        assert np.array_equal(g["unit_offsets"][:n_units + 1].view(np.uint32), o["unit_offsets"])
        assert np.array_equal(g["unit_invocations"][:n_units].view(np.uint32), o["unit_invocations"])


def _run(stage, mesh, sp, strategy, bt, nu, want, **opts):
    from paper_1805_08893_amd import vr
    kw = {k: (k in want) for k in ("corners", "tris", "verts", "local_idx", "units")}
    rc, o = vro.process_draw(mesh.indices, mesh.vertices, sp, strategy, bt, vro.make_opts(max_unique=nu), **kw)
    assert rc == vro.OK
    res = stage.draw(_dev(mesh.indices), _dev(mesh.vertices), sp, strategy, bt, dict(max_unique=nu, **opts), **kw)
    st, inv = stage.sync()
    assert st == vr.VR_OK, vr.vr_last_error(stage.ctx)
    assert inv == int(o["counters"][0])
    _compare({k: v.cpu().numpy() for k, v in res.items()}, o, want)


PER_CORNER = [("dyn_hash_1365_1024", vro.DYN_HASH, 1365, 1024), ("dyn_phash_2048_2048", vro.DYN_PHASH, 2048, 2048),
              ("dyn_hash_2730_2048", vro.DYN_HASH, 2730, 2048), ("dyn_sort_2048_2048", vro.DYN_SORT, 2048, 2048),
              ("dyn_sort_1365_1024", vro.DYN_SORT, 1365, 1024), ("dyn_ballot_4096_64", vro.DYN_BALLOT, 4096, 64),
              ("dyn_ballot_4096_4096", vro.DYN_BALLOT, 4096, 4096)]


@pytest.mark.parametrize("sname,strategy,bt,nu", PER_CORNER, ids=[s[0] for s in PER_CORNER])
def test_large_units_per_corner(stage, sname, strategy, bt, nu):
    """Every output, per-corner vertices included, bitwise."""
    for mi, mesh in enumerate(_draw_meshes()):
        kind = (W.SHADER_PHONG, W.SHADER_MVP)[mi]
        sp = W.shader_for_mesh(mesh, kind, 50 + mi, num_lights=8)
        _log(f"case large per-corner {sname} mesh={mesh.name} T={mesh.num_tris}")
        _run(stage, mesh, sp, strategy, bt, nu, ("corners", "tris", "verts", "local_idx", "units"))


INDEXED = [("dyn_hash_4096_4096", vro.DYN_HASH, 4096, 4096), ("dyn_phash_4096_4096", vro.DYN_PHASH, 4096, 4096),
           ("dyn_hash_4096_3000", vro.DYN_HASH, 4096, 3000), ("dyn_sort_2048_2048", vro.DYN_SORT, 2048, 2048),
           ("dyn_hash_341_256", vro.DYN_HASH, 341, 256), ("dyn_sort_341_256", vro.DYN_SORT, 341, 256),
           ("static_hash_64", vro.STATIC_HASH, 64, 0), ("dyn_phash_85_64", vro.DYN_PHASH, 85, 64)]


@pytest.mark.parametrize("sname,strategy,bt,nu", INDEXED, ids=[s[0] for s in INDEXED])
def test_indexed_outputs_only(stage, sname, strategy, bt, nu):
    """Without corners the shaded vertices stream out in workgroup-sized
    chunks after the unit's offset is known; verts, tris, local ids and unit
    arrays bitwise, and with verts alone."""
    for mi, mesh in enumerate(_draw_meshes()):
        sp = W.shader_for_mesh(mesh, W.SHADER_PHONG, 60 + mi, num_lights=4)
        _log(f"case indexed-only {sname} mesh={mesh.name} T={mesh.num_tris}")
        _run(stage, mesh, sp, strategy, bt, nu, ("tris", "verts", "local_idx", "units"))
        _run(stage, mesh, sp, strategy, bt, nu, ("verts",), wg_size=64)


def test_configurations_beyond_one_workgroup_are_argument_errors(stage):
    """Per-corner hashing of 4096 unique vertices needs 192 KB of shaded
    vertices; a sort of 12,288 indices needs more than 1024 threads; a frame
    runs 256 threads per unit.  All are VR_ERR_ARG before any launch, and the
    context keeps working."""
    from paper_1805_08893_amd import vr
    mesh = W.grid_mesh(40, 40, 3, "hilbert")
    sp = W.shader_for_mesh(mesh, W.SHADER_MVP, 3)
    idx, vtx = _dev(mesh.indices), _dev(mesh.vertices)
    T = mesh.num_tris
    for strategy, bt, nu, corners in ((vr.VR_DYN_HASH, 4096, 4096, True), (vr.VR_DYN_SORT, 4096, 4096, False),
                                      (vr.VR_DYN_PHASH, 4096, 3500, True)):
        res = stage.alloc_outputs(T, strategy, bt, corners=corners, verts=True)
        st = vr.vr_process_draw(stage.ctx, idx, vtx, vr.make_shader(sp), strategy, bt,
                                vr.make_opts(max_unique=nu), stage.describe(res))
        assert st == vr.VR_ERR_ARG, (strategy, bt, nu, st)
    corners = torch.empty((3 * T, 12), dtype=torch.float32, device="cuda")
    plan = torch.empty(T + 2, dtype=torch.int32, device="cuda")
    assert vr.vr_plan_dynamic(stage.ctx, idx, mesh.num_verts, 1024, 1024, plan) == vr.VR_OK
    d = vr.make_draw(idx, vtx, 0, vr.VR_DYN_SORT, 1024, corners, max_unique=1024, plan=plan)
    rc, _ = vr.vr_frame_create(stage.ctx, [d], [sp])
    assert rc == vr.VR_ERR_ARG
    st, _ = stage.sync()
    assert st == vr.VR_OK
    _run(stage, mesh, sp, vro.DYN_HASH, 1024, 1024, ("corners", "tris"))
