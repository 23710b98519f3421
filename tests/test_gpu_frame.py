"""Frames: many draws in one persistent launch, eager and as a hipGraph.

Every draw of a frame must produce exactly what the single-draw path
produces for it (corners bit for bit, counters equal); a subset is also
compared with the oracle directly.  Graph replays are checked one by one
with unrelated eager work between them.
"""
import numpy as np
import pytest

from oracle import vro
from paper_1805_08893_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _dev(a):
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    return torch.from_numpy(a).cuda()


@pytest.fixture(scope="module")
def stage():
    from paper_1805_08893_amd import vr
    s = vr.GeometryStage(0)
    yield s
    s.close()


def _scene(seed=3):
    """Draws over a few base meshes (prefixes of uneven size), every strategy,
    three shaders."""
    rng = np.random.default_rng(seed)
    bases = [W.grid_mesh(41, 37, 5, "hilbert"), W.icosphere_mesh(4, 6, "hilbert", swap_frac=0.05),
             W.icosphere_mesh(3, 7, "random"), W.grid_mesh(30, 30, 8, "scan")]
    shaders = [W.shader_for_mesh(bases[1], W.SHADER_MVP, 1), W.shader_for_mesh(bases[1], W.SHADER_PHONG, 2, num_lights=4),
               W.shader_for_mesh(bases[0], W.SHADER_PHONG, 3, num_lights=16),
               W.shader_for_mesh(bases[0], W.SHADER_OFFSET, 4, iterations=64)]
    strats = [(vro.NAIVE, 1, 0), (vro.STATIC_BALLOT, 64, 0), (vro.STATIC_BALLOT, 200, 0), (vro.STATIC_SORT, 64, 0),
              (vro.STATIC_HASH, 128, 0), (vro.DYN_SORT, 256, 256), (vro.DYN_HASH, 341, 256), (vro.DYN_PHASH, 128, 128),
              (vro.DYN_BALLOT, 85, 64), (vro.DYN_HASH, 33, 100)]
    draws = []
    for i in range(36):
        m = bases[i % len(bases)]
        T = int(rng.integers(0, m.num_tris + 1)) if i % 9 else 0   # some empty draws
        s, bt, nu = strats[i % len(strats)]
        draws.append(dict(mesh=m, T=T, strategy=s, bt=bt, nu=nu, shader=int(rng.integers(0, len(shaders)))))
    return bases, shaders, draws


def _build(stage, bases, shaders, draws):
    from paper_1805_08893_amd import vr
    dev = {id(m): (_dev(m.indices), _dev(m.vertices)) for m in bases}
    entries, outs = [], []
    for d in draws:
        idx, vtx = dev[id(d["mesh"])]
        idx = idx[:3 * d["T"]]
        plan = None
        if d["strategy"] in vr.DYNAMIC:
            plan = torch.empty(d["T"] + 2, dtype=torch.int32, device="cuda")
            assert vr.vr_plan_dynamic(stage.ctx, idx, d["mesh"].num_verts, d["nu"], d["bt"], plan) == vr.VR_OK
        corners = torch.zeros((3 * d["T"], 12), dtype=torch.float32, device="cuda")
        counters = torch.full((4,), 7, dtype=torch.int64, device="cuda")
        entries.append(vr.make_draw(idx, vtx, d["shader"], d["strategy"], d["bt"], corners, counters, d["nu"], plan))
        outs.append(dict(idx=idx, vtx=vtx, plan=plan, corners=corners, counters=counters))
    return entries, outs


def _reference(stage, shaders, draws, outs):
    from paper_1805_08893_amd import vr
    refs = []
    for d, o in zip(draws, outs):
        r = stage.draw(o["idx"], o["vtx"], shaders[d["shader"]], d["strategy"], d["bt"],
                       dict(max_unique=d["nu"], plan=o["plan"]), corners=True)
        refs.append(r)
    st, inv = stage.sync()
    assert st == vr.VR_OK
    return refs, inv


def _check(outs, refs):
    for i, (o, r) in enumerate(zip(outs, refs)):
        assert torch.equal(o["corners"].view(torch.int32), r["corners"].view(torch.int32)), f"draw {i} corners"
        assert o["counters"][:2].tolist() == r["counters"][:2].tolist(), f"draw {i} counters"


def test_frame_matches_single_draws_and_oracle(stage):
    from paper_1805_08893_amd import vr
    bases, shaders, draws = _scene()
    entries, outs = _build(stage, bases, shaders, draws)
    refs, inv_ref = _reference(stage, shaders, draws, outs)
    assert vr.vr_process_draws(stage.ctx, entries, shaders) == vr.VR_OK
    st, inv = stage.sync()
    assert st == vr.VR_OK and inv == inv_ref
    _check(outs, refs)
    for i in (1, 3, 6, 8):   # direct oracle comparison for a few draws
        d = draws[i]
        rc, ora = vro.process_draw(d["mesh"].indices[:3 * d["T"]], d["mesh"].vertices, shaders[d["shader"]],
                                   d["strategy"], d["bt"], {"max_unique": d["nu"]}, tris=False, verts=False,
                                   local_idx=False, units=False)
        np.testing.assert_array_equal(outs[i]["corners"].cpu().numpy().view(np.uint32), ora["corners"].view(np.uint32))
        assert outs[i]["counters"][:2].tolist() == [int(ora["counters"][0]), int(ora["counters"][1])]


def test_frame_graph_replays(stage):
    from paper_1805_08893_amd import vr
    bases, shaders, draws = _scene(seed=11)
    entries, outs = _build(stage, bases, shaders, draws)
    refs, inv_ref = _reference(stage, shaders, draws, outs)
    rc, frame = vr.vr_frame_create(stage.ctx, entries, shaders, capture_graph=True)
    assert rc == vr.VR_OK, vr.vr_last_error(stage.ctx)
    try:
        for rep in range(3):
            for o in outs:
                o["corners"].zero_()
                o["counters"].fill_(9)
            # unrelated eager work between replays
            other = stage.draw(outs[1]["idx"], outs[1]["vtx"], shaders[0], vr.VR_STATIC_HASH, 64, corners=True)
            torch.cuda.synchronize()
            assert vr.vr_frame_run(frame) == vr.VR_OK
            st, inv = stage.sync()
            assert st == vr.VR_OK
            assert inv == inv_ref + int(other["counters"][0].item())
            _check(outs, refs)
    finally:
        vr.vr_frame_destroy(frame)


def test_frame_argument_errors(stage):
    from paper_1805_08893_amd import vr
    bases, shaders, draws = _scene(seed=5)
    entries, outs = _build(stage, bases, shaders, draws)
    dyn = next(i for i, d in enumerate(draws) if d["strategy"] in vr.DYNAMIC and d["T"] > 0)
    bad = list(entries)
    bad[dyn] = vr.vr_draw(entries[dyn].d_indices, entries[dyn].num_indices, entries[dyn].d_vertices,
                          entries[dyn].num_vertices, entries[dyn].shader, entries[dyn].strategy,
                          entries[dyn].batch_tris, entries[dyn].max_unique, None, entries[dyn].d_corners, None)
    assert vr.vr_process_draws(stage.ctx, bad, shaders) == vr.VR_ERR_ARG
    bad = list(entries)
    bad[0] = vr.vr_draw(entries[0].d_indices, entries[0].num_indices, entries[0].d_vertices, entries[0].num_vertices,
                        len(shaders), entries[0].strategy, entries[0].batch_tris, 0, None, entries[0].d_corners, None)
    assert vr.vr_process_draws(stage.ctx, bad, shaders) == vr.VR_ERR_ARG
    assert vr.vr_process_draws(stage.ctx, [], shaders) == vr.VR_OK
    assert stage.sync()[0] == vr.VR_OK


def test_frame_plan_with_more_batches_than_reserved_is_capacity_error(stage):
    """A dynamic draw whose plan was built with a smaller N_u than the draw
    states has more batches than the frame reserved aggregate slots for: the
    frame raises VR_ERR_CAPACITY instead of writing past them, and the
    context works normally afterwards."""
    from paper_1805_08893_amd import vr
    mesh = W.grid_mesh(60, 60, 5, "random")
    sp = W.shader_for_mesh(mesh, W.SHADER_MVP, 5)
    idx, vtx = _dev(mesh.indices), _dev(mesh.vertices)
    small = torch.empty(mesh.num_tris + 2, dtype=torch.int32, device="cuda")
    assert vr.vr_plan_dynamic(stage.ctx, idx, mesh.num_verts, 3, 341, small) == vr.VR_OK
    assert stage.sync()[0] == vr.VR_OK
    B = int(small[0].item())
    assert B > mesh.num_tris // 85 + 1          # beyond the bound for N_u = 256, N_pmax = 341
    corners = torch.empty((3 * mesh.num_tris, 12), dtype=torch.float32, device="cuda")
    d = vr.make_draw(idx, vtx, 0, vr.VR_DYN_HASH, 341, corners, max_unique=256, plan=small)
    print("case frame foreign plan", flush=True)
    rc, fr = vr.vr_frame_create(stage.ctx, [d], [sp])
    assert rc == vr.VR_OK, vr.vr_last_error(stage.ctx)
    assert vr.vr_frame_run(fr) == vr.VR_OK
    st, _ = stage.sync()
    vr.vr_frame_destroy(fr)
    assert st == vr.VR_ERR_CAPACITY
    # the same draw with its own plan afterwards is exact
    plan = torch.empty(mesh.num_tris + 2, dtype=torch.int32, device="cuda")
    assert vr.vr_plan_dynamic(stage.ctx, idx, mesh.num_verts, 256, 341, plan) == vr.VR_OK
    d = vr.make_draw(idx, vtx, 0, vr.VR_DYN_HASH, 341, corners, max_unique=256, plan=plan)
    assert vr.vr_process_draws(stage.ctx, [d], [sp]) == vr.VR_OK
    st, _ = stage.sync()
    assert st == vr.VR_OK
    rc, ora = vro.process_draw(mesh.indices, mesh.vertices, sp, vro.DYN_HASH, 341, {"max_unique": 256},
                               tris=False, verts=False, local_idx=False, units=False)
    np.testing.assert_array_equal(corners.cpu().numpy().view(np.uint32), ora["corners"].view(np.uint32))
