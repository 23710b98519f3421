"""The two-pass reference (shade the whole vertex buffer, then gather the
corners) on the GPU, through the C ABI, against the CPU oracle: corners and
shaded vertices bitwise, assembled indices, the single unit and counters
exactly; unreferenced vertices are shaded too; argument rules."""
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


def _dev(a):
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    return torch.from_numpy(a).cuda()


def _run(stage, idx, vb, sp, outputs=True):
    from paper_1805_08893_amd import vr
    res = stage.alloc_outputs(len(idx) // 3, vr.VR_MULTI, 1, corners=True, tris=outputs, verts=outputs,
                              units=outputs, num_vertices=len(vb))
    st = vr.vr_process_draw(stage.ctx, _dev(idx), _dev(vb), vr.make_shader(sp), vr.VR_MULTI, 1, None,
                            stage.describe(res))
    assert st == vr.VR_OK, vr.vr_last_error(stage.ctx)
    st, inv = stage.sync()
    assert st == vr.VR_OK, vr.vr_last_error(stage.ctx)
    return {k: v.cpu().numpy() for k, v in res.items()}, inv


CASES = [("grid 41x37 hilbert, phong-5, 29 unreferenced", lambda: W.grid_mesh(41, 37, 5, "hilbert"), W.SHADER_PHONG, 29),
         ("icosphere 4 scan, mvp", lambda: W.icosphere_mesh(4, 6, "scan"), W.SHADER_MVP, 0),
         ("grid 33x33 random, offset-16, 1 unreferenced", lambda: W.grid_mesh(33, 33, 8, "random"), W.SHADER_OFFSET, 1)]


@pytest.mark.parametrize("name,make,kind,extra", CASES, ids=[c[0] for c in CASES])
def test_multi_matches_oracle(stage, name, make, kind, extra):
    print(f"[multi] {name}", flush=True)
    m = make()
    rng = np.random.default_rng(len(name))
    vb = np.concatenate([m.vertices, rng.random((extra, 8), dtype=np.float32)]) if extra else m.vertices
    sp = W.shader_for_mesh(m, kind, 9, num_lights=5, iterations=16)
    got, inv = _run(stage, m.indices, vb, sp)
    rc, ora = vro.process_draw(m.indices, vb, sp, vro.MULTI, 1)
    assert rc == vro.OK
    V, T = len(vb), m.num_tris
    assert got["counters"][:2].tolist() == [V, 1] and inv == V
    assert got["unit_offsets"][:2].tolist() == [0, T] and got["unit_invocations"][:1].tolist() == [V]
    np.testing.assert_array_equal(got["tris"].view(np.uint32), ora["tris"])
    np.testing.assert_array_equal(got["corners"].view(np.uint32), ora["corners"].view(np.uint32))
    np.testing.assert_array_equal(got["verts"][:V].view(np.uint32), ora["verts"].view(np.uint32))


def test_multi_ragged_sizes_and_empty(stage):
    """Vertex counts that are not multiples of the 256-vertex block, a
    triangle count whose float4 rows end mid-block, and the empty draw."""
    m = W.grid_mesh(23, 19, 4, "scan")   # 437 vertices, 792 triangles
    sp = W.shader_for_mesh(m, W.SHADER_PHONG, 4, num_lights=2)
    for T in (1, 85, 792):
        idx = m.indices[:3 * T]
        got, inv = _run(stage, idx, m.vertices, sp, outputs=False)
        rc, ora = vro.process_draw(idx, m.vertices, sp, vro.MULTI, 1)
        assert inv == m.num_verts and got["counters"][:2].tolist() == [m.num_verts, 1]
        np.testing.assert_array_equal(got["corners"].view(np.uint32), ora["corners"].view(np.uint32))
    got, inv = _run(stage, np.zeros(0, np.uint32), m.vertices, sp, outputs=False)
    assert inv == 0 and got["counters"].tolist() == [0, 0, 0, 0]


def test_multi_bench_size_sampled(stage):
    """The bench mesh (1,310,720 triangles): sampled corners against the
    oracle's shading of their vertices, and equality with the dynamic hash
    draw's corners everywhere."""
    from paper_1805_08893_amd import vr
    m, sp = W.icosphere8_hilbert_phong8()
    got, inv = _run(stage, m.indices, m.vertices, sp, outputs=False)
    assert inv == m.num_verts
    rng = np.random.default_rng(8)
    ks = rng.integers(0, 3 * m.num_tris, 2000)
    ref = vro.shade(sp, m.vertices[m.indices[ks]])
    np.testing.assert_array_equal(got["corners"][ks].view(np.uint32), ref.view(np.uint32))
    r = stage.draw(_dev(m.indices), _dev(m.vertices), sp, vr.VR_DYN_HASH, 256, dict(max_unique=256), corners=True)
    st, _ = stage.sync()
    assert st == vr.VR_OK
    assert np.array_equal(r["corners"].cpu().numpy().view(np.uint32), got["corners"].view(np.uint32))


def test_multi_argument_rules(stage):
    from paper_1805_08893_amd import vr
    m = W.grid_mesh(9, 9, 1, "scan")
    sp = vr.make_shader(W.shader_for_mesh(m, W.SHADER_MVP, 1))
    idx, vtx = _dev(m.indices), _dev(m.vertices)
    res = stage.alloc_outputs(m.num_tris, vr.VR_MULTI, 1, corners=True, local_idx=True)
    assert vr.vr_process_draw(stage.ctx, idx, vtx, sp, vr.VR_MULTI, 1, None, stage.describe(res)) == vr.VR_ERR_ARG
    small = stage.alloc_outputs(m.num_tris, vr.VR_MULTI, 1, corners=True)
    small["verts"] = torch.empty((m.num_verts - 1, 12), dtype=torch.float32, device="cuda")   # V - 1 < 3T rows
    assert m.num_verts - 1 < 3 * m.num_tris
    assert vr.vr_process_draw(stage.ctx, idx, vtx, sp, vr.VR_MULTI, 1, None,
                              stage.describe(small)) == vr.VR_ERR_CAPACITY
    corners = torch.empty((3 * m.num_tris, 12), dtype=torch.float32, device="cuda")
    d = vr.make_draw(idx, vtx, 0, vr.VR_MULTI, 1, corners)
    st, _ = vr.vr_frame_create(stage.ctx, [d], [sp], capture_graph=False)
    assert st == vr.VR_ERR_ARG
    from paper_1805_08893_amd.serve import Server
    with Server(64 << 20) as srv:                        # the server serves streaming strategies only
        mid = srv.add_mesh(idx, vtx)
        assert vr.vr_server_submit(srv.h, vr.make_request(mid, m.num_tris, W.shader_for_mesh(m, W.SHADER_MVP, 1),
                                                          vr.VR_MULTI, 1))[0] == vr.VR_ERR_ARG
    bad = m.indices.copy()
    bad[5] = m.num_verts
    got = stage.alloc_outputs(m.num_tris, vr.VR_MULTI, 1, corners=True)
    assert vr.vr_process_draw(stage.ctx, _dev(bad), vtx, sp, vr.VR_MULTI, 1, None, stage.describe(got)) == vr.VR_OK
    st, _ = stage.sync()
    assert st == vr.VR_ERR_INDEX_RANGE
