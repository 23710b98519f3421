"""Streaming (draw chunks as they arrive, triangle setup on a second HIP
stream, a bounded ring of corner buffers) through the C ABI against the CPU
oracle: every record bitwise, the visible and invocation totals exactly,
for ragged chunks, one to three ring buffers and each static strategy;
argument rules."""
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


def _oracle(m, sp, chunks, strategy, bt, width, height):
    recs, vis, inv, t0 = [], 0, 0, 0
    for T in chunks:
        idx = m.indices[3 * t0:3 * (t0 + T)]
        rc, o = vro.process_draw(idx, m.vertices, sp, strategy, bt, corners=True, tris=False, verts=False,
                                 local_idx=False, units=False)
        assert rc == vro.OK
        r, v = vro.setup(o["corners"], width, height)
        recs.append(r)
        vis += v
        inv += int(o["counters"][0])
        t0 += T
    return np.concatenate(recs), vis, inv


@pytest.mark.parametrize("slots,strategy,bt", [(1, "naive", 1), (2, "static_ballot", 64), (3, "static_hash", 128),
                                               (2, "static_sort", 64)])
def test_stream_matches_oracle(stage, slots, strategy, bt):
    from paper_1805_08893_amd import vr
    print(f"[stream] slots {slots} {strategy}", flush=True)
    m = W.icosphere_mesh(5, 4, "hilbert")
    sp = W.shader_for_mesh(m, W.SHADER_PHONG, 6, num_lights=3)
    chunks = [4096, 1000, 4096, 1, 3333, 4096, m.num_tris - (4096 * 3 + 1000 + 1 + 3333)]
    gs, os_ = vr.STRATEGIES[strategy], vro.STRATEGY_NAMES.index(strategy)
    idx, vtx = _dev(m.indices), _dev(m.vertices)
    rec = torch.zeros((m.num_tris, 8), dtype=torch.float32, device="cuda")
    st, h = vr.vr_stream_create(stage.ctx, slots, 4096, 1280, 720, rec)
    assert st == vr.VR_OK, vr.vr_last_error(stage.ctx)
    try:
        t0 = 0
        for T in chunks:
            st = vr.vr_stream_push(h, idx[3 * t0:3 * (t0 + T)], vtx, sp, gs, bt)
            assert st == vr.VR_OK, vr.vr_last_error(stage.ctx)
            t0 += T
        st, tris, vis, inv = vr.vr_stream_finish(h)
        assert st == vr.VR_OK
    finally:
        vr.vr_stream_destroy(h)
    s, _ = stage.sync()
    assert s == vr.VR_OK
    ref, rvis, rinv = _oracle(m, sp, chunks, os_, bt, 1280, 720)
    assert tris == m.num_tris and vis == rvis and inv == rinv
    np.testing.assert_array_equal(rec.cpu().numpy().view(np.uint32), ref.view(np.uint32))


def test_stream_argument_rules(stage):
    from paper_1805_08893_amd import vr
    m = W.grid_mesh(9, 9, 1, "scan")
    sp = W.shader_for_mesh(m, W.SHADER_MVP, 1)
    idx, vtx = _dev(m.indices), _dev(m.vertices)
    rec = torch.zeros((m.num_tris, 8), dtype=torch.float32, device="cuda")
    assert vr.vr_stream_create(stage.ctx, 0, 64, 100, 100, rec)[0] == vr.VR_ERR_ARG
    assert vr.vr_stream_create(stage.ctx, 9, 64, 100, 100, rec)[0] == vr.VR_ERR_ARG
    st, h = vr.vr_stream_create(stage.ctx, 2, 64, 100, 100, rec)
    assert st == vr.VR_OK
    try:
        assert vr.vr_stream_push(h, idx[:3 * 65], vtx, sp, vr.VR_NAIVE, 1) == vr.VR_ERR_ARG       # above chunk_tris
        assert vr.vr_stream_push(h, idx[:3 * 64], vtx, sp, vr.VR_DYN_HASH, 64) == vr.VR_ERR_ARG   # needs a plan
        assert vr.vr_stream_push(h, idx[:3 * 64], vtx, sp, vr.VR_STATIC_HASH, 64) == vr.VR_OK
        assert vr.vr_stream_push(h, idx[:3 * 64], vtx, sp, vr.VR_STATIC_HASH, 64) == vr.VR_OK
        assert vr.vr_stream_push(h, idx[:3 * 64], vtx, sp, vr.VR_STATIC_HASH, 64) == vr.VR_ERR_CAPACITY  # 192 > 128
        st, tris, vis, inv = vr.vr_stream_finish(h)
        assert st == vr.VR_OK and tris == 128
    finally:
        vr.vr_stream_destroy(h)
    assert stage.sync()[0] == vr.VR_OK
