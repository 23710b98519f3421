"""The allocation-free draw (vr_process_draw_noalloc) against vr_process_draw.

Both are called through the C ABI on the same inputs; every output (corners,
assembled indices, shaded vertices, local ids, unit offsets and invocations,
counters) must be bitwise equal, and equal to the oracle's.  Each strategy
runs twice in a row, the second time on a smaller draw, so the second call
finds the static scratch as the first left it.
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


def _dev(a):
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    return torch.from_numpy(a).cuda()


CASES = [("naive", vro.NAIVE, 1, 0), ("static_ballot_64", vro.STATIC_BALLOT, 64, 0),
         ("static_sort_64", vro.STATIC_SORT, 64, 0), ("static_hash_128", vro.STATIC_HASH, 128, 0),
         ("dyn_sort_256_256", vro.DYN_SORT, 256, 256), ("dyn_hash_341_256", vro.DYN_HASH, 341, 256),
         ("dyn_phash_341_256", vro.DYN_PHASH, 341, 256), ("dyn_ballot_85_64", vro.DYN_BALLOT, 85, 64),
         ("multi", vro.MULTI, 1, 0)]


@pytest.mark.parametrize("name,strategy,bt,nu", CASES, ids=[c[0] for c in CASES])
def test_noalloc_equals_process_draw(stage, name, strategy, bt, nu):
    from paper_1805_08893_amd import vr
    base = W.icosphere_mesh(5, 21, "hilbert", swap_frac=0.05)
    sp = W.shader_for_mesh(base, W.SHADER_PHONG, 21, num_lights=4)
    vtx = _dev(base.vertices)
    for T in (base.num_tris, 7001):          # the second call is smaller
        ind = base.indices[:3 * T]
        idx = _dev(ind)
        plan = None
        if strategy in (vro.DYN_SORT, vro.DYN_HASH, vro.DYN_PHASH, vro.DYN_BALLOT):
            plan = torch.empty(T + 2, dtype=torch.int32, device="cuda")
            assert vr.vr_plan_dynamic(stage.ctx, idx, base.num_verts, nu, bt, plan) == vr.VR_OK
        opts = vr.make_opts(max_unique=nu, plan=plan)
        want = dict(corners=True, tris=True, verts=True, local_idx=strategy != vro.MULTI, units=True,
                    num_vertices=base.num_verts)
        ref = stage.alloc_outputs(T, strategy, bt, **want)
        got = stage.alloc_outputs(T, strategy, bt, **want)
        for t in got.values():
            t.fill_(-7)                      # stale contents must not leak through
        print(f"case noalloc {name} T={T}", flush=True)
        stage.check(vr.vr_process_draw(stage.ctx, idx, vtx, sp, strategy, bt, opts, stage.describe(ref)))
        stage.check(vr.vr_process_draw_noalloc(stage.ctx, idx, vtx, sp, strategy, bt, opts, stage.describe(got)))
        st, _ = stage.sync()
        assert st == vr.VR_OK, vr.vr_last_error(stage.ctx)
        inv, units = int(ref["counters"][0].item()), int(ref["counters"][1].item())
        rc, ora = vro.process_draw(ind, base.vertices, sp, strategy, bt, {"max_unique": nu},
                                   local_idx=strategy != vro.MULTI)
        assert rc == vro.OK
        assert inv == int(ora["counters"][0]) and units == int(ora["counters"][1])
        np.testing.assert_array_equal(got["counters"].cpu().numpy(), ref["counters"].cpu().numpy())
        np.testing.assert_array_equal(got["corners"].cpu().numpy().view(np.uint32),
                                      ora["corners"].view(np.uint32))
        np.testing.assert_array_equal(got["tris"].cpu().numpy().view(np.uint32), ora["tris"])
        np.testing.assert_array_equal(got["verts"][:inv].cpu().numpy().view(np.uint32),
                                      ora["verts"].view(np.uint32))
        if strategy != vro.MULTI:
            np.testing.assert_array_equal(got["local_idx"].cpu().numpy().view(np.uint16), ora["local_idx"])
        np.testing.assert_array_equal(got["unit_offsets"][:units + 1].cpu().numpy().view(np.uint32),
                                      ora["unit_offsets"])
        np.testing.assert_array_equal(got["unit_invocations"][:units].cpu().numpy().view(np.uint32),
                                      ora["unit_invocations"])
        for k in ("corners", "tris", "local_idx"):
            if k in ref:
                assert torch.equal(got[k], ref[k]), k


def test_noalloc_rejects_what_it_cannot_hold(stage):
    """Rejections happen on the host, before anything is enqueued: a draw
    with more batches than the static array holds, a dynamic draw without
    its plan, MULTI without its shaded buffer."""
    from paper_1805_08893_amd import vr
    T = 524288 + 1
    idx = torch.zeros(3 * T, dtype=torch.int32, device="cuda")      # valid indices (all 0)
    vtx = _dev(W.grid_mesh(2, 2, 1).vertices)
    sp = W.make_shader(W.SHADER_MVP, 1)
    res = stage.alloc_outputs(T, vr.VR_STATIC_HASH, 1, corners=True)
    res["counters"].fill_(5)
    st = vr.vr_process_draw_noalloc(stage.ctx, idx, vtx, sp, vr.VR_STATIC_HASH, 1, None, stage.describe(res))
    assert st == vr.VR_ERR_CAPACITY
    st = vr.vr_process_draw_noalloc(stage.ctx, idx[:300], vtx, sp, vr.VR_DYN_HASH, 64, vr.make_opts(max_unique=64),
                                    stage.describe(res))
    assert st == vr.VR_ERR_ARG
    st = vr.vr_process_draw_noalloc(stage.ctx, idx[:300], vtx, sp, vr.VR_MULTI, 1, None, stage.describe(res))
    assert st == vr.VR_ERR_ARG
    assert stage.sync()[0] == vr.VR_OK
    assert res["counters"].cpu().tolist() == [5, 5, 5, 5]            # nothing ran
