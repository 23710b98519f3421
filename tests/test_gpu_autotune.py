"""Autotuner: candidate timing through the C ABI and per-class choices."""
import json

import numpy as np
import pytest

from paper_1805_08893_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def stage():
    from paper_1805_08893_amd import vr
    s = vr.GeometryStage(0)
    yield s
    s.close()


def test_autotune_times_every_candidate(stage):
    from paper_1805_08893_amd import vr
    from paper_1805_08893_amd.autotune import DEFAULT_CANDIDATES, vr_autotune
    m = W.icosphere_mesh(5, 3, "hilbert", swap_frac=0.05)
    sp = W.shader_for_mesh(m, W.SHADER_PHONG, 3, num_lights=8)
    idx = torch.from_numpy(m.indices.view(np.int32)).cuda()
    vtx = torch.from_numpy(m.vertices).cuda()
    cands = list(DEFAULT_CANDIDATES) + [(vr.VR_STATIC_SORT, 300, 0)]   # the last one is invalid
    best, rows = vr_autotune(stage.ctx, idx, vtx, sp, cands)
    assert rows[-1]["kernel_ms"] < 0
    valid = [r for r in rows[:-1]]
    assert all(r["kernel_ms"] > 0 for r in valid)
    assert rows[best]["kernel_ms"] == min(r["kernel_ms"] for r in valid)
    naive = rows[0]
    assert naive["invocations"] == 3 * m.num_tris
    assert all(r["invocations"] <= 3 * m.num_tris for r in valid)
    assert all(r["plan_ms"] > 0 for r in valid if r["strategy"] in vr.DYNAMIC)


def test_autotune_keeps_caller_state(stage):
    from paper_1805_08893_amd import vr
    from paper_1805_08893_amd.autotune import vr_autotune
    m = W.grid_mesh(40, 30, 2, "hilbert")
    sp = W.shader_for_mesh(m, W.SHADER_MVP, 2)
    idx = torch.from_numpy(m.indices.view(np.int32)).cuda()
    vtx = torch.from_numpy(m.vertices).cuda()
    r = stage.draw(idx, vtx, sp, vr.VR_STATIC_HASH, 64, corners=True)   # pending work of the caller
    vr_autotune(stage.ctx, idx, vtx, sp)
    st, inv = stage.sync()
    assert st == vr.VR_OK and inv == int(r["counters"][0].item())


def test_autotuner_classes_and_persistence(stage, tmp_path):
    from paper_1805_08893_amd.autotune import Autotuner
    a = W.grid_mesh(60, 60, 4, "hilbert")
    b = W.grid_mesh(60, 60, 4, "random")
    sp = W.shader_for_mesh(a, W.SHADER_PHONG, 4, num_lights=16)
    tuner = Autotuner(stage.ctx, path=str(tmp_path / "tune.json"))
    keys = []
    for m in (a, b, a):
        idx = torch.from_numpy(m.indices.view(np.int32)).cuda()
        vtx = torch.from_numpy(m.vertices).cuda()
        key, cfg = tuner.choose(idx, m.indices, vtx, sp)
        keys.append(key)
    assert keys[0] == keys[2] and keys[0] != keys[1]      # locality separates the orders
    tuner.save()
    again = Autotuner(stage.ctx, path=str(tmp_path / "tune.json"))
    assert set(again.table) == set(tuner.table)
    json.loads((tmp_path / "tune.json").read_text())
