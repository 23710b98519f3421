"""Seeded random configurations through the C ABI against the CPU oracle:
mesh family and order, size (ragged against every batch size), strategy,
batch size and unique budget anywhere in their ranges, shader kind and
output subset.  Every output the case requests must match bitwise."""
import numpy as np
import pytest

from oracle import vro
from paper_1805_08893_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CASES = 48


@pytest.fixture(scope="module")
def stage():
    from paper_1805_08893_amd import vr
    s = vr.GeometryStage(0)
    yield s
    s.close()


def _case(seed):
    rng = np.random.default_rng(1000 + seed)
    fam = rng.integers(0, 3)
    if fam == 0:
        m = W.grid_mesh(int(rng.integers(3, 40)), int(rng.integers(3, 40)), seed, ["scan", "hilbert", "random"][rng.integers(0, 3)])
    elif fam == 1:
        m = W.icosphere_mesh(int(rng.integers(0, 5)), seed, ["scan", "hilbert", "random"][rng.integers(0, 3)])
    else:
        V = int(rng.integers(3, 600))
        T = int(rng.integers(1, 1500))
        m = W.Mesh("random_indices", rng.integers(0, V, 3 * T).astype(np.uint32), W.grid_mesh(25, 25, seed).vertices[:V])
    T = int(rng.integers(0, m.num_tris + 1))   # a prefix, possibly empty
    idx = m.indices[:3 * T]
    strategy = int(rng.integers(0, 8))
    cap = {0: 1000, 1: 1024, 2: 256, 3: 256}.get(strategy, 512)
    bt = int(rng.integers(1, cap + 1))
    nu = int(rng.integers(3, 513)) if strategy >= 4 else 0
    kind = int(rng.integers(0, 3))
    sp = W.shader_for_mesh(m, kind, seed, num_lights=int(rng.integers(0, 17)), iterations=int(rng.integers(0, 20)))
    want = dict(tris=bool(rng.integers(0, 2)), verts=bool(rng.integers(0, 2)), local_idx=bool(rng.integers(0, 2)),
                units=bool(rng.integers(0, 2)))
    return m, idx, strategy, bt, nu, sp, want


@pytest.mark.parametrize("seed", range(CASES))
def test_random_configuration(stage, seed):
    from paper_1805_08893_amd import vr
    m, idx, strategy, bt, nu, sp, want = _case(seed)
    print(f"[fuzz] seed {seed}: T={len(idx) // 3} V={m.num_verts} strategy={strategy} bt={bt} nu={nu} {want}",
          flush=True)
    rc, o = vro.process_draw(idx, m.vertices, sp, strategy, bt, vro.make_opts(max_unique=nu), corners=True, **want)
    assert rc == vro.OK
    d_idx = torch.from_numpy(np.ascontiguousarray(idx).view(np.int32)).cuda()
    d_vtx = torch.from_numpy(m.vertices).cuda()
    res = stage.draw(d_idx, d_vtx, sp, strategy, bt, dict(max_unique=nu), corners=True, **want)
    st, inv = stage.sync()
    assert st == vr.VR_OK, vr.vr_last_error(stage.ctx)
    g = {k: v.cpu().numpy() for k, v in res.items()}
    n_inv, n_units = int(o["counters"][0]), int(o["counters"][1])
    assert int(g["counters"][0]) == n_inv and int(g["counters"][1]) == n_units and inv == n_inv
    assert np.array_equal(g["corners"].view(np.uint32), o["corners"].view(np.uint32))
    if want["tris"]:
        assert np.array_equal(g["tris"].view(np.uint32), o["tris"])
    if want["verts"]:
        assert np.array_equal(g["verts"][:n_inv].view(np.uint32), o["verts"].view(np.uint32))
    if want["local_idx"]:
        assert np.array_equal(g["local_idx"].view(np.uint16), o["local_idx"])
    if want["units"]:
        assert np.array_equal(g["unit_offsets"][:n_units + 1].view(np.uint32), o["unit_offsets"])
        assert np.array_equal(g["unit_invocations"][:n_units].view(np.uint32), o["unit_invocations"])
