"""The vertex programs outside the short rounded-arithmetic ranges, end to end.

The shaders take a short sequence for 1/sqrt(d2) and the attenuation
1/(katt.d2 + 1) while d2 lies in [2^-96, 2^126] and the attenuation's
argument in [2^-125, 2^125], and the compiler's full IEEE sequences
otherwise.  A grid mesh scaled to 1e-20 (every light distance and view
vector below the range, in denormals) or to 4e18 (above it), with katt 0.05
and 1.0, drives whole draws through those fallbacks; naive, dynamic hash and
static ballot corners must equal the oracle's bit for bit (NaN positions
compared as positions)."""
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


def _scaled(scale, katt):
    m = W.grid_mesh(16, 16, seed=31, order="hilbert")
    v = m.vertices.copy()
    v[:, :3] = (v[:, :3].astype(np.float64) * scale).astype(np.float32)
    mesh = W.Mesh(m.name + f"_x{scale:g}", m.indices, v)
    sp = W.shader_for_mesh(mesh, W.SHADER_PHONG, 32, num_lights=4)
    sp.katt = katt
    return mesh, sp


def _outside_fraction(mesh, sp):
    """Fraction of (vertex, light) pairs whose d2 or attenuation argument lies
    outside the short sequences' ranges (float64 estimate)."""
    p = mesh.vertices[:, :3].astype(np.float64)
    model = np.asarray(sp.model, dtype=np.float64).reshape(3, 4)
    w = p @ model[:, :3].T + model[:, 3]
    L = np.asarray(sp.lights, dtype=np.float64).reshape(-1, 6)[:sp.num_lights, :3]
    d2 = ((L[None, :, :] - w[:, None, :]) ** 2).sum(-1)
    ad = np.abs(sp.katt * d2 + 1.0)
    out = (d2 < 2.0 ** -96) | (d2 > 2.0 ** 126) | (ad < 2.0 ** -125) | (ad > 2.0 ** 125)
    return float(out.mean())


CASES = [(1e-20, 0.05), (4e18, 0.05), (4e18, 1.0)]


@pytest.mark.parametrize("scale,katt", CASES, ids=["tiny", "huge", "huge_katt1"])
def test_fallback_ranges_match_oracle(stage, scale, katt):
    from paper_1805_08893_amd import vr
    mesh, sp = _scaled(scale, katt)
    assert _outside_fraction(mesh, sp) > 0.25   # the draw really takes the fallbacks
    idx = torch.from_numpy(np.ascontiguousarray(mesh.indices).view(np.int32)).cuda()
    vtx = torch.from_numpy(np.ascontiguousarray(mesh.vertices)).cuda()
    for name, strategy, bt, nu in (("naive", vr.VR_NAIVE, 1, 0), ("dyn_hash", vr.VR_DYN_HASH, 128, 128),
                                   ("static_ballot", vr.VR_STATIC_BALLOT, 64, 0)):
        print(f"[ranges] scale {scale:g} katt {katt} {name}", flush=True)
        res = stage.draw(idx, vtx, sp, strategy, bt, dict(max_unique=nu), corners=True)
        st, _ = stage.sync()
        assert st == vr.VR_OK, vr.vr_last_error(stage.ctx)
        got = res["corners"].cpu().numpy()
        rc, ora = vro.process_draw(mesh.indices, mesh.vertices, sp, strategy, bt, {"max_unique": nu},
                                   tris=False, verts=False, local_idx=False, units=False)
        assert rc == vro.OK
        exp = ora["corners"]
        assert int(res["counters"][0].item()) == int(ora["counters"][0])
        gn, en = np.isnan(got), np.isnan(exp)
        np.testing.assert_array_equal(gn, en)
        np.testing.assert_array_equal(got[~gn].view(np.uint32), exp[~en].view(np.uint32))


@pytest.mark.parametrize("kind", [W.SHADER_MVP, W.SHADER_PHONG], ids=["mvp", "phong"])
def test_zero_normals_match_oracle(stage, kind):
    """Zero normals: the normalisation's square root is 0, so 1/sqrt is inf
    and the normal outputs are NaN (0 x inf) on both sides; the rest of
    every corner is compared bitwise."""
    from paper_1805_08893_amd import vr
    m = W.grid_mesh(16, 16, seed=33, order="hilbert")
    v = m.vertices.copy()
    v[::3, 3] = 0.0   # every third vertex: n = (0, 0, 0)
    v[::3, 4] = 0.0
    v[::3, 5] = 0.0
    mesh = W.Mesh(m.name + "_zero_normals", m.indices, v)
    sp = W.shader_for_mesh(mesh, kind, 34, num_lights=4 if kind == W.SHADER_PHONG else 0)
    idx = torch.from_numpy(np.ascontiguousarray(mesh.indices).view(np.int32)).cuda()
    vtx = torch.from_numpy(np.ascontiguousarray(mesh.vertices)).cuda()
    for name, strategy, bt, nu in (("naive", vr.VR_NAIVE, 1, 0), ("dyn_sort", vr.VR_DYN_SORT, 128, 128)):
        print(f"[ranges] zero normals kind {kind} {name}", flush=True)
        res = stage.draw(idx, vtx, sp, strategy, bt, dict(max_unique=nu), corners=True)
        st, _ = stage.sync()
        assert st == vr.VR_OK, vr.vr_last_error(stage.ctx)
        got = res["corners"].cpu().numpy()
        rc, ora = vro.process_draw(mesh.indices, mesh.vertices, sp, strategy, bt, {"max_unique": nu},
                                   tris=False, verts=False, local_idx=False, units=False)
        assert rc == vro.OK
        exp = ora["corners"]
        gn, en = np.isnan(got), np.isnan(exp)
        assert en.any()   # the case reaches the non-finite path
        np.testing.assert_array_equal(gn, en)
        np.testing.assert_array_equal(got[~gn].view(np.uint32), exp[~en].view(np.uint32))


def test_phong_hand_cases_on_gpu(stage):
    """The exact Phong cases that pin the oracle (row-major model matrix,
    each light's own position, colour and attenuation, accumulation from
    light 0), shaded by the library: naive and static hash on a draw whose
    triangles all use one vertex."""
    from paper_1805_08893_amd import vr
    from test_oracle_pins import PERM_MODEL, PHONG_HAND_CASES, phong_on_axis_shader
    for ci, (p, heights, cols, katt, amb, rgb) in enumerate(PHONG_HAND_CASES):
        sp = phong_on_axis_shader(PERM_MODEL, p, heights, cols, katt, amb)
        vb = np.array([[*p, 0, 0, 1, 0.25, 0.75]], np.float32)
        idx = torch.zeros(3 * 5, dtype=torch.int32, device="cuda")
        vtx = torch.from_numpy(vb).cuda()
        for strategy, bt in ((vr.VR_NAIVE, 1), (vr.VR_STATIC_HASH, 4)):
            print(f"[phong hand] case {ci} strategy {vr.STRATEGY_NAMES[strategy]}", flush=True)
            res = stage.draw(idx, vtx, sp, strategy, bt, corners=True)
            st, _ = stage.sync()
            assert st == vr.VR_OK, vr.vr_last_error(stage.ctx)
            got = res["corners"].cpu().numpy()
            np.testing.assert_array_equal(got[:, 9:], np.broadcast_to(np.float32(rgb), (15, 3)))
            np.testing.assert_array_equal(got[:, :4], np.broadcast_to(np.float32([*p, 1.0]), (15, 4)))
