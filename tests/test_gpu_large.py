"""A draw far larger than the bench mesh: 40M triangles of a strip-like index
stream (corner k of triangle t is vertex (t + k) mod V, V = 2^20) with
random vertices, so the corner output (5.76 GB) and the index offsets pass
4 GiB.  Checked by closed forms that hold at any size (a static batch of b
strip triangles has b + 2 distinct indices; a dynamic batch under N_u = 256
holds exactly 254 strip triangles, so the planner's general path runs) and
by sampled corners against the oracle's shading of their vertices."""
import numpy as np
import pytest

from oracle import vro
from paper_1805_08893_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

T = 40_000_000
V = 1 << 20


@pytest.fixture(scope="module")
def big():
    from paper_1805_08893_amd import vr
    s = vr.GeometryStage(0)
    t = torch.arange(T, device="cuda", dtype=torch.int64)
    idx = torch.stack([t, t + 1, t + 2], dim=1).remainder_(V).to(torch.int32).reshape(-1)
    del t
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    vtx = torch.rand((V, 8), device="cuda", generator=g, dtype=torch.float32) * 2 - 1
    yield s, idx, vtx
    s.close()


def _check(s, idx, vtx, strategy, bt, nu, want_inv):
    from paper_1805_08893_amd import vr
    sp = W.make_shader(W.SHADER_PHONG, 3, num_lights=4)
    res = s.draw(idx, vtx, sp, strategy, bt, dict(max_unique=nu), corners=True)
    st, inv = s.sync()
    assert st == vr.VR_OK, vr.vr_last_error(s.ctx)
    assert inv == want_inv and int(res["counters"][0].item()) == want_inv
    rng = np.random.default_rng(strategy)
    rows = np.concatenate([rng.integers(0, 3 * T, 2048), np.arange(3 * T - 64, 3 * T)])   # include the tail
    got = res["corners"][torch.from_numpy(rows).cuda()].cpu().numpy()
    verts = (torch.from_numpy(rows).cuda() // 3 + torch.from_numpy(rows % 3).cuda()).remainder(V)
    ref = vro.shade(sp, vtx[verts].cpu().numpy())
    np.testing.assert_array_equal(got.view(np.uint32), ref.view(np.uint32))
    del res
    torch.cuda.empty_cache()


def test_large_naive(big):
    from paper_1805_08893_amd import vr
    print("[large] naive", flush=True)
    _check(*big, vr.VR_NAIVE, 1, 0, 3 * T)


def test_large_static_hash(big):
    from paper_1805_08893_amd import vr
    print("[large] static hash 256", flush=True)
    full, rest = divmod(T, 256)
    _check(*big, vr.VR_STATIC_HASH, 256, 0, full * 258 + (rest + 2 if rest else 0))


def test_large_dynamic_hash_general_plan(big):
    from paper_1805_08893_amd import vr
    print("[large] dynamic hash 256/256", flush=True)
    B = -(-T // 254)
    _check(*big, vr.VR_DYN_HASH, 256, 256, T + 2 * B)


def test_large_static_ballot(big):
    """A 64-triangle strip batch has 66 distinct indices: a round of 62
    triangles (64 distinct) and one of 2 (4 distinct), 68 invocations."""
    from paper_1805_08893_amd import vr
    print("[large] static ballot 64", flush=True)
    full, rest = divmod(T, 64)
    tail = 0 if rest == 0 else (rest + 2 if rest <= 62 else 64 + (rest - 62 + 2))
    _check(*big, vr.VR_STATIC_BALLOT, 64, 0, full * 68 + tail)


def test_large_dynamic_sort(big):
    from paper_1805_08893_amd import vr
    print("[large] dynamic sort 256/256", flush=True)
    B = -(-T // 254)
    _check(*big, vr.VR_DYN_SORT, 256, 256, T + 2 * B)
