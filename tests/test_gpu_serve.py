"""Request server on the GPU: every request's result, alone or in any mix,
equals the single-draw path's (bitwise corners, equal counts); requests
queued in one call; admission under a tiny budget; argument errors and
cancellation."""
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


BASES = None


def _bases():
    global BASES
    if BASES is None:
        BASES = [W.grid_mesh(41, 37, 5, "hilbert"), W.icosphere_mesh(4, 6, "scan"),
                 W.grid_mesh(33, 33, 8, "random")]
    return BASES


def _configs():
    from paper_1805_08893_amd import vr
    return [(vr.VR_NAIVE, 1, 0), (vr.VR_STATIC_BALLOT, 64, 0), (vr.VR_STATIC_SORT, 64, 0),
            (vr.VR_STATIC_HASH, 128, 0), (vr.VR_DYN_SORT, 256, 256), (vr.VR_DYN_HASH, 341, 256),
            (vr.VR_DYN_PHASH, 256, 256), (vr.VR_DYN_BALLOT, 85, 64), (vr.VR_DYN_HASH, 64, 64)]


def _requests(n, seed):
    """(base, first triangle of the window, num_tris, shader, config) tuples."""
    rng = np.random.default_rng(seed)
    bases, cfgs = _bases(), _configs()
    out = []
    for i in range(n):
        b = int(rng.integers(0, len(bases)))
        T = bases[b].num_tris
        start = 0 if i % 3 == 0 else int(rng.integers(0, T // 2))
        size = int(rng.integers(0, T - start + 1)) if i % 5 else T - start
        kind = int(rng.integers(0, 3))
        sp = W.shader_for_mesh(bases[b], kind, seed + i, num_lights=int(rng.integers(1, 17)), iterations=8)
        out.append((b, start, size, sp, cfgs[i % len(cfgs)]))
    return out


def _single(stage, idx, vtx, size, sp, cfg):
    """The single-draw path on the same prefix (its own plan)."""
    from paper_1805_08893_amd import vr
    s, bt, nu = cfg
    sub = idx[:3 * size]
    opts = None
    if s in vr.DYNAMIC:
        plan = torch.empty(size + 2, dtype=torch.int32, device="cuda")
        stage.check(vr.vr_plan_dynamic(stage.ctx, sub, vtx.shape[0], nu, bt, plan))
        opts = vr.make_opts(max_unique=nu, plan=plan)
    else:
        opts = vr.make_opts(max_unique=nu)
    r = stage.draw(sub, vtx, sp, s, bt, opts=opts, corners=True)
    st, _ = stage.sync()
    stage.check(st)
    return r["corners"].cpu().numpy(), r["counters"].cpu().numpy()


def _register(srv, windows):
    dev = [(_dev(m.indices), _dev(m.vertices)) for m in _bases()]
    ids = {}
    for (b, start) in windows:
        if (b, start) not in ids:
            idx, vtx = dev[b]
            ids[(b, start)] = srv.add_mesh(idx[3 * start:], vtx)
    return dev, ids


def test_results_alone_equal_in_the_mix(stage):
    from paper_1805_08893_amd import vr
    from paper_1805_08893_amd.serve import Server
    reqs = _requests(40, 21)
    with Server(256 << 20, max_inflight=2, max_tick_draws=8) as srv:
        dev, ids = _register(srv, [(b, st) for b, st, *_ in reqs])
        tickets = {}
        for i, (b, start, size, sp, (s, bt, nu)) in enumerate(reqs):
            t = srv.submit(vr.make_request(ids[(b, start)], size, sp, s, bt, nu, user=i))
            tickets[t] = i
        got = srv.drain(len(reqs), release=False)
        assert sorted(c["user"] for c in got) == list(range(len(reqs)))
        assert max(c["tick"] for c in got) >= len(reqs) // 8 - 1      # several ticks, up to 8 requests each
        for c in got:
            i = c["user"]
            b, start, size, sp, cfg = reqs[i]
            assert c["status"] == vr.VR_OK and c["num_tris"] == size
            mine = srv.fetch(c["ticket"], size)
            idx, vtx = dev[b]
            ref, cnt = _single(stage, idx[3 * start:], vtx, size, sp, cfg)
            assert c["invocations"] == cnt[0] and c["units"] == cnt[1], (i, cfg)
            assert np.array_equal(mine.view(np.uint32), ref.view(np.uint32)), (i, cfg, size)
            srv.release(c["ticket"])
        st = srv.stats()
        assert st["completed"] == len(reqs) and st["reserved_bytes"] == 0 and st["plan_bytes"] > 0


def test_mix_matches_the_oracle_directly():
    from paper_1805_08893_amd import vr
    from paper_1805_08893_amd.serve import Server
    reqs = [r for r in _requests(12, 5) if r[2] <= 1500][:6]
    with Server(64 << 20) as srv:
        dev, ids = _register(srv, [(b, st) for b, st, *_ in reqs])
        for i, (b, start, size, sp, (s, bt, nu)) in enumerate(reqs):
            srv.submit(vr.make_request(ids[(b, start)], size, sp, s, bt, nu, user=i))
        for c in srv.drain(len(reqs), release=False):
            b, start, size, sp, (s, bt, nu) = reqs[c["user"]]
            m = _bases()[b]
            rc, o = vro.process_draw(m.indices[3 * start:3 * (start + size)], m.vertices, sp, s, bt,
                                     vro.make_opts(max_unique=nu), corners=True)
            assert rc == 0
            assert c["invocations"] == int(o["counters"][0]) and c["units"] == int(o["counters"][1])
            mine = srv.fetch(c["ticket"], size)
            assert np.array_equal(mine.view(np.uint32), o["corners"].view(np.uint32))
            srv.release(c["ticket"])


def test_submit_many_matches_the_oracle_and_stops_at_a_rejected_request():
    """Requests queued in one call are processed as if submitted one by one
    (bitwise against the oracle); a rejected request in the middle ends the
    call with its status, the ones before it queued and the ones after not;
    an empty call queues nothing."""
    from paper_1805_08893_amd import vr
    from paper_1805_08893_amd.serve import Server
    reqs = [r for r in _requests(14, 9) if r[2] <= 1500][:6]
    with Server(64 << 20) as srv:
        dev, ids = _register(srv, [(b, st) for b, st, *_ in reqs])
        made = [vr.make_request(ids[(b, start)], size, sp, s, bt, nu, user=i)
                for i, (b, start, size, sp, (s, bt, nu)) in enumerate(reqs)]
        b0, start0 = reqs[0][0], reqs[0][1]
        bad = vr.make_request(ids[(b0, start0)], _bases()[b0].num_tris - start0 + 1, reqs[0][3], vr.VR_NAIVE, 1,
                              user=99)
        st, tickets = vr.vr_server_submit_many(srv.h, made[:4] + [bad] + made[4:])
        assert st == vr.VR_ERR_ARG and len(tickets) == 4
        assert srv.submit_many([]) == []
        assert len(srv.submit_many(made[4:])) == len(made) - 4
        got = srv.drain(len(made), release=False)
        assert sorted(c["user"] for c in got) == list(range(len(made)))
        for c in got:
            b, start, size, sp, (s, bt, nu) = reqs[c["user"]]
            m = _bases()[b]
            rc, o = vro.process_draw(m.indices[3 * start:3 * (start + size)], m.vertices, sp, s, bt,
                                     vro.make_opts(max_unique=nu), corners=True)
            assert rc == 0
            assert c["status"] == vr.VR_OK
            assert c["invocations"] == int(o["counters"][0]) and c["units"] == int(o["counters"][1])
            mine = srv.fetch(c["ticket"], size)
            assert np.array_equal(mine.view(np.uint32), o["corners"].view(np.uint32))
            srv.release(c["ticket"])
        assert srv.stats()["submitted"] == len(made)


def test_tiny_budget_queues_and_stays_correct(stage):
    from paper_1805_08893_amd import vr
    from paper_1805_08893_amd.serve import Server
    m = _bases()[0]
    sp = W.shader_for_mesh(m, W.SHADER_PHONG, 3, num_lights=4)
    one = 144 * m.num_tris
    with Server(3 * one + 4096, max_inflight=1, max_tick_draws=4) as srv:
        idx, vtx = _dev(m.indices), _dev(m.vertices)
        mid = srv.add_mesh(idx, vtx)
        for i in range(10):
            srv.submit(vr.make_request(mid, m.num_tris, sp, vr.VR_DYN_HASH, 256, 256, user=i))
        got = []
        while len(got) < 10:   # hold each result until the next one arrives
            got += srv.drain(1, release=False)
            if len(got) >= 2:
                srv.release(got[-2]["ticket"])
        srv.release(got[-1]["ticket"])
        st = srv.stats()
        assert st["peak_reserved_bytes"] <= 3 * one + 4096 and st["admission_blocked"] > 0
        assert all(c["status"] == vr.VR_OK for c in got)
        assert len({c["invocations"] for c in got}) == 1
        assert [c["user"] for c in got] == list(range(10))          # FIFO


def test_errors_and_cancellation():
    from paper_1805_08893_amd import vr
    from paper_1805_08893_amd.serve import Server
    m = _bases()[1]
    sp = W.shader_for_mesh(m, W.SHADER_MVP, 1)
    one = 144 * m.num_tris
    with Server(one + 1024, max_inflight=1) as srv:
        idx, vtx = _dev(m.indices), _dev(m.vertices)
        mid = srv.add_mesh(idx, vtx)
        bad = idx.clone()
        bad[7] = m.num_verts
        st, _ = vr.vr_server_add_mesh(srv.h, bad, vtx)
        assert st == vr.VR_ERR_INDEX_RANGE
        assert vr.vr_server_submit(srv.h, vr.make_request(mid + 5, 10, sp, vr.VR_NAIVE, 1))[0] == vr.VR_ERR_ARG
        assert vr.vr_server_submit(srv.h, vr.make_request(mid, m.num_tris + 1, sp, vr.VR_NAIVE, 1))[0] == vr.VR_ERR_ARG
        assert vr.vr_server_submit(srv.h, vr.make_request(mid, 10, sp, vr.VR_STATIC_SORT, 300))[0] == vr.VR_ERR_ARG
        a = srv.submit(vr.make_request(mid, m.num_tris, sp, vr.VR_STATIC_HASH, 64, user=1))
        b = srv.submit(vr.make_request(mid, m.num_tris, sp, vr.VR_STATIC_HASH, 64, user=2))   # waits for a's memory
        first = srv.drain(1, release=False)[0]
        assert first["ticket"] == a
        assert vr.vr_server_release(srv.h, b) == vr.VR_ERR_BUSY
        assert vr.vr_server_cancel(srv.h, a) == vr.VR_ERR_BUSY
        assert vr.vr_server_cancel(srv.h, b) == vr.VR_OK
        second = srv.drain(1, release=False)[0]
        assert second["ticket"] == b and second["status"] == vr.VR_CANCELLED
        srv.release(a)
        srv.release(b)
        assert vr.vr_server_release(srv.h, a) == vr.VR_ERR_ARG
        st = srv.stats()
        assert st["cancelled"] == 1 and st["reserved_bytes"] == 0
