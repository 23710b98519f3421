"""Request-server admission and tick policy on a simulated clock (CPU only).

vr_server_simulate runs the scheduler object the HIP server runs, with a
simulated device that executes ticks one after another in
tick_fixed_s + tick_s_per_tri x triangles.  These tests pin the policy:
FIFO admission against the memory budget, non-overlapping reservations,
tick limits, continuous batching, rejection and cancellation.
"""
import numpy as np
import pytest

from paper_1805_08893_amd import vr

GRANULE = 256


def rnd(b):
    return (max(b, 1) + GRANULE - 1) // GRANULE * GRANULE


def sim(reqs, budget=1 << 30, inflight=2, draws=1024, tris=0, fixed=1e-3, per_tri=1e-9):
    cfg = vr.make_server_config(budget, inflight, draws, tris)
    st, res, stats = vr.vr_server_simulate(cfg, reqs, fixed, per_tri)
    assert st == vr.VR_OK
    return res, stats


def req(arrival, num_tris, nbytes=None, cancel_at=-1.0, hold=0.0):
    return (arrival, num_tris, 144 * num_tris if nbytes is None else nbytes, cancel_at, hold)


def ticks_of(res):
    out = {}
    for i, r in enumerate(res):
        if r["status"] == vr.VR_OK:
            out.setdefault(r["tick"], []).append(i)
    return out


def check_memory(res, reqs, budget):
    """Reservations of requests alive at the same time never overlap and stay inside the budget."""
    live = [(r["t_admit"], r["t_release"], r["offset"], rnd(q[2])) for r, q in zip(res, reqs) if r["t_admit"] >= 0]
    for a0, a1, o, b in live:
        assert o + b <= budget
    for i in range(len(live)):
        for j in range(i + 1, len(live)):
            (s0, e0, o0, b0), (s1, e1, o1, b1) = live[i], live[j]
            if s0 < e1 and s1 < e0:   # alive together
                assert o0 + b0 <= o1 or o1 + b1 <= o0


def test_light_load_latency_is_the_service_time():
    reqs = [req(0.01 * i, 1000 * (i + 1)) for i in range(20)]
    res, stats = sim(reqs)
    for (a, t, *_), r in zip(reqs, res):
        assert r["status"] == vr.VR_OK
        assert r["t_admit"] == a and r["t_launch"] == a
        assert r["t_done"] - a == pytest.approx(1e-3 + 1e-9 * t, rel=1e-12)
    assert stats["ticks"] == 20 and stats["max_tick_draws"] == 1
    assert stats["completed"] == 20 and stats["reserved_bytes"] == 0


def test_tiny_budget_forces_fifo_queueing():
    budget = 1 << 20
    reqs = [req(0.0, 2000, hold=5e-4) for _ in range(12)]   # 288,000 B each: three fit
    res, stats = sim(reqs, budget=budget)
    assert all(r["status"] == vr.VR_OK for r in res)
    assert stats["peak_reserved_bytes"] <= budget and stats["admission_blocked"] > 0
    admits = [r["t_admit"] for r in res]
    assert admits == sorted(admits)                       # submission order
    assert max(admits) > 0.0                              # later ones waited for memory
    for t in admits:                                      # never more than three alive
        alive = sum(1 for r in res if r["t_admit"] <= t < r["t_release"])
        assert alive <= 3
    check_memory(res, reqs, budget)


def test_continuous_batching_under_burst():
    reqs = [req(1e-5 * i, 1000) for i in range(100)]
    res, stats = sim(reqs, inflight=1, draws=16)
    ticks = ticks_of(res)
    assert ticks[0] == [0]                                # the first request runs alone
    assert max(len(v) for v in ticks.values()) == 16
    assert stats["ticks"] == 1 + -(-99 // 16)
    ends = sorted((min(res[i]["t_launch"] for i in v), max(res[i]["t_done"] for i in v)) for v in ticks.values())
    for (l0, d0), (l1, d1) in zip(ends, ends[1:]):
        assert l1 >= d0                                   # one tick in flight at a time
    # the same burst with one launch per request takes 100 fixed costs
    res1, stats1 = sim(reqs, inflight=1, draws=1)
    assert stats1["ticks"] == 100
    last = max(r["t_done"] for r in res)
    last1 = max(r["t_done"] for r in res1)
    assert last1 > 5 * last


def test_tick_triangle_limit():
    reqs = [req(0.0, 1000) for _ in range(9)] + [req(0.0, 5000)]
    res, _ = sim(reqs, inflight=1, tris=2500)
    for tick, members in ticks_of(res).items():
        t = sum(reqs[i][1] for i in members)
        assert t <= 2500 or len(members) == 1
    assert len(ticks_of(res)[res[9]["tick"]]) == 1        # larger than the limit: alone


def test_rejection_and_cancellation():
    budget = 1 << 20
    reqs = [req(0.0, 2000, hold=1.0),                     # holds a third of the budget for 1 s
            req(0.0, 2000, hold=1.0),
            req(0.0, 2000, hold=1.0),
            req(0.001, 100000),                           # 14.4 MB: can never fit
            req(0.002, 2000, cancel_at=0.5),              # waits for memory, cancelled first
            req(0.003, 100, cancel_at=2.0)]               # launched before its cancel time
    res, stats = sim(reqs, budget=budget)
    assert res[3]["status"] == vr.VR_ERR_CAPACITY and res[3]["t_admit"] < 0
    assert res[4]["status"] == vr.VR_CANCELLED and res[4]["t_launch"] < 0 and res[4]["t_done"] == 0.5
    # FIFO: blocked behind the waiting request 4 although it fits, admitted
    # the moment 4 is cancelled
    assert res[5]["status"] == vr.VR_OK and res[5]["t_admit"] == 0.5
    assert stats["rejected"] == 1 and stats["cancelled"] == 1
    assert stats["reserved_bytes"] == 0


def test_fifo_does_not_starve_a_large_request():
    budget = 1 << 22
    reqs = [req(0.0, 10000, hold=2e-3)]                   # 1.44 MB
    reqs += [req(1e-4 * i, 9000, hold=2e-3) for i in range(1, 5)]
    reqs += [req(6e-4, 20000)]                            # 2.88 MB: needs most of the budget
    reqs += [req(7e-4 + 1e-4 * i, 500, hold=2e-3) for i in range(50)]
    res, _ = sim(reqs, budget=budget)
    big = res[5]
    assert big["status"] == vr.VR_OK
    assert all(r["t_admit"] >= big["t_admit"] for r in res[6:])
    check_memory(res, reqs, budget)


def test_random_mix_keeps_reservations_disjoint():
    rng = np.random.default_rng(7)
    budget = 8 << 20
    arr = np.cumsum(rng.exponential(2e-4, 400))
    sizes = np.clip(np.exp(rng.normal(np.log(3000), 1.2, 400)), 10, 40000).astype(int)
    holds = rng.exponential(1e-3, 400)
    cancels = np.where(rng.random(400) < 0.1, arr + rng.exponential(5e-4, 400), -1.0)
    reqs = [req(float(a), int(t), cancel_at=float(c), hold=float(h)) for a, t, c, h in zip(arr, sizes, cancels, holds)]
    res, stats = sim(reqs, budget=budget, inflight=3, draws=32, tris=200000, fixed=2e-4, per_tri=2e-9)
    assert stats["peak_reserved_bytes"] <= budget and stats["reserved_bytes"] == 0
    assert stats["completed"] + stats["cancelled"] + stats["rejected"] == 400
    admitted = [r["t_admit"] for r in res if r["t_admit"] >= 0]
    assert admitted == sorted(admitted)
    check_memory(res, reqs, budget)
    for r, q in zip(res, reqs):
        if r["status"] == vr.VR_OK:
            assert q[0] <= r["t_admit"] <= r["t_launch"] < r["t_done"] <= r["t_release"]


def test_config_and_order_errors():
    cfg = vr.make_server_config(1 << 20, 9)
    st, _, _ = vr.vr_server_simulate(cfg, [req(0.0, 10)], 1e-3, 0.0)
    assert st == vr.VR_ERR_ARG
    cfg = vr.make_server_config(1 << 20, 2, 5000)
    assert vr.vr_server_simulate(cfg, [req(0.0, 10)], 1e-3, 0.0)[0] == vr.VR_ERR_ARG
    cfg = vr.make_server_config(1 << 20)
    assert vr.vr_server_simulate(cfg, [req(1.0, 10), req(0.5, 10)], 1e-3, 0.0)[0] == vr.VR_ERR_ARG
    assert vr.vr_server_simulate(cfg, [], 1e-3, 0.0)[0] == vr.VR_OK
