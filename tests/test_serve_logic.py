"""Serving logic on a fake device (virtual clock, modeled durations): footprint
admission, FIFO with bounded bypass, shortest-first admission with a bound on
overtaking, no starvation, latency percentiles."""
import numpy as np
import pytest

from paper_2501_02483_amd.serve import FakeExecutor, Request, Server, summarize


def _reqs(arrivals, pats):
    return [Request(rid=i, arrival=a, pattern=p, op=0, seed=i) for i, (a, p) in enumerate(zip(arrivals, pats))]


def test_sequential_latencies_are_exact():
    # one slot, each request takes 1 s at rate 1: latencies 1, 1.5, 2.0 ...
    ex = FakeExecutor(flops=[1.0], ws_bytes=[10], rate=1.0, overhead=0.0)
    srv = Server(ex, budget_bytes=100, slots=1)
    done = srv.run(_reqs([0.0, 0.5, 1.0], [0, 0, 0]))
    lat = sorted(r.latency for r in done)
    assert np.allclose(lat, [1.0, 1.5, 2.0])
    s = summarize(done)
    assert s["requests"] == 3
    assert abs(s["p50_ms"] - 1500.0) < 1e-6


@pytest.mark.parametrize("policy", ["fifo", "sjf"])
def test_budget_is_never_exceeded_and_all_complete(policy):
    rng = np.random.default_rng(0)
    ws = [5, 20, 40, 70]
    ex = FakeExecutor(flops=[1e9, 5e9, 2e10, 8e10], ws_bytes=ws, rate=1e11, overhead=1e-4)
    arr = np.cumsum(rng.exponential(0.05, size=300))
    pats = rng.integers(0, 4, size=300)
    srv = Server(ex, budget_bytes=100, slots=4, policy=policy)
    done = srv.run(_reqs(arr, pats))
    assert len(done) == 300
    assert srv.max_used <= 100
    assert all(r.t_done >= r.t_admit >= r.arrival - 1e-12 for r in done)


def test_bounded_bypass_prevents_starvation():
    # a large request behind a stream of small ones: it may be bypassed at
    # most max_bypass times, then the small ones wait until it fits
    ex = FakeExecutor(flops=[1.0, 10.0], ws_bytes=[30, 80], rate=1.0, overhead=0.0)
    arrivals = [0.0] + [0.01 * (k + 1) for k in range(30)]
    pats = [0] + [0] * 30
    reqs = _reqs(arrivals, pats)
    big = Request(rid=99, arrival=0.005, pattern=1, op=0, seed=0)
    srv = Server(ex, budget_bytes=100, slots=4, max_bypass=3)
    done = srv.run(reqs + [big])
    order = srv.admit_order
    pos = order.index(99)
    assert big.bypassed == 3
    # the big request is admitted after at most 3 bypasses beyond the running one
    assert pos <= 1 + 3 + 1
    assert len(done) == 32


def test_request_larger_than_budget_is_rejected():
    ex = FakeExecutor(flops=[1.0], ws_bytes=[500], rate=1.0)
    srv = Server(ex, budget_bytes=100, slots=2)
    with pytest.raises(ValueError):
        srv.run(_reqs([0.0], [0]))


def test_open_loop_latency_grows_with_load():
    ws = [10, 10]
    lo = Server(FakeExecutor(flops=[1e9, 2e9], ws_bytes=ws, rate=1e11), 1000, slots=4)
    hi = Server(FakeExecutor(flops=[1e9, 2e9], ws_bytes=ws, rate=1e11), 1000, slots=4)
    rng = np.random.default_rng(1)
    pats = rng.integers(0, 2, 400)
    slow = np.cumsum(rng.exponential(1 / 20.0, 400))     # 20 req/s, about 0.3 of capacity
    fast = slow / 3.0                                      # 60 req/s, about 0.9 of capacity
    p_lo = summarize(lo.run(_reqs(slow, pats)))["p99_ms"]
    p_hi = summarize(hi.run(_reqs(fast, pats)))["p99_ms"]
    assert p_hi > p_lo


def test_summary_per_pattern_and_per_op_percentiles():
    ex = FakeExecutor(flops=[1e9, 8e9, 3e10], ws_bytes=[10, 10, 10], rate=1e11, overhead=1e-4)
    rng = np.random.default_rng(3)
    arr = np.cumsum(rng.exponential(0.02, size=400))
    reqs = [Request(rid=i, arrival=a, pattern=int(rng.integers(3)), op=i % 3, seed=i) for i, a in enumerate(arr)]
    done = Server(ex, 1000, slots=4).run(reqs)
    s = summarize(done)
    assert sum(s["per_pattern_count"].values()) == 400
    for k, p99 in s["per_pattern_p99_ms"].items():
        lat = sorted(r.latency for r in done if r.pattern == k)
        assert s["per_pattern_p50_ms"][k] <= p99 <= lat[-1] * 1e3 + 1e-9
        assert p99 >= lat[int(0.98 * (len(lat) - 1))] * 1e3 - 1e-9
    # the largest pattern has the slowest tail
    assert s["per_pattern_p99_ms"][2] == max(s["per_pattern_p99_ms"].values())
    assert set(s["per_op_p99_ms"]) == {"factorize", "factorize+solve", "factorize+logdet"}


def test_sjf_admits_the_least_work_first():
    # one slot busy with a request of pattern 3; four more arrive meanwhile
    # in the order 2, 0, 3, 1: they run shortest first, ties by arrival
    ex = FakeExecutor(flops=[1.0, 2.0, 3.0, 4.0], ws_bytes=[1, 1, 1, 1], rate=1.0, overhead=0.0)
    reqs = _reqs([0.0, 0.1, 0.2, 0.3, 0.4], [3, 2, 0, 3, 1])
    srv = Server(ex, budget_bytes=100, slots=1, policy="sjf")
    done = srv.run(reqs)
    assert srv.admit_order == [0, 2, 4, 1, 3]
    assert len(done) == 5
    # FIFO keeps the arrival order
    fifo = Server(FakeExecutor(flops=[1.0, 2.0, 3.0, 4.0], ws_bytes=[1, 1, 1, 1], rate=1.0, overhead=0.0),
                  budget_bytes=100, slots=1)
    fifo.run(_reqs([0.0, 0.1, 0.2, 0.3, 0.4], [3, 2, 0, 3, 1]))
    assert fifo.admit_order == [0, 1, 2, 3, 4]


def test_sjf_bounds_overtaking_of_a_large_request():
    # a large request queued behind a dense stream of small ones is overtaken
    # at most max_overtake times, then admitted before any later arrival
    ex = FakeExecutor(flops=[1.0, 10.0], ws_bytes=[1, 1], rate=1.0, overhead=0.0)
    arrivals = [0.0] + [0.05 * (k + 1) for k in range(60)]
    reqs = _reqs(arrivals, [0] * 61)
    big = Request(rid=99, arrival=0.01, pattern=1, op=0, seed=0)
    srv = Server(ex, budget_bytes=100, slots=1, policy="sjf", max_overtake=5)
    done = srv.run(reqs + [big])
    assert len(done) == 62
    pos = srv.admit_order.index(99)
    assert big.bypassed == 5
    assert pos == 1 + 5          # the running request, then five overtakes


def test_sjf_waits_for_a_starving_request_that_does_not_fit():
    # the starving request needs the whole budget: nothing else is admitted
    # ahead of it once it has been overtaken max_overtake times
    ex = FakeExecutor(flops=[1.0, 1.0], ws_bytes=[30, 100], rate=1.0, overhead=0.0)
    arrivals = [0.0] + [0.01 * (k + 1) for k in range(20)]
    reqs = _reqs(arrivals, [0] * 21)
    big = Request(rid=99, arrival=0.001, pattern=1, op=0, seed=0)
    srv = Server(ex, budget_bytes=100, slots=3, policy="sjf", max_overtake=2)
    srv.run(reqs + [big])
    order = srv.admit_order
    assert big.bypassed == 2
    # requests admitted after the big one arrived and before it: at most the
    # two overtakes plus those already running
    assert order.index(99) <= 1 + 2 + 2
    assert srv.max_used <= 100


def test_sjf_lowers_mean_latency_on_a_mixed_load():
    flops = [1e9, 4e9, 1.6e10, 2.4e11]
    rng = np.random.default_rng(7)
    n = 1500
    pats = rng.integers(0, 4, n)
    mean_service = np.mean([f / 1e12 + 1e-3 for f in flops])
    arr = np.cumsum(rng.exponential(mean_service / 0.8 / 2, n))   # 0.8 of two slots' capacity
    out = {}
    for policy in ("fifo", "sjf"):
        ex = FakeExecutor(flops=flops, ws_bytes=[1] * 4, rate=1e12, overhead=1e-3)
        out[policy] = summarize(Server(ex, 1000, slots=2, policy=policy).run(_reqs(arr, pats)))
    assert out["sjf"]["mean_ms"] < out["fifo"]["mean_ms"]
    assert out["sjf"]["p50_ms"] < out["fifo"]["p50_ms"]
    assert out["sjf"]["per_pattern_p99_ms"][0] < out["fifo"]["per_pattern_p99_ms"][0]


def test_unknown_policy_is_rejected():
    with pytest.raises(ValueError):
        Server(FakeExecutor(flops=[1.0], ws_bytes=[1]), 10, 1, policy="lifo")
