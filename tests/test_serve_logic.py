"""Serving logic on a fake device (virtual clock, modeled durations): footprint
admission, FIFO with bounded bypass, no starvation, latency percentiles."""
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


def test_budget_is_never_exceeded_and_all_complete():
    rng = np.random.default_rng(0)
    ws = [5, 20, 40, 70]
    ex = FakeExecutor(flops=[1e9, 5e9, 2e10, 8e10], ws_bytes=ws, rate=1e11, overhead=1e-4)
    arr = np.cumsum(rng.exponential(0.05, size=300))
    pats = rng.integers(0, 4, size=300)
    srv = Server(ex, budget_bytes=100, slots=4)
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
