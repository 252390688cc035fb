"""Serving-loop policy on the CPU: a fake clock and a fake backend with a
known service time make every admission and latency exactly predictable."""
import numpy as np
import pytest

from paper_1310_7556_amd.serve import (FakeBackend, FakeClock, Request, Scheduler, latency_stats,
                                       run_trace)


def reqs(arrivals, n_hits=100, nbytes=10):
    return [Request(rid=i, arrival=float(a), event=i, n_hits=n_hits, nbytes=nbytes)
            for i, a in enumerate(arrivals)]


def run(rs, slots=1, max_batch=1, max_hits=10**9, budget=10**9, service=lambda b: 1.0):
    clock = FakeClock()
    be = FakeBackend(clock, service)
    sched = Scheduler(slots, max_batch, max_hits, budget)
    run_trace(rs, sched, be, clock)
    return be


def test_plain_fifo_single_slot_latencies():
    rs = reqs([0.0, 0.1, 0.2, 5.0])
    run(rs)
    assert [r.done for r in rs] == [1.0, 2.0, 3.0, 6.0]
    assert [round(r.done - r.arrival, 6) for r in rs] == [1.0, 1.9, 2.8, 1.0]


def test_continuous_batching_admits_waiting_requests_together():
    rs = reqs([0.0, 0.1, 0.2, 0.3, 0.35])
    be = run(rs, slots=1, max_batch=8)
    # first request alone at t=0, the four that arrived meanwhile together at t=1
    assert be.launches[0][1] == [0]
    assert be.launches[1] == (0, [1, 2, 3, 4], 1.0)
    assert [r.done for r in rs] == [1.0, 2.0, 2.0, 2.0, 2.0]


def test_slots_overlap_and_fifo_order_is_kept():
    rs = reqs([0.0, 0.0, 0.0, 0.0, 0.5])
    be = run(rs, slots=2, max_batch=1)
    order = [ids[0] for _, ids, _ in be.launches]
    assert order == [0, 1, 2, 3, 4]
    assert [r.done for r in rs] == [1.0, 1.0, 2.0, 2.0, 3.0]


def test_budget_limits_bytes_in_flight():
    rs = reqs([0.0] * 6, nbytes=40)
    be = run(rs, slots=4, max_batch=8, budget=100)
    # at most two 40-byte requests fit a 100-byte budget at any time
    assert [len(ids) for _, ids, _ in be.launches] == [2, 2, 2]
    assert [t for _, _, t in be.launches] == [0.0, 1.0, 2.0]


def test_oversized_request_is_admitted_alone():
    rs = reqs([0.0, 0.0], nbytes=500)
    be = run(rs, slots=2, max_batch=8, budget=100)
    assert [ids for _, ids, _ in be.launches] == [[0], [1]]
    assert [r.done for r in rs] == [1.0, 2.0]


def test_request_larger_than_a_slot_is_refused():
    rs = reqs([0.0, 0.0], n_hits=800)
    with pytest.raises(ValueError):
        run(rs, slots=2, max_batch=8, max_hits=700)


def test_max_batch_hits_splits_batches():
    rs = reqs([0.0] * 5, n_hits=300)
    be = run(rs, slots=1, max_batch=8, max_hits=700)
    assert [len(ids) for _, ids, _ in be.launches] == [2, 2, 1]


def test_latency_stats_and_throughput():
    rs = reqs(np.arange(10) * 0.5)
    run(rs, service=lambda b: 0.25)
    st = latency_stats(rs)
    assert st["p50_ms"] == pytest.approx(250.0)
    assert st["p99_ms"] == pytest.approx(250.0)
    assert st["events_per_s"] == pytest.approx(10 / 4.75)


def test_batching_beats_plain_under_load():
    rng = np.random.default_rng(0)
    arr = np.cumsum(rng.exponential(1 / 2000.0, 400))
    # fixed cost per launch plus a small per-event cost: batching amortises it
    service = lambda b: 1e-3 + 1e-5 * len(b)
    plain = reqs(arr)
    run(plain, slots=1, max_batch=1, service=service)
    batched = reqs(arr)
    run(batched, slots=2, max_batch=64, service=service)
    sp, sb = latency_stats(plain), latency_stats(batched)
    assert sb["p99_ms"] < sp["p99_ms"] / 10
    assert sb["events_per_s"] > 1.5 * sp["events_per_s"]
