"""Host logic of the continuous-batching scheduler (no GPU): admission in
arrival order, the memory budget over the calls in flight, overlapping calls
in several slots, and the per-batch bookkeeping.  The index is a stub that
records what each call receives."""
import threading
import time

import numpy as np
import pytest

import gen
from paper_1711_07295_amd import serve


class StubIndex:
    def __init__(self, delay=0.0):
        self.calls = []
        self.delay = delay
        self.lock = threading.Lock()
        self.active = 0
        self.max_active = 0
        self.capacities = []

    def query(self, views, p, q, queue_capacity=0, flags=0):
        with self.lock:
            self.calls.append([(v.n_sets, v.n_tokens) for v in views])
            self.capacities.append(queue_capacity)
            self.active += 1
            self.max_active = max(self.max_active, self.active)
        time.sleep(self.delay)
        with self.lock:
            self.active -= 1
        # one fake pair per set, so the caller's split can be checked
        pairs = [np.stack([np.arange(v.n_sets, dtype=np.uint32)] * 2, axis=1) for v in views]
        st = {"ms_total": 1.0, "ms_prepare": 0.1, "ms_filter": 0.5, "ms_verify": 0.2,
              "ms_emit": 0.1, "band_pairs": 10 * len(views), "survivors": 0,
              "results": sum(v.n_sets for v in views)}
        return pairs, st


def _batches(sizes):
    return [gen.from_lists([[k, k + 1]] * n) for k, n in enumerate(sizes)]


def test_everything_waiting_goes_into_one_call():
    idx = StubIndex()
    srv = serve.ContinuousBatcher(idx, keep_pairs=True)
    b = _batches([3, 1, 4, 1, 5])
    r = srv.run(b, [(1, 2)] * 5, np.zeros(5), device="cpu")
    assert r.calls == 1 and idx.calls == [[(3, 6), (1, 2), (4, 8), (1, 2), (5, 10)]]
    assert [len(x) for x in r.pairs] == [3, 1, 4, 1, 5]
    assert r.band_pairs == 50 and r.results == 14
    assert np.all(r.latency_s >= 0) and np.all(r.wait_s >= 0)


def test_memory_budget_splits_calls_in_arrival_order():
    idx = StubIndex()
    q = 1 << 12
    one = serve.call_bytes(10, 20, q)  # a call of one batch of 10 sets, 20 tokens
    two = serve.call_bytes(20, 40, q)
    srv = serve.ContinuousBatcher(idx, memory_budget=two, queue_capacity=q)
    b = _batches([10] * 5)
    r = srv.run(b, [(1, 2)] * 5, np.zeros(5), device="cpu")
    assert [len(c) for c in idx.calls] == [2, 2, 1]
    assert list(r.batches_per_call) == [2, 2, 1]
    # the budget holds one call at a time here, so no two were in flight
    assert r.max_in_flight == 1 and idx.max_active == 1
    assert r.peak_bytes <= two and one < two
    assert idx.capacities == [q] * 3


def test_calls_overlap_in_slots_and_late_arrivals_join_a_free_slot():
    """Slot 1 is busy with the first batch when the next ones arrive: they
    go into slot 2 at once instead of waiting for the first call."""
    idx = StubIndex(delay=0.3)
    srv = serve.ContinuousBatcher(idx, slots=2, memory_budget=1 << 40, keep_pairs=True)
    b = _batches([2, 3, 4])
    arr = np.array([0.0, 0.05, 0.06])
    r = srv.run(b, [(1, 2)] * 3, arr, device="cpu")
    assert r.max_in_flight == 2 and idx.max_active == 2
    assert [len(c) for c in idx.calls] == [1, 1, 1] or [len(c) for c in idx.calls] == [1, 2]
    assert r.wait_s[1] < 0.2  # admitted while the first call still ran
    assert [len(x) for x in r.pairs] == [2, 3, 4]
    assert np.all(r.latency_s >= 0.3 - 1e-3)


def test_memory_gate_holds_back_a_second_call():
    """Two free slots, but the first call's memory leaves no room for a
    second one: the next batch waits for the first call to end."""
    idx = StubIndex(delay=0.2)
    q = 1 << 12
    srv = serve.ContinuousBatcher(idx, slots=2, memory_budget=serve.call_bytes(10, 20, q) + 100,
                                  queue_capacity=q)
    b = _batches([10, 10])
    r = srv.run(b, [(1, 2)] * 2, np.array([0.0, 0.01]), device="cpu")
    assert r.max_in_flight == 1 and r.calls == 2
    assert r.wait_s[1] >= 0.15


def test_errors_of_a_call_reach_the_caller():
    class Failing(StubIndex):
        def query(self, *a, **k):
            raise RuntimeError("boom")
    srv = serve.ContinuousBatcher(Failing(), slots=2)
    with pytest.raises(RuntimeError, match="boom"):
        srv.run(_batches([1, 1]), [(1, 2)] * 2, np.zeros(2), device="cpu")


def test_a_batch_larger_than_the_budget_still_runs_alone():
    idx = StubIndex()
    srv = serve.ContinuousBatcher(idx, memory_budget=1)
    b = _batches([7, 2])
    r = srv.run(b, [(1, 2)] * 2, np.zeros(2), device="cpu")
    assert [len(c) for c in idx.calls] == [1, 1] and r.calls == 2


def test_batches_arriving_later_wait_for_the_next_call():
    idx = StubIndex()
    srv = serve.ContinuousBatcher(idx)
    b = _batches([1, 1, 1])
    arr = np.array([0.0, 0.05, 0.05])
    r = srv.run(b, [(1, 2)] * 3, arr, device="cpu")
    assert [len(c) for c in idx.calls] == [1, 2]
    # nothing completes before it arrives
    assert np.all(r.latency_s > 0)


def test_poisson_arrivals_rate_and_seed():
    a = serve.poisson_arrivals(20000, 100.0, seed=3)
    assert np.all(np.diff(a) >= 0)
    assert abs(20000 / a[-1] - 100.0) < 3.0
    assert np.array_equal(a, serve.poisson_arrivals(20000, 100.0, seed=3))
