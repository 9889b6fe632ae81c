"""Host logic of the continuous-batching scheduler (no GPU): admission in
arrival order, the per-call memory budget, and the per-batch bookkeeping.
The index is a stub that records what each call receives."""
import numpy as np

import gen
from paper_1711_07295_amd import serve


class StubIndex:
    def __init__(self):
        self.calls = []

    def query(self, views, p, q, queue_capacity=0, flags=0):
        self.calls.append([(v.n_sets, v.n_tokens) for v in views])
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
    per = serve.call_bytes(10, 20)
    srv = serve.ContinuousBatcher(idx, memory_budget=2 * per)
    b = _batches([10] * 5)
    r = srv.run(b, [(1, 2)] * 5, np.zeros(5), device="cpu")
    assert [len(c) for c in idx.calls] == [2, 2, 1]
    assert list(r.batches_per_call) == [2, 2, 1]


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
