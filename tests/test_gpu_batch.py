"""GPU parity of the batched form (many self-joins in one call) and the
served form (R-S queries against a resident index), through the C ABI,
against the CPU oracle instance by instance.  Bit-exact throughout."""
import numpy as np
import pytest

import gen
import oracle
import paper_1711_07295_amd as ssj

pytestmark = pytest.mark.gpu


def _dev(c):
    return ssj.to_device(c.offsets, c.tokens)


def _col(seed, n, universe=400, hi=60, median=10.0, planted=0.15, lo=1):
    return gen.generate(n_sets=n, universe=universe, zipf_s=1.0, size_dist=gen.SIZE_LOGNORMAL,
                        size_a=median, size_b=0.8, size_lo=lo, size_hi=hi,
                        planted_frac=planted, seed=seed)


def _mixed_instances():
    """Uneven instances: empty, tiny, ragged, wide sets, several thresholds."""
    cols = [gen.from_lists([]), gen.from_lists([[3, 4]]), gen.from_lists([[], [], []]),
            gen.from_lists([[1, 2, 3], [1, 2, 3], [2, 3, 4], []])]
    cols += [_col(500 + k, n) for k, n in enumerate((50, 300, 1500, 2500))]
    cols += [_col(600, 1200, universe=3000, hi=700, median=60.0, planted=0.3)]
    pq = [(1, 2), (4, 5), (7, 10), (1, 1), (1, 2), (7, 10), (4, 5), (9, 10), (3, 5)]
    return cols, pq


@pytest.mark.parametrize("b", [0, 64, 128])
def test_batch_matches_oracle_per_instance(b):
    cols, pq = _mixed_instances()
    got, st = ssj.ssj_self_join_batch([_dev(c) for c in cols], [p for p, _ in pq],
                                      [q for _, q in pq], b_bits=b)
    assert len(got) == len(cols)
    band = 0
    for c, (p, q), g in zip(cols, pq, got):
        want = oracle.self_join(c.offsets, c.tokens, p, q)
        assert np.array_equal(g, want), (c.n_sets, p, q, len(g), len(want))
        band += oracle.band_pairs(c.sizes(), p, q)
    assert st["band_pairs"] == band
    assert st["results"] == sum(len(g) for g in got)


def test_many_tasks_with_large_sets_match_the_oracle():
    """48 instances whose largest sets reach 2000 tokens: the library plans
    their width classes on several host threads (the tasks' largest sizes
    sum past its threshold); each instance's pairs equal the oracle's, on
    a repeat of the call too."""
    cols = [_col(900 + k, 120 + 7 * k, universe=20000, hi=2000, median=300.0, planted=0.3, lo=2)
            for k in range(48)]
    pq = [[(1, 2), (7, 10), (4, 5), (9, 10)][k % 4] for k in range(48)]
    devs = [_dev(c) for c in cols]
    assert sum(int(c.sizes().max()) for c in cols) >= 65536
    want = [oracle.self_join(c.offsets, c.tokens, p, q) for c, (p, q) in zip(cols, pq)]
    for _ in range(2):
        got, st = ssj.ssj_self_join_batch(devs, [p for p, _ in pq], [q for _, q in pq])
        for g, w, c, t in zip(got, want, cols, pq):
            assert np.array_equal(g, w), (c.n_sets, t, len(g), len(w))
        assert st["results"] == sum(len(w) for w in want)


def _long_sets():
    """Instances of long sets (medians 60 to 700 tokens, up to 2000): their
    widest width classes run past 512 bits."""
    specs = [(3000, 400.0, (1, 2)), (2500, 150.0, (7, 10)), (6000, 60.0, (4, 5)),
             (1500, 700.0, (1, 2))]
    cols = [_col(950 + k, n, universe=40000, hi=2000, median=m, planted=0.2, lo=2)
            for k, (n, m, _) in enumerate(specs)]
    return cols, [t for _, _, t in specs]


def test_wide_width_classes_match_the_oracle_in_a_call_and_a_plan():
    """The classes past 512 bits build their bitmaps only for the sets their
    row blocks read (their rows and the columns of their bands); every
    instance's pairs equal the oracle's, through the batched call and
    through a prepared plan's replays."""
    cols, pq = _long_sets()
    devs = [_dev(c) for c in cols]
    ps, qs = [p for p, _ in pq], [q for _, q in pq]
    want = [oracle.self_join(c.offsets, c.tokens, p, q) for c, (p, q) in zip(cols, pq)]
    got, st = ssj.ssj_self_join_batch(devs, ps, qs)
    assert max(st["class_bits"][:st["n_classes"]]) >= 1024, st["class_bits"]
    for g, w in zip(got, want):
        assert np.array_equal(g, w)
    with ssj.Plan(devs, ps, qs) as plan:
        for _ in range(2):
            again, _ = plan.execute()
            for g, w in zip(again, want):
                assert np.array_equal(g, w)


def test_wide_width_classes_of_an_rs_join_match_the_oracle():
    """An R-S join of long sets: the row side's wide bitmaps cover the rows
    of the wide classes, the column side's the columns of their bands."""
    r = _col(990, 1200, universe=40000, hi=2000, median=500.0, planted=0.2, lo=2)
    o = _col(991, 1200, universe=40000, hi=2000, median=400.0, planted=0.2, lo=2)
    rows = [r.tokens[r.offsets[k]:r.offsets[k + 1]] for k in range(r.n_sets)]
    other = [o.tokens[o.offsets[k]:o.offsets[k + 1]] for k in range(o.n_sets)]
    # every second row set, less its largest token, is a column set too
    s = gen.from_lists([x[:-1].tolist() for x in rows[::2]] + [x.tolist() for x in other])
    for p, q in [(1, 2), (4, 5)]:
        want = oracle.rs_join(r.offsets, r.tokens, s.offsets, s.tokens, p, q)
        assert len(want) > 0
        got, st = ssj.ssj_rs_join(_dev(r), _dev(s), p, q, b_bits=0)
        assert max(st["class_bits"][:st["n_classes"]]) >= 1024, st["class_bits"]
        assert np.array_equal(got, want)


def test_batch_equals_single_calls_and_resumes_after_overflow():
    cols = [_col(700 + k, n, universe=300, planted=0.3) for k, n in enumerate((3000, 800, 5000))]
    pq = [(1, 2), (1, 2), (3, 5)]
    devs = [_dev(c) for c in cols]
    single = [ssj.ssj_self_join(d, p, q, b_bits=0)[0] for d, (p, q) in zip(devs, pq)]
    for cap, tc in [(0, 0), (1, 0), (7000, 64), (40_000, 5)]:
        got, st = ssj.ssj_self_join_batch(devs, [p for p, _ in pq], [q for _, q in pq],
                                          b_bits=0, queue_capacity=cap, tile_cols=tc)
        for g, s in zip(got, single):
            assert np.array_equal(g, s), (cap, tc)
        if st["survivors"] > max(cap, 4096) and cap:
            assert st["filter_launches"] > st["n_classes"]


def test_batch_no_instances_and_errors():
    got, st = ssj.ssj_self_join_batch([], [], [])
    assert got == [] and st["results"] == 0
    good, bad = gen.from_lists([[1, 2], [1, 2]]), gen.from_lists([[1, 2], [4, 3]])
    with pytest.raises(ssj.SsjError) as e:
        ssj.ssj_self_join_batch([_dev(good), _dev(bad)], [1, 1], [2, 2])
    assert e.value.status == ssj.SSJ_E_UNSORTED
    with pytest.raises(ssj.SsjError) as e:
        ssj.ssj_self_join_batch([_dev(good), _dev(good)], [1, 3], [2, 2])
    assert e.value.status == ssj.SSJ_E_INVALID


def test_batched_workload_sample():
    """48 instances of the batched workload's shape (up to 20,000 sets each):
    every instance bit-exact against the banded oracle."""
    inst = gen.batched_instances(48, n_max=20_000)
    got, st = ssj.ssj_self_join_batch([_dev(c) for c, _ in inst], [t[0] for _, t in inst],
                                      [t[1] for _, t in inst])
    for (c, (p, q)), g in zip(inst, got):
        want, _ = oracle.self_join_banded(c.offsets, c.tokens, p, q)
        assert np.array_equal(g, want), (c.n_sets, p, q)


# ------------------------------------------------------------------- served


@pytest.mark.parametrize("b", [0, 128])
def test_index_queries_match_oracle(b):
    sw = gen.served_workload(12, resident_sets=6000, max_batch=400)
    res = sw.resident
    with ssj.Index(_dev(res), b_bits=b) as idx:
        got, st = idx.query([_dev(x) for x in sw.batches], [t[0] for t in sw.thresholds],
                            [t[1] for t in sw.thresholds])
        for x, (p, q), g in zip(sw.batches, sw.thresholds, got):
            want = oracle.rs_join(x.offsets, x.tokens, res.offsets, res.tokens, p, q)
            assert np.array_equal(g, want), (x.n_sets, p, q)
        # the perturbed copies find their source sets
        assert sum(len(g) for g in got) > 0


def test_index_queries_of_long_sets_match_oracle():
    """An index over long sets (up to 2000 tokens) holds every width; query
    batches of long sets take classes past 512 bits, whose bitmaps and sign
    planes the query side builds only for the rows of those classes."""
    res = _col(995, 2500, universe=40000, hi=2000, median=400.0, planted=0.2, lo=2)
    rows = [res.set(k) for k in range(res.n_sets)]
    batches = []
    for k, n in enumerate((40, 300, 900)):
        own = _col(996 + k, n, universe=40000, hi=2000, median=500.0, planted=0.1, lo=2)
        mine = [own.set(i).tolist() for i in range(own.n_sets)]
        # every 7th resident set, less its largest token, is queried too
        mine += [x[:-1].tolist() for x in rows[k::7][: n // 3]]
        batches.append(gen.from_lists(mine))
    pq = [(1, 2), (7, 10), (4, 5)]
    with ssj.Index(_dev(res)) as idx:
        got, st = idx.query([_dev(x) for x in batches], [t[0] for t in pq], [t[1] for t in pq])
        assert max(st["class_bits"][:st["n_classes"]]) >= 1024, st["class_bits"]
        for x, (p, q), g in zip(batches, pq, got):
            want = oracle.rs_join(x.offsets, x.tokens, res.offsets, res.tokens, p, q)
            assert len(want) > 0
            assert np.array_equal(g, want), (x.n_sets, p, q, len(g), len(want))


def test_index_batch_alone_equals_batch_in_mix():
    sw = gen.served_workload(10, resident_sets=5000, max_batch=300, seed=gen.SEED_BASE + 40)
    res = sw.resident
    d = _dev(res)
    with ssj.Index(d) as idx:
        devs = [_dev(x) for x in sw.batches]
        ps, qs = [t[0] for t in sw.thresholds], [t[1] for t in sw.thresholds]
        mixed, _ = idx.query(devs, ps, qs)
        for k in range(len(devs)):
            alone, _ = idx.query([devs[k]], [ps[k]], [qs[k]])
            assert np.array_equal(alone[0], mixed[k])
            direct, _ = ssj.ssj_rs_join(devs[k], d, ps[k], qs[k], b_bits=0)
            assert np.array_equal(direct, mixed[k])
        # reversed order, and a small queue: same pairs per batch
        rev, _ = idx.query(devs[::-1], ps[::-1], qs[::-1], queue_capacity=1)
        for k in range(len(devs)):
            assert np.array_equal(rev[len(devs) - 1 - k], mixed[k])


def test_index_outlives_the_callers_collection_and_edge_cases():
    res = _col(800, 3000, universe=500)
    d = _dev(res)
    idx = ssj.Index(d)
    want_rows = _col(801, 200, universe=500)
    want = oracle.rs_join(want_rows.offsets, want_rows.tokens, res.offsets, res.tokens, 1, 2)
    del d  # the index holds its own copy
    import torch
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    got, _ = idx.query([_dev(want_rows)], [1], [2])
    assert np.array_equal(got[0], want)
    got, _ = idx.query([], [], [])
    assert got == []
    got, _ = idx.query([_dev(gen.from_lists([])), _dev(gen.from_lists([[], []]))], [1, 1], [2, 2])
    assert [len(g) for g in got] == [0, 0]
    idx.close()
    with pytest.raises(RuntimeError):
        idx.query([_dev(want_rows)], [1], [2])
    with pytest.raises(ssj.SsjError) as e:
        ssj.Index(_dev(gen.from_lists([[2, 1]])))
    assert e.value.status == ssj.SSJ_E_UNSORTED
    empty = ssj.Index(_dev(gen.from_lists([])))
    got, _ = empty.query([_dev(want_rows)], [1], [2])
    assert len(got[0]) == 0
    empty.close()


@pytest.mark.parametrize("b", [0, 64, 128])
def test_rs_join_with_small_r(b):
    """A small R against a large S (few row blocks, long column bands); the
    pairs are (i in R, j in S), ascending."""
    s = _col(900, 4000, universe=600, hi=120, median=20.0, planted=0.3)
    r = gen.from_lists([s.set(k) for k in range(0, 4000, 60)] +
                       [_col(901, 50, universe=600, hi=120, median=20.0).set(k) for k in range(50)])
    assert r.n_sets * 8 < s.n_sets
    for sim, osim, pq in [(ssj.SSJ_SIM_JACCARD, oracle.JACCARD, (1, 2)),
                          (ssj.SSJ_SIM_JACCARD, oracle.JACCARD, (4, 5)),
                          (ssj.SSJ_SIM_COSINE, oracle.COSINE, (7, 10))]:
        p, q = pq
        want = oracle.rs_join(r.offsets, r.tokens, s.offsets, s.tokens, p, q, sim=osim)
        for flags in (0, ssj.SSJ_FLAG_CUTOFF):
            got, st = ssj.ssj_rs_join(_dev(r), _dev(s), p, q, b_bits=b, sim=sim, flags=flags)
            assert np.array_equal(got, want), (b, sim, p, q, flags)
            assert st["band_pairs"] == oracle.band_pairs_rs(r.sizes(), s.sizes(), p, q, sim=osim)


def test_index_small_batches():
    sw = gen.served_workload(6, resident_sets=8000, max_batch=60, seed=gen.SEED_BASE + 41)
    res = sw.resident
    with ssj.Index(_dev(res)) as idx:
        devs = [_dev(x) for x in sw.batches]
        ps, qs = [t[0] for t in sw.thresholds], [t[1] for t in sw.thresholds]
        got, _ = idx.query(devs, ps, qs)
        for x, p, q, g in zip(sw.batches, ps, qs, got):
            want = oracle.rs_join(x.offsets, x.tokens, res.offsets, res.tokens, p, q)
            assert np.array_equal(g, want)
        got_cut, _ = idx.query(devs, ps, qs, flags=ssj.SSJ_FLAG_CUTOFF)
        for a, b in zip(got, got_cut):
            assert np.array_equal(a, b)


def test_served_calls_overlap_and_give_the_same_pairs_alone_and_mixed():
    """Continuous batching with two calls in flight on two streams: batches
    that arrive while a call runs go into the other slot, and every batch's
    pairs equal the oracle's R-S join (Eq. 1) and its own call alone."""
    from paper_1711_07295_amd.serve import ContinuousBatcher
    sw = gen.served_workload(16, resident_sets=20000, max_batch=500, seed=gen.SEED_BASE + 42)
    res = sw.resident
    with ssj.Index(_dev(res)) as idx:
        arr = np.linspace(0.0, 0.004, len(sw.batches))
        srv = ContinuousBatcher(idx, slots=2, memory_budget=8 << 30, queue_capacity=1 << 16,
                                keep_pairs=True, max_batches_per_call=3)
        r = srv.run(sw.batches, sw.thresholds, arr)
        assert r.calls >= 6 and r.max_in_flight == 2, (r.calls, r.max_in_flight)
        assert sorted({d["slot"] for d in r.calls_detail}) == [0, 1]
        alone = ContinuousBatcher(idx, slots=1, keep_pairs=True, max_batches_per_call=1)
        solo = alone.run(sw.batches, sw.thresholds, np.zeros(len(sw.batches)))
        for x, (p, q), g, a in zip(sw.batches, sw.thresholds, r.pairs, solo.pairs):
            want = oracle.rs_join(x.offsets, x.tokens, res.offsets, res.tokens, p, q)
            assert np.array_equal(g, want), (x.n_sets, p, q)
            assert np.array_equal(a, want)
        assert r.results == solo.results == sum(len(g) for g in r.pairs)
