"""Prepared joins (ssj_plan_*): the plan is made once from the set sizes and
its first round is replayed from a HIP graph.  Every execution must return
exactly the oracle's pairs (Eq. 1, Table 1 predicate) for the tokens the
buffers hold at that moment, also when the tokens change between
executions, when the survivor queue fills and the host drains and resumes,
and between executions the program interleaves with eager work."""
import numpy as np
import pytest
import torch

import gen
import oracle
import paper_1711_07295_amd as ssj

pytestmark = pytest.mark.gpu


def _dev(c):
    return ssj.to_device(c.offsets, c.tokens)


def _col(seed, n=2500, universe=500, hi=80, median=12.0, planted=0.2):
    return gen.generate(n_sets=n, universe=universe, zipf_s=1.0, size_dist=gen.SIZE_LOGNORMAL,
                        size_a=median, size_b=0.8, size_lo=1, size_hi=hi, planted_frac=planted,
                        seed=seed)


def _same_sizes_new_tokens(c, seed, universe):
    """A collection with c's offsets and, in every set, fresh distinct
    tokens (sorted); a few sets copy others, so that there are pairs."""
    rng = np.random.default_rng(seed)
    sizes = np.diff(c.offsets).astype(np.int64)
    sets = [np.sort(rng.choice(universe, size=int(n), replace=False)) for n in sizes]
    by_size = {}
    for k, n in enumerate(sizes):
        by_size.setdefault(int(n), []).append(k)
    for ks in by_size.values():
        for a, b in zip(ks[::7], ks[1::7]):
            sets[b] = sets[a].copy()
    return gen.from_lists([s.tolist() for s in sets])


@pytest.mark.parametrize("b", [0, 64, 128])
def test_plan_replays_match_the_oracle_and_follow_new_tokens(b):
    c = _col(11)
    d = _dev(c)
    want = oracle.self_join(c.offsets, c.tokens, 7, 10)
    with ssj.Plan([d], [7], [10], b_bits=b) as plan:
        for _ in range(3):
            got, st = plan.execute()
            assert np.array_equal(got[0], want)
            assert st["results"] == len(want)
            # eager work and a synchronisation between replays
            eager, _ = ssj.ssj_self_join(d, 7, 10, b_bits=b)
            assert np.array_equal(eager, want)
            torch.cuda.synchronize()
        # new tokens in the same buffers, same sizes: the replay sees them
        c2 = _same_sizes_new_tokens(c, 5, universe=600)
        assert np.array_equal(c2.offsets, c.offsets)
        d.tokens.copy_(torch.from_numpy(c2.tokens.view(np.int32)).to(d.tokens.device))
        want2 = oracle.self_join(c2.offsets, c2.tokens, 7, 10)
        assert not np.array_equal(want2, want)
        for _ in range(2):
            got, _ = plan.execute()
            assert np.array_equal(got[0], want2)


def test_plan_of_many_instances_equals_the_batched_call_and_the_oracle():
    inst = [(_col(20 + k, n=300 + 400 * k, hi=40 + 30 * k), pq)
            for k, pq in enumerate([(1, 2), (7, 10), (4, 5), (9, 10), (1, 1)])]
    devs = [_dev(c) for c, _ in inst]
    ps, qs = [t[0] for _, t in inst], [t[1] for _, t in inst]
    batched, _ = ssj.ssj_self_join_batch(devs, ps, qs)
    with ssj.Plan(devs, ps, qs) as plan:
        for _ in range(2):
            got, st = plan.execute()
            for (c, (p, q)), g, bt in zip(inst, got, batched):
                assert np.array_equal(g, oracle.self_join(c.offsets, c.tokens, p, q))
                assert np.array_equal(g, bt)
            assert st["band_pairs"] == sum(oracle.band_pairs(c.sizes(), p, q) for c, (p, q) in inst)


def test_plan_drains_a_full_queue_on_every_execution():
    """A queue of 4096 entries at b = 64 and t = 1/2 fills in the graph's
    round; the host drains and resumes, and the pairs stay exact."""
    c = _col(31, n=4000, universe=200, hi=50, median=10.0)
    d = _dev(c)
    want = oracle.self_join(c.offsets, c.tokens, 1, 2)
    with ssj.Plan([d], [1], [2], b_bits=64, queue_capacity=4096) as plan:
        for _ in range(3):
            got, st = plan.execute()
            assert np.array_equal(got[0], want)
            assert st["filter_launches"] > 0  # rounds after the graph's


def test_plan_reports_unsorted_tokens_and_bad_arguments():
    c = _col(41, n=500)
    d = _dev(c)
    with ssj.Plan([d], [4], [5]) as plan:
        got, _ = plan.execute()
        bad = c.tokens.copy()
        k = int(np.argmax(np.diff(c.offsets) >= 2))
        a = int(c.offsets[k])
        bad[a], bad[a + 1] = bad[a + 1], bad[a]  # set k is no longer increasing
        d.tokens.copy_(torch.from_numpy(bad.view(np.int32)).to(d.tokens.device))
        with pytest.raises(ssj.SsjError) as e:
            plan.execute()
        assert e.value.status == ssj.SSJ_E_UNSORTED
        d.tokens.copy_(torch.from_numpy(c.tokens.view(np.int32)).to(d.tokens.device))
        again, _ = plan.execute()
        assert np.array_equal(again[0], got[0])
    with pytest.raises(ssj.SsjError) as e:
        ssj.Plan([], [], [])
    assert e.value.status == ssj.SSJ_E_INVALID
    with pytest.raises(ssj.SsjError) as e:
        ssj.Plan([d], [3], [2])
    assert e.value.status == ssj.SSJ_E_INVALID
