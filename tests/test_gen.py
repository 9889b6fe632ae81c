"""The seeded input generator: determinism, CSR validity and the shape of
the named workloads (token frequency order, size law, planted clusters)."""
import numpy as np
import pytest

import gen


def test_deterministic_and_thread_independent():
    cfg = dict(gen.WORKLOADS["selfjoin-10k"]["gen"])
    a = gen.generate(**cfg)
    b = gen.generate(**cfg)
    c = gen.generate(**dict(cfg, n_threads=3))
    assert a.checksum() == b.checksum() == c.checksum()
    d = gen.generate(**dict(cfg, seed=cfg["seed"] + 1))
    assert d.checksum() != a.checksum()


def _check_csr(c):
    assert c.offsets[0] == 0 and c.offsets[-1] == c.n_tokens
    assert np.all(np.diff(c.offsets.astype(np.int64)) >= 0)
    for k in range(c.n_sets):
        s = c.set(k).astype(np.int64)
        assert np.all(np.diff(s) > 0)


def test_selfjoin_10k_shape():
    c = gen.workload("selfjoin-10k")
    _check_csr(c)
    sz = c.sizes()
    assert c.n_sets == 10_000 and sz.min() >= 5 and sz.max() <= 50
    assert abs(sz.mean() - 27.5) < 0.5
    # relabelled by ascending global frequency: id order is frequency order
    freq = np.bincount(c.tokens, minlength=c.n_distinct)
    assert c.n_distinct == int(c.tokens.max()) + 1
    assert np.all(np.diff(freq) >= 0)


def test_lognormal_sizes_and_planted_clusters():
    c = gen.generate(n_sets=40_000, universe=40_000, zipf_s=1.1, size_dist=gen.SIZE_LOGNORMAL,
                     size_a=20.0, size_b=0.8, size_lo=2, size_hi=500, planted_frac=0.05,
                     seed=99)
    _check_csr(c)
    sz = c.sizes()
    assert sz.min() >= 2 and sz.max() <= 500
    assert 19 <= np.median(sz) <= 21
    # planted copies of small sets (n <= 4 gets no swaps) show up as exact duplicates;
    # without planting, exact duplicates are far rarer
    def dups(col):
        seen, d = set(), 0
        for k in range(col.n_sets):
            t = col.set(k).tobytes()
            d += t in seen
            seen.add(t)
        return d
    free = gen.generate(n_sets=40_000, universe=40_000, zipf_s=1.1,
                        size_dist=gen.SIZE_LOGNORMAL, size_a=20.0, size_b=0.8, size_lo=2,
                        size_hi=500, planted_frac=0.0, seed=99)
    assert dups(c) >= 40 and dups(c) >= 3 * max(dups(free), 1)


def test_uniform_and_poisson_without_relabel():
    c = gen.generate(n_sets=5000, universe=220, zipf_s=0.0, size_dist=gen.SIZE_POISSON,
                     size_a=10.0, size_lo=1, size_hi=220, relabel=False, seed=4)
    _check_csr(c)
    assert int(c.tokens.max()) < 220
    assert abs(c.sizes().mean() - 10.0) < 0.3


def test_from_lists_and_subset():
    c = gen.from_lists([[1, 2], [], [7]])
    assert c.offsets.tolist() == [0, 2, 2, 3] and c.tokens.tolist() == [1, 2, 7]
    s = c.subset([2, 0])
    assert s.offsets.tolist() == [0, 1, 3] and s.tokens.tolist() == [7, 1, 2]


@pytest.mark.parametrize("name", ["selfjoin-1m", "selfjoin-10m", "resident-5m"])
def test_scaled_workloads_are_valid(name):
    c = gen.workload(name, n_sets=20_000)
    _check_csr(c)


def test_batched_instances_are_seeded_and_shaped():
    a = gen.batched_instances(6, n_max=3000)
    b = gen.batched_instances(6, n_max=3000)
    assert [c.checksum() for c, _ in a] == [c.checksum() for c, _ in b]
    for c, t in a:
        assert 1000 <= c.n_sets <= 3000
        s = c.sizes()
        assert s.min() >= 2 and s.max() <= 2000
        assert t in gen.BATCH_THRESHOLDS
        for k in range(0, c.n_sets, 97):
            x = c.set(k)
            assert np.all(np.diff(x.astype(np.int64)) > 0)


def test_served_workload_copies_and_fresh_sets():
    sw = gen.served_workload(8, resident_sets=3000, max_batch=200)
    assert sw.resident.n_sets == 3000 and len(sw.batches) == 8
    assert all(t in gen.SERVE_THRESHOLDS for t in sw.thresholds)
    res = {tuple(sw.resident.set(k)) for k in range(sw.resident.n_sets)}
    n_copy = n_close = 0
    for bt, cp in zip(sw.batches, sw.copies):
        assert bt.n_sets == len(cp)
        for k in range(bt.n_sets):
            x = bt.set(k)
            assert np.all(np.diff(x.astype(np.int64)) > 0)
            if cp[k]:
                n_copy += 1
                # a copy keeps about 90% of some resident set
                xs = set(int(v) for v in x)
                best = max(len(xs & set(r)) / len(xs) for r in res if abs(len(r) - len(xs)) <= 1)
                n_close += best >= 0.8
    assert n_copy > 0 and n_close == n_copy
