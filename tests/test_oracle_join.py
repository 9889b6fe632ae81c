"""Pins of the oracle's joins: brute force over Python sets with exact
fractions on tiny inputs, the invariants of Eq. 1 (symmetry, transpose,
relabelling, monotonicity in t), and banded == plain (Table 2)."""
from fractions import Fraction

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import gen
import oracle


def _brute_self(sets, p, q):
    t = Fraction(p, q)
    out = []
    for i in range(len(sets)):
        for j in range(i + 1, len(sets)):
            a, b = set(sets[i]), set(sets[j])
            if a | b and Fraction(len(a & b), len(a | b)) >= t:
                out.append((i, j))
    return out


def _brute_rs(rsets, ssets, p, q):
    t = Fraction(p, q)
    out = []
    for i, a in enumerate(rsets):
        for j, b in enumerate(ssets):
            a_, b_ = set(a), set(b)
            if a_ | b_ and Fraction(len(a_ & b_), len(a_ | b_)) >= t:
                out.append((i, j))
    return out


def _as_list(pairs):
    return [tuple(map(int, x)) for x in pairs]


sets_strategy = st.lists(st.lists(st.integers(0, 24), max_size=12, unique=True).map(sorted),
                         max_size=14)
thr_strategy = st.integers(1, 10).flatmap(lambda q: st.tuples(st.integers(1, q), st.just(q)))


@settings(max_examples=200, deadline=None)
@given(sets_strategy, thr_strategy)
def test_self_join_matches_bruteforce(sets, pq):
    p, q = pq
    c = gen.from_lists(sets)
    got = _as_list(oracle.self_join(c.offsets, c.tokens, p, q, threads=2))
    assert got == _brute_self(sets, p, q)


@settings(max_examples=200, deadline=None)
@given(sets_strategy, sets_strategy, thr_strategy)
def test_rs_join_matches_bruteforce_and_transpose(rsets, ssets, pq):
    p, q = pq
    r, s = gen.from_lists(rsets), gen.from_lists(ssets)
    got = _as_list(oracle.rs_join(r.offsets, r.tokens, s.offsets, s.tokens, p, q, threads=2))
    assert got == _brute_rs(rsets, ssets, p, q)
    back = _as_list(oracle.rs_join(s.offsets, s.tokens, r.offsets, r.tokens, p, q, threads=2))
    assert sorted((j, i) for i, j in back) == got


@settings(max_examples=100, deadline=None)
@given(sets_strategy, thr_strategy)
def test_self_join_is_upper_triangle_of_rs(sets, pq):
    p, q = pq
    c = gen.from_lists(sets)
    full = _as_list(oracle.rs_join(c.offsets, c.tokens, c.offsets, c.tokens, p, q, threads=2))
    tri = [(i, j) for i, j in full if i < j]
    assert _as_list(oracle.self_join(c.offsets, c.tokens, p, q, threads=2)) == tri


@settings(max_examples=100, deadline=None)
@given(sets_strategy, thr_strategy, st.randoms(use_true_random=False))
def test_relabelling_sets_relabels_pairs(sets, pq, rnd):
    p, q = pq
    perm = list(range(len(sets)))
    rnd.shuffle(perm)
    c = gen.from_lists(sets)
    c2 = gen.from_lists([sets[k] for k in perm])
    a = _as_list(oracle.self_join(c.offsets, c.tokens, p, q, threads=2))
    b = _as_list(oracle.self_join(c2.offsets, c2.tokens, p, q, threads=2))
    mapped = sorted(tuple(sorted((perm[i], perm[j]))) for i, j in b)
    assert mapped == a


def test_monotone_in_threshold():
    c = gen.generate(n_sets=600, universe=80, zipf_s=1.0, size_lo=2, size_hi=12,
                     planted_frac=0.2, seed=5)
    prev = None
    for p, q in [(1, 2), (3, 5), (7, 10), (4, 5), (9, 10), (1, 1)]:
        cur = set(_as_list(oracle.self_join(c.offsets, c.tokens, p, q)))
        if prev is not None:
            assert cur <= prev
        prev = cur
    assert prev  # planted exact duplicates stay at t = 1


def test_planted_exact_duplicates_always_reported():
    sets = [[1, 2, 3], [4, 5], [1, 2, 3], [9], [4, 5], [1, 2, 3]]
    c = gen.from_lists(sets)
    got = set(_as_list(oracle.self_join(c.offsets, c.tokens, 1, 1)))
    assert got == {(0, 2), (0, 5), (2, 5), (1, 4)}


@pytest.mark.parametrize("p,q", [(1, 2), (7, 10), (4, 5), (9, 10)])
def test_banded_equals_plain(p, q):
    c = gen.generate(n_sets=3000, universe=400, zipf_s=1.0, size_dist=gen.SIZE_LOGNORMAL,
                     size_a=8.0, size_b=0.8, size_lo=1, size_hi=60, planted_frac=0.1, seed=17)
    plain = oracle.self_join(c.offsets, c.tokens, p, q)
    banded, evaluated = oracle.self_join_banded(c.offsets, c.tokens, p, q)
    assert np.array_equal(plain, banded)
    assert evaluated == oracle.band_pairs(c.sizes(), p, q)
    assert len(plain) > 0


def test_band_pairs_bruteforce():
    rng = np.random.default_rng(3)
    sizes = rng.integers(0, 30, size=200)
    for p, q in [(1, 2), (4, 5), (1, 1), (2, 3)]:
        brute = sum(1 for i in range(200) for j in range(i + 1, 200)
                    if sizes[i] and sizes[j]
                    and q * min(sizes[i], sizes[j]) >= p * max(sizes[i], sizes[j]))
        assert oracle.band_pairs(sizes, p, q) == brute


def test_sampled_rows_agree_with_full_join():
    c = gen.generate(n_sets=2000, universe=300, zipf_s=1.1, size_lo=2, size_hi=25,
                     planted_frac=0.1, seed=23)
    full = _as_list(oracle.self_join(c.offsets, c.tokens, 1, 2))
    rows = [0, 5, 17, 999, 1500, 1999]
    sub = _as_list(oracle.self_join_rows(c.offsets, c.tokens, rows, 1, 2))
    assert sub == [x for x in full if x[0] in rows or x[1] in rows]
    assert sub


def test_banded_rows_subset():
    c = gen.generate(n_sets=2000, universe=300, zipf_s=1.1, size_lo=2, size_hi=25,
                     planted_frac=0.1, seed=29)
    order = oracle.size_order(c.offsets)
    full, ev_all = oracle.self_join_banded(c.offsets, c.tokens, 1, 2, order=order)
    rows = np.arange(0, 2000, 7)
    part, ev = oracle.self_join_banded(c.offsets, c.tokens, 1, 2, rows=rows, order=order)
    # pairs found by a processed row: (order[x], order[y]) with y < x
    pos = np.empty(2000, dtype=np.int64)
    pos[order] = np.arange(2000)
    keep = set(int(x) for x in rows)
    expect = [tuple(map(int, x)) for x in full if max(pos[x[0]], pos[x[1]]) in keep]
    assert _as_list(part) == expect
    assert 0 < ev < ev_all


def test_size_order():
    c = gen.from_lists([[1, 2, 3], [4], [5, 6], [7], []])
    assert oracle.size_order(c.offsets).tolist() == [4, 1, 3, 2, 0]


def test_check_pairs_agrees_with_join():
    c = gen.generate(n_sets=800, universe=90, zipf_s=1.0, size_lo=1, size_hi=12,
                     planted_frac=0.2, seed=41)
    res = oracle.self_join(c.offsets, c.tokens, 3, 5)
    assert oracle.check_pairs(c.offsets, c.tokens, c.offsets, c.tokens, res, 3, 5).all()
    found = set(map(tuple, res.tolist()))
    rng = np.random.default_rng(1)
    cand = rng.integers(0, 800, size=(3000, 2)).astype(np.uint32)
    cand = cand[cand[:, 0] < cand[:, 1]]
    ok = oracle.check_pairs(c.offsets, c.tokens, c.offsets, c.tokens, cand, 3, 5)
    assert ok.tolist() == [tuple(x) in found for x in cand.tolist()]


def test_band_pairs_rs_bruteforce():
    rng = np.random.default_rng(5)
    r = rng.integers(0, 30, size=60)
    s = rng.integers(0, 30, size=80)
    for sim in (oracle.JACCARD, oracle.DICE, oracle.COSINE):
        for p, q in ((1, 2), (4, 5), (1, 1)):
            want = sum(1 for a in r for c in s
                       if a and c and oracle.length_ok(sim, int(a), int(c), p, q))
            assert oracle.band_pairs_rs(r, s, p, q, sim=sim) == want
