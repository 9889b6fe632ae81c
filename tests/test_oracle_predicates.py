"""Pins of the oracle's predicates against values the paper prints and the
closed forms of Table 1 / Table 2, checked by exact rational arithmetic
(``fractions.Fraction``) and Python's own set operations."""
import json
import os
from fractions import Fraction
from math import isqrt

import numpy as np
import pytest

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def test_binary_sets_example():
    """Section 3.1: r={1,5,8}, s={3,4,5,6} -> overlap 1, union 6, Jaccard 1/6."""
    g = _gold("binary_sets_example.json")
    o, u = oracle.merge_count(g["r"], g["s"])
    assert o == g["popcount_and"] and u == g["popcount_or"]
    # the paper's 1-based bit strings mark exactly the tokens of each set
    for key, toks in (("bits_r_1based", g["r"]), ("bits_s_1based", g["s"])):
        assert [k + 1 for k, ch in enumerate(g[key]) if ch == "1"] == toks
    p, q = g["jaccard"]
    assert Fraction(o, u) == Fraction(p, q)
    assert oracle.similar(oracle.JACCARD, o, u, 3, 4, p, q)          # inclusive at t = 1/6
    assert not oracle.similar(oracle.JACCARD, o, u, 3, 4, 1, 5)      # 1/6 < 1/5


def test_positional_example():
    """Section 2.3.3: |r|=7, |s|=6, overlap at most 4 -> union >= 9 -> J <= 4/9 < 0.6."""
    g = _gold("positional_example.json")
    r = list(range(0, 7))                    # 7 tokens
    s = [3, 4, 5, 6, 100, 101]               # 6 tokens, 4 of them shared
    o, u = oracle.merge_count(r, s)
    assert (len(r), len(s)) == (g["size_r"], g["size_s"])
    assert o == g["max_overlap"] and u == g["min_union"]
    assert Fraction(o, u) == Fraction(*g["jaccard_bound"])
    p, q = g["tau_j"]
    assert not oracle.similar(oracle.JACCARD, o, u, 7, 6, p, q)
    assert oracle.similar(oracle.JACCARD, o, u, 7, 6, 4, 9)
    # Table 2 prefix length for Jaccard: floor((1 - t)|r|) + 1 = 3 for |r| = 7 and |s| = 6
    for n in (7, 6):
        assert int((1 - Fraction(p, q)) * n) + 1 == g["prefix_size"]


@pytest.mark.parametrize("p,q,expect", [(4, 5, True), (9, 10, False), (8, 10, True)])
def test_threshold_is_inclusive(p, q, expect):
    """|r| = |s| = 9 sharing 8 tokens: J = 8/10, in at 4/5 (and 8/10), out at 9/10."""
    r = list(range(9))
    s = list(range(1, 10))
    o, u = oracle.merge_count(r, s)
    assert (o, u) == (8, 10)
    assert oracle.similar(oracle.JACCARD, o, u, 9, 9, p, q) is expect


def test_empty_sets_never_pair():
    """Jaccard of two empty sets is 0/0; one empty set gives 0 for every function."""
    for sim in (oracle.JACCARD, oracle.DICE, oracle.COSINE, oracle.OVERLAP):
        assert not oracle.similar(sim, 0, 0, 0, 0, 1, 2)
        assert not oracle.similar(sim, 0, 3, 0, 3, 1, 2)
    assert oracle.merge_count([], []) == (0, 0)
    assert oracle.merge_count([], [1, 2]) == (0, 2)


def _rand_set(rng, n, universe):
    return sorted(rng.choice(universe, size=n, replace=False).tolist())


def test_merge_count_matches_python_sets():
    rng = np.random.default_rng(7)
    for _ in range(2000):
        a = _rand_set(rng, int(rng.integers(0, 30)), 60)
        b = _rand_set(rng, int(rng.integers(0, 30)), 60)
        assert oracle.merge_count(a, b) == (len(set(a) & set(b)), len(set(a) | set(b)))


def _exact_sim(sim, o, u, nr, ns):
    """Similarity as an exact number, from the definitions in Table 1 (None = undefined)."""
    if sim == oracle.JACCARD:
        return Fraction(o, u) if u else None
    if sim == oracle.DICE:
        return Fraction(2 * o, nr + ns) if nr + ns else None
    if sim == oracle.OVERLAP:
        return Fraction(o)
    if sim == oracle.COSINE:
        m = nr * ns
        if m == 0:
            return None
        return ("cos", o, m)  # compared below without rounding
    raise AssertionError


def _ge(val, p, q):
    if isinstance(val, tuple):
        _, o, m = val
        # o / sqrt(m) >= p / q  with sqrt(m) = r exact when m is a square; otherwise
        # bracket sqrt(m) between isqrt(m) and isqrt(m) + 1 with enough slack, and fall
        # back to the squared comparison only when the bracket cannot decide.
        r = isqrt(m)
        if r * r == m:
            return Fraction(o, r) >= Fraction(p, q)
        lo, hi = Fraction(o, r + 1), Fraction(o, r)  # o/sqrt(m) is strictly inside
        t = Fraction(p, q)
        if lo >= t:
            return True
        if hi < t:
            return False
        # refine with a decimal expansion of sqrt(m) to 40 digits
        from decimal import Decimal, getcontext
        getcontext().prec = 60
        return Decimal(o) / Decimal(m).sqrt() >= Decimal(p) / Decimal(q)
    return val >= Fraction(p, q)


@pytest.mark.parametrize("sim", [oracle.JACCARD, oracle.DICE, oracle.COSINE, oracle.OVERLAP])
def test_similar_matches_table1_definitions(sim):
    rng = np.random.default_rng(11 + sim)
    for _ in range(4000):
        nr, ns = int(rng.integers(1, 40)), int(rng.integers(1, 40))
        o = int(rng.integers(0, min(nr, ns) + 1))
        u = nr + ns - o
        q = int(rng.integers(1, 21))
        p = int(rng.integers(1, q + 1)) if sim != oracle.OVERLAP else int(rng.integers(1, 60))
        val = _exact_sim(sim, o, u, nr, ns)
        assert oracle.similar(sim, o, u, nr, ns, p, q) == _ge(val, p, q), (sim, o, nr, ns, p, q)


def test_cosine_exact_tie():
    """|r| = |s| = 4, overlap 2: cosine = 2/4 = 1/2 exactly, so t = 1/2 is in."""
    assert oracle.similar(oracle.COSINE, 2, 6, 4, 4, 1, 2)
    assert not oracle.similar(oracle.COSINE, 2, 6, 4, 4, 51, 100)


@pytest.mark.parametrize("sim", [oracle.JACCARD, oracle.DICE, oracle.COSINE, oracle.OVERLAP])
def test_length_filter_is_sound_and_tight(sim):
    """Table 2: outside the bounds the pair can never reach t; inside, the best case
    (the smaller set contained in the larger) does reach it."""
    for q in range(1, 11):
        for p in range(1, q + 1):
            for nr in range(1, 25):
                for ns in range(1, 25):
                    best_o = min(nr, ns)
                    best_u = max(nr, ns)
                    best = oracle.similar(sim, best_o, best_u, nr, ns, p, q)
                    assert oracle.length_ok(sim, nr, ns, p, q) == best, (sim, p, q, nr, ns)


def test_length_bound_boundary_inclusive():
    """|r| t <= |s| with equality: |s| = 4, |r| = 5, t = 4/5, s subset of r gives J = 4/5."""
    assert oracle.length_ok(oracle.JACCARD, 5, 4, 4, 5)
    assert not oracle.length_ok(oracle.JACCARD, 5, 3, 4, 5)
    o, u = oracle.merge_count([1, 2, 3, 4, 5], [1, 2, 3, 4])
    assert oracle.similar(oracle.JACCARD, o, u, 5, 4, 4, 5)
