"""Pins of the oracle's branches for the functions other than Jaccard and for
Bitmap-Combined:

  - the normalized threshold (the overlap fraction two n-sets need, the scale
    of the cutoff analysis, Section 3.4) against the predicate of Table 1:
    two n-sets sharing o tokens reach t exactly when o/n reaches it;
  - Bitmap-Combined (Alg. 6, Section 3.5) at the range edges the paper prints
    (0.56 and 0.73 on that scale), and against the cutoff curves (Eqs. 4-6):
    the generator it picks is the one with the largest cutoff, which is how
    the paper motivates the ranges;
  - the bitmap filter's survivors (Alg. 7 over the length band of Table 2)
    for all four functions, against a brute force in exact rationals.
CPU only."""
from fractions import Fraction

import numpy as np
import pytest

import gen
import oracle

SIMS = [oracle.JACCARD, oracle.DICE, oracle.COSINE, oracle.OVERLAP]
METHODS = [oracle.BM_XOR, oracle.BM_SET, oracle.BM_NEXT]


def _sim_value(sim, o, nr, ns):
    """Table 1, as printed: |r n s| / |r u s|, 2|r n s| / (|r| + |s|),
    |r n s| / sqrt(|r||s|) (returned squared, to stay rational) and |r n s|."""
    if sim == oracle.JACCARD:
        return Fraction(o, nr + ns - o)
    if sim == oracle.DICE:
        return Fraction(2 * o, nr + ns)
    if sim == oracle.COSINE:
        return Fraction(o * o, nr * ns)
    return Fraction(o)


def _reaches(sim, value, t):
    return value >= (t * t if sim == oracle.COSINE else t)


@pytest.mark.parametrize("sim", [oracle.JACCARD, oracle.DICE, oracle.COSINE])
def test_normalized_threshold_is_where_equal_sets_flip(sim):
    """Two n-sets sharing o tokens are similar exactly when o/n reaches the
    normalized threshold (Jaccard 2t/(1+t); Dice and Cosine t)."""
    for q in range(1, 13):
        for p in range(1, q + 1):
            tau = oracle.normalized_threshold(sim, p, q)
            for n in range(1, 40):
                for o in range(0, n + 1):
                    want = oracle.similar(sim, o, 2 * n - o, n, n, p, q)
                    assert (Fraction(o, n) >= tau) == want, (sim, p, q, n, o)


def test_normalized_threshold_flip_is_exact_on_the_boundary():
    """At t = 3/5 Dice and Cosine need o/n >= 3/5 and Jaccard o/n >= 3/4:
    n = 20 flips between o = 11 and 12 (Dice, Cosine) and 14 and 15 (Jaccard)."""
    for sim, lo in ((oracle.DICE, 11), (oracle.COSINE, 11), (oracle.JACCARD, 14)):
        assert not oracle.similar(sim, lo, 40 - lo, 20, 20, 3, 5)
        assert oracle.similar(sim, lo + 1, 40 - lo - 1, 20, 20, 3, 5)


# ---- Bitmap-Combined (Alg. 6) -------------------------------------------------

def _normalized(p, q):
    return Fraction(2 * p, p + q)


@pytest.mark.parametrize("p,q,method", [
    (7, 18, oracle.BM_NEXT),          # 2t/(1+t) = 0.56 exactly: Next (tau <= 0.56)
    (7001, 18000, oracle.BM_SET),     # just above 0.56
    (73, 127, oracle.BM_XOR),         # 2t/(1+t) = 0.73 exactly: Xor (tau >= 0.73)
    (7299, 12700, oracle.BM_SET),     # just below 0.73
    (1, 5, oracle.BM_NEXT), (1, 2, oracle.BM_SET), (7, 10, oracle.BM_XOR),
    (1, 1, oracle.BM_XOR)])
def test_combined_at_the_printed_edges(p, q, method):
    tau = _normalized(p, q)
    if (p, q) == (7, 18):
        assert tau == Fraction(56, 100)
    if (p, q) == (73, 127):
        assert tau == Fraction(73, 100)
    assert oracle.combined_method(p, q) == method


@pytest.mark.parametrize("b", [256, 1024, 4096])
def test_combined_picks_the_largest_cutoff(b):
    """Section 3.5: Next has the highest cutoff for small thresholds, Set in the
    middle range and Xor for high ones; Alg. 6 picks by that.  Away from the
    crossings (within 0.02 of 0.56 or 0.73 the curves are too close to order),
    the generator Combined takes has the largest cutoff of Eqs. 4-6."""
    checked = 0
    for tj in [Fraction(k, 100) for k in range(10, 100, 3)]:
        tau = 2 * tj / (1 + tj)
        if abs(tau - Fraction(56, 100)) < Fraction(2, 100) or \
                abs(tau - Fraction(73, 100)) < Fraction(2, 100):
            continue
        cut = {m: oracle.cutoff(m, b, tau) for m in METHODS}
        best = max(cut.values())
        pick = oracle.combined_method(tj.numerator, tj.denominator)
        assert cut[pick] == best, (b, tj, cut, pick)
        checked += 1
    assert checked > 20


def test_combined_bitmaps_are_the_picked_generator():
    c = gen.generate(n_sets=300, universe=700, zipf_s=1.0, size_lo=1, size_hi=90, seed=5)
    for p, q in ((1, 5), (1, 2), (4, 5)):
        m = oracle.combined_method(p, q)
        for b in (64, 192):
            got = oracle.bitmaps(c.offsets, c.tokens, b, oracle.BM_COMBINED, p, q)
            assert np.array_equal(got, oracle.bitmaps(c.offsets, c.tokens, b, m))
    with pytest.raises(ValueError):
        oracle.bitmaps(c.offsets, c.tokens, 64, oracle.BM_COMBINED)


# ---- survivors of the bitmap filter, every function ------------------------

def _popcount_xor(x, y):
    return sum(bin(int(a) ^ int(b)).count("1") for a, b in zip(x, y))


def _brute_survivors(col, bm, sim, p, q):
    """Every pair (i < j) of non-empty sets whose best case (overlap
    min(|r|, |s|)) reaches t -- the length filter, Table 2 -- and whose bound
    floor((|r| + |s| - popcount(b_r xor b_s)) / 2) (Eq. 2) is not below the
    overlap t requires (Alg. 7 against Table 1's threshold)."""
    t = Fraction(p, q)
    sizes = col.sizes()
    band, keep = 0, []
    for i in range(col.n_sets):
        for j in range(i + 1, col.n_sets):
            nr, ns = int(sizes[i]), int(sizes[j])
            if nr == 0 or ns == 0:
                continue
            if not _reaches(sim, _sim_value(sim, min(nr, ns), nr, ns), t):
                continue
            band += 1
            ub = (nr + ns - _popcount_xor(bm[i], bm[j])) // 2
            if sim == oracle.JACCARD:
                need = t / (1 + t) * (nr + ns)
                ok = not ub < need
            elif sim == oracle.DICE:
                ok = not ub < t / 2 * (nr + ns)
            elif sim == oracle.COSINE:
                ok = not ub * ub < t * t * nr * ns
            else:
                ok = not ub < t
            if ok:
                keep.append((i, j))
    return band, np.array(keep, dtype=np.uint32).reshape(-1, 2)


@pytest.mark.parametrize("sim", SIMS)
@pytest.mark.parametrize("method", METHODS)
def test_survivors_every_function_bruteforce(sim, method):
    c = gen.generate(n_sets=260, universe=90, zipf_s=1.0, size_dist=gen.SIZE_LOGNORMAL,
                     size_a=7.0, size_b=0.8, size_lo=1, size_hi=40, planted_frac=0.2,
                     seed=100 + 10 * sim + method)
    thresholds = [(1, 2), (7, 10), (9, 10)] if sim != oracle.OVERLAP else [(3, 1), (5, 2), (7, 1)]
    for b in (64, 128):
        bm = oracle.bitmaps(c.offsets, c.tokens, b, method)
        for p, q in thresholds:
            band, want = _brute_survivors(c, bm, sim, p, q)
            cnt, got_band, got = oracle.survivors(c.offsets, bm, b, p, q, listing=True, sim=sim)
            assert got_band == band and cnt == len(want)
            assert np.array_equal(got, want), (sim, method, b, p, q)
            # no false negatives (Theorem 1): every result survives
            res = oracle.self_join(c.offsets, c.tokens, p, q, sim=sim)
            assert set(map(tuple, res.tolist())) <= set(map(tuple, got.tolist()))


def test_bitmap_survives_every_function_exact():
    """The integer decision against the printed thresholds of Table 1, over a
    grid of sizes, distances and thresholds (exact rationals; Cosine squared)."""
    for sim in SIMS:
        for p, q in ((1, 2), (2, 3), (4, 5), (9, 10), (1, 1), (3, 1)):
            if sim != oracle.OVERLAP and p > q:
                continue
            t = Fraction(p, q)
            for nr in range(1, 16):
                for ns in range(1, 16):
                    for h in range(0, nr + ns + 1):
                        ub = (nr + ns - h) // 2
                        if sim == oracle.JACCARD:
                            want = not ub < t / (1 + t) * (nr + ns)
                        elif sim == oracle.DICE:
                            want = not ub < t / 2 * (nr + ns)
                        elif sim == oracle.COSINE:
                            want = not Fraction(ub * ub) < t * t * nr * ns
                        else:
                            want = not ub < t
                        assert oracle.bitmap_survives(nr, ns, h, p, q, sim=sim) == want
                        if sim == oracle.JACCARD:
                            assert oracle.bitmap_survives(nr, ns, h, p, q) == want
