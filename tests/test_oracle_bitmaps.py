"""Pins of the oracle's bitmap generators (Alg. 3-5), the overlap bound of
Theorem 1 (Eq. 2) and the filter decision (Alg. 7): hand-computed bitmaps,
order independence, parity, the exact no-collision case, no false
negatives, the Fig. 4 arithmetic, and Monte Carlo means against the closed
forms of Eqs. 4-6."""
import json
import os

import numpy as np
import pytest

import gen
import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")
METHODS = [oracle.BM_XOR, oracle.BM_SET, oracle.BM_NEXT]


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def _bits(words):
    out = []
    for w, x in enumerate(words):
        x = int(x)
        out += [64 * w + k for k in range(64) if (x >> k) & 1]
    return out


def _popcount(words):
    return sum(bin(int(x)).count("1") for x in words)


def test_hand_bitmaps_b64():
    """tokens {0, 64, 65, 130} with h(t) = t mod 64 -> slots 0, 0, 1, 2."""
    toks = [0, 64, 65, 130]
    assert _bits(oracle.bitmap(toks, 64, oracle.BM_SET)) == [0, 1, 2]
    assert _bits(oracle.bitmap(toks, 64, oracle.BM_XOR)) == [1, 2]       # slot 0 flipped twice
    assert _bits(oracle.bitmap(toks, 64, oracle.BM_NEXT)) == [0, 1, 2, 3]  # 64 -> 1, 65 -> 2, 130 -> 3


def test_next_wraps_around_and_saturates():
    assert _bits(oracle.bitmap([63, 127], 64, oracle.BM_NEXT)) == [0, 63]   # 127 -> slot 63 busy -> 0
    assert _popcount(oracle.bitmap(list(range(64)), 64, oracle.BM_NEXT)) == 64
    full = oracle.bitmap(list(range(0, 200, 3)), 64, oracle.BM_NEXT)     # n = 67 >= b
    assert _popcount(full) == 64


def test_word_layout_b128():
    bm = oracle.bitmap([0, 63, 64, 127, 128, 300], 128, oracle.BM_XOR)
    # 128 mod 128 = 0 cancels token 0; 300 mod 128 = 44
    assert _bits(bm) == [44, 63, 64, 127]
    assert int(bm[1]) == (1 << 0) | (1 << 63)


def test_bitmap_width_non_power_of_two():
    bm = oracle.bitmap([5, 197, 191, 383], 192, oracle.BM_XOR)   # 197 -> 5 cancels; 383 -> 191
    assert _bits(bm) == []
    assert _bits(oracle.bitmap([5, 197, 191, 383], 192, oracle.BM_SET)) == [5, 191]


def test_invalid_width_rejected():
    with pytest.raises(ValueError):
        oracle.bitmap([1, 2], 100, oracle.BM_XOR)


@pytest.mark.parametrize("method", METHODS)
def test_order_independence(method):
    """Section 3.3: each generator is an associative, commutative series of operations."""
    rng = np.random.default_rng(100 + method)
    for b in (64, 128, 192):
        for _ in range(300):
            n = int(rng.integers(0, 2 * b // 3 + 5))
            toks = rng.choice(10 * b, size=n, replace=False)
            a = oracle.bitmap(np.sort(toks), b, method)
            for _ in range(3):
                assert np.array_equal(a, oracle.bitmap(rng.permutation(toks), b, method))


def test_xor_parity_and_set_next_counts():
    rng = np.random.default_rng(5)
    for b in (64, 128, 256):
        for _ in range(300):
            n = int(rng.integers(0, 400))
            toks = rng.choice(100000, size=n, replace=False)
            slots = set(int(t) % b for t in toks)
            assert _popcount(oracle.bitmap(toks, b, oracle.BM_XOR)) % 2 == n % 2
            assert _popcount(oracle.bitmap(toks, b, oracle.BM_SET)) == len(slots)
            assert _popcount(oracle.bitmap(toks, b, oracle.BM_NEXT)) == min(n, b)


def test_xor_is_parity_of_slot_counts():
    rng = np.random.default_rng(6)
    for _ in range(200):
        toks = rng.choice(5000, size=int(rng.integers(0, 300)), replace=False)
        counts = np.bincount(toks % 128, minlength=128)
        assert _bits(oracle.bitmap(toks, 128, oracle.BM_XOR)) == np.nonzero(counts % 2)[0].tolist()


def test_fig4_arithmetic():
    g = _gold("overlap_bound_example.json")
    fits = [L for L in range(10, 40)
            if oracle.overlap_ub(L // 2, L - L // 2, g["set_hamming"]) == g["set_bound"]]
    assert fits == g["size_sum_candidates"]
    for L in fits:
        h = L - 2 * g["xor_next_bound"]          # even L - h: the xor/next parity
        assert (L - h) % 2 == 0
        assert oracle.overlap_ub(L // 2, L - L // 2, h) == g["xor_next_bound"]
        # two more differing bits cost one unit of the bound
        assert oracle.overlap_ub(L // 2, L - L // 2, h + 2) == g["xor_next_bound"] - 1


def _pairs_collection(rng, n_pairs, max_n, universe, share=True):
    sets, overl = [], []
    for _ in range(n_pairs):
        na, nb = int(rng.integers(0, max_n)), int(rng.integers(0, max_n))
        pool = rng.choice(universe, size=na + nb, replace=False)
        a = pool[:na]
        b = pool[na:na + nb]
        if share and na and nb:
            k = int(rng.integers(0, min(na, nb) + 1))
            b = np.concatenate([a[:k], b[k:]])
        sets.append(np.sort(a)); sets.append(np.sort(b))
        overl.append(len(set(a.tolist()) & set(b.tolist())))
    return gen.from_lists(sets), np.array(overl)


@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("b", [64, 128, 192])
def test_theorem1_no_false_negatives(method, b):
    """Eq. 2 bounds the true overlap for every pair and every generator."""
    rng = np.random.default_rng(b + method)
    c, o = _pairs_collection(rng, 3000, 150, 20000)
    bm = oracle.bitmaps(c.offsets, c.tokens, b, method)
    sz = c.sizes()
    for k in range(len(o)):
        h = _popcount(np.bitwise_xor(bm[2 * k], bm[2 * k + 1]))
        ub = oracle.overlap_ub(int(sz[2 * k]), int(sz[2 * k + 1]), h)
        assert ub >= o[k]


@pytest.mark.parametrize("method", METHODS)
def test_exact_when_no_collisions(method):
    """b above the largest token: the bitmap is the set's characteristic vector, the
    xor weight is |r xor s| and the bound equals the overlap."""
    rng = np.random.default_rng(40 + method)
    c, o = _pairs_collection(rng, 1000, 30, 256)
    bm = oracle.bitmaps(c.offsets, c.tokens, 256, method)
    sz = c.sizes()
    for k in range(len(o)):
        h = _popcount(np.bitwise_xor(bm[2 * k], bm[2 * k + 1]))
        assert oracle.overlap_ub(int(sz[2 * k]), int(sz[2 * k + 1]), h) == o[k]


def test_filter_decision_matches_table1_threshold():
    """Alg. 7 prunes when the bound is below t/(1+t)(|r|+|s|), Table 1 (exact)."""
    from fractions import Fraction
    for q in range(1, 12):
        for p in range(1, q + 1):
            t = Fraction(p, q)
            for nr in range(1, 20):
                for ns in range(1, 20):
                    for h in range(0, nr + ns + 1):
                        if (nr + ns - h) % 2:
                            continue
                        ub = (nr + ns - h) // 2
                        tau = t / (1 + t) * (nr + ns)
                        assert oracle.bitmap_survives(nr, ns, h, p, q) == (not ub < tau)


@pytest.mark.parametrize("p,q", [(1, 2), (4, 5), (9, 10)])
def test_survivors_superset_of_results(p, q):
    c = gen.generate(n_sets=1500, universe=500, zipf_s=1.0, size_dist=gen.SIZE_LOGNORMAL,
                     size_a=10.0, size_b=0.7, size_lo=1, size_hi=80, planted_frac=0.15, seed=31)
    res = set(map(tuple, oracle.self_join(c.offsets, c.tokens, p, q).tolist()))
    assert res
    for method in METHODS:
        bm = oracle.bitmaps(c.offsets, c.tokens, 64, method)
        cnt, band, surv = oracle.survivors(c.offsets, bm, 64, p, q, listing=True)
        sv = set(map(tuple, surv.tolist()))
        assert cnt == len(sv) and band == oracle.band_pairs(c.sizes(), p, q)
        assert res <= sv


def test_survivors_equal_results_without_collisions():
    c = gen.generate(n_sets=1200, universe=60, zipf_s=1.0, size_lo=1, size_hi=20,
                     planted_frac=0.2, seed=37)
    assert int(c.tokens.max()) < 64
    for p, q in [(1, 2), (7, 10), (9, 10)]:
        res = oracle.self_join(c.offsets, c.tokens, p, q)
        bm = oracle.bitmaps(c.offsets, c.tokens, 64, oracle.BM_XOR)
        cnt, _, surv = oracle.survivors(c.offsets, bm, 64, p, q, listing=True)
        assert np.array_equal(surv, res)


# ---- Eqs. 4-6: expected overlap bound of two random disjoint n-sets ----------

def _eq4_set(b, n):
    return oracle.expected_bound(oracle.BM_SET, b, n)


def _eq5_xor(b, n):
    return oracle.expected_bound(oracle.BM_XOR, b, n)


def _eq6_next(b, n):
    return oracle.expected_bound(oracle.BM_NEXT, b, n)


def _mean_bound(method, b, n, pairs, seed):
    rng = np.random.default_rng(seed)
    sets = []
    for _ in range(pairs):
        t = rng.choice(1 << 30, size=2 * n, replace=False)
        sets.append(np.sort(t[:n])); sets.append(np.sort(t[n:]))
    c = gen.from_lists(sets)
    bm = oracle.bitmaps(c.offsets, c.tokens, b, method)
    x = np.bitwise_xor(bm[0::2], bm[1::2])
    h = np.array([sum(bin(int(w)).count("1") for w in row) for row in x])
    ub = (2 * n - h) / 2.0   # Eq. 2 without the floor, as the closed forms are
    return ub.mean(), ub.std() / np.sqrt(pairs)


@pytest.mark.parametrize("method,eq", [(oracle.BM_SET, _eq4_set), (oracle.BM_XOR, _eq5_xor),
                                       (oracle.BM_NEXT, _eq6_next)])
@pytest.mark.parametrize("n", [1, 10, 55, 100])
def test_expected_bound_closed_forms(method, eq, n):
    mean, se = _mean_bound(method, 64, n, 20000, seed=1000 * n + method)
    assert abs(mean - eq(64, n)) <= 4.5 * se + 1e-9, (mean, eq(64, n), se)


def test_expected_bound_at_55():
    """Section 3.4: at b = 64, n = 55 the normalized bound is about 0.72 for Set and Xor."""
    g = _gold("expected_bound_b64.json")
    for eq in (_eq4_set, _eq5_xor):
        assert abs(eq(g["b"], g["n"]) / g["n"] - g["normalized_bound_set_xor"]) <= \
            g["normalized_bound_rounding"]
