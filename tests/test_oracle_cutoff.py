"""Pins of the oracle's expected bound (Eqs. 4-6) and cutoff point (Section
3.4), and the library's cutoff (a host function of the C ABI) against them.
CPU only."""
import json
import os

import numpy as np
import pytest

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def test_worked_example_b64():
    g = _gold("cutoff_example.json")["example"]
    for m in (oracle.BM_SET, oracle.BM_XOR):
        assert oracle.cutoff(m, g["b"], g["normalized_tau"]) == g["cutoff"]


def test_b1024_values_and_ratios():
    g = _gold("cutoff_example.json")["b1024"]
    t9 = oracle.normalized_threshold(oracle.JACCARD, 9, 10)
    t8 = oracle.normalized_threshold(oracle.JACCARD, 4, 5)
    set9 = oracle.cutoff(oracle.BM_SET, 1024, t9)
    xor9 = oracle.cutoff(oracle.BM_XOR, 1024, t9)
    # the printed Set value rounds the crossing up; ours is the last size below it
    assert set9 + 1 == g["jaccard_0.9"]["set_printed"]
    assert round(xor9 / set9, 1) == g["jaccard_0.9"]["xor_over_set"]
    xor8, set8 = oracle.cutoff(oracle.BM_XOR, 1024, t8), oracle.cutoff(oracle.BM_SET, 1024, t8)
    assert round(xor8 / set8, 2) == g["jaccard_0.8"]["xor_over_set"]
    # Eq. 5 crosses 0.9's normalized threshold between 4863 and 4864, not at
    # the printed 4983
    assert xor9 == 4863 and g["jaccard_0.9"]["xor_printed"] != xor9


def test_next_cutoff_is_tau_times_b():
    """Eq. 6: E/n = n/b below saturation, so the cutoff is floor(tau b)."""
    for b in (64, 256, 1000):
        for tau in (0.1, 0.5, 0.73, 0.99):
            assert oracle.cutoff(oracle.BM_NEXT, b, tau) == int(np.floor(tau * b + 1e-12))


def test_xor_sum_against_its_odd_term_identity_and_limits():
    """Eq. 5's odd-k sum equals (1 - (1 - 2/b)^(2n)) / 2 (the odd half of the
    binomial expansion); E(b, 1) = 1/b; E(b, n)/n tends to 1 - b/(4n)."""
    for b in (64, 128, 4096):
        for n in (1, 7, 55, 300):
            e = oracle.expected_bound(oracle.BM_XOR, b, n)
            assert abs(e - (n - b / 4 * (1 - (1 - 2 / b) ** (2 * n)))) < 1e-9 * n
        assert abs(oracle.expected_bound(oracle.BM_XOR, b, 1) - 1 / b) < 1e-12
    big = 200_000
    assert abs(oracle.expected_bound(oracle.BM_XOR, 64, big) - (big - 16)) < 1e-6


def test_normalized_bound_grows_with_n():
    for m in (oracle.BM_SET, oracle.BM_XOR, oracle.BM_NEXT):
        v = [oracle.expected_bound(m, 128, n) / n for n in range(1, 400)]
        assert all(b >= a - 1e-15 for a, b in zip(v, v[1:]))


def _lib_cutoff(b, method, sim, p, q):
    import ctypes
    import paper_1711_07295_amd as ssj
    out = ctypes.c_uint32()
    st = ssj.load().ssj_cutoff(b, method, sim, p, q, ctypes.byref(out))
    return st, out.value


@pytest.mark.parametrize("b", [64, 128, 192, 256, 512, 1024, 4096])
def test_library_cutoff_matches_oracle(b):
    import paper_1711_07295_amd as ssj
    if not os.path.exists(ssj.LIB_PATH):
        pytest.skip("library not built")
    for method, om in ((ssj.SSJ_BM_XOR, oracle.BM_XOR), (ssj.SSJ_BM_SET, oracle.BM_SET),
                       (ssj.SSJ_BM_NEXT, oracle.BM_NEXT)):
        for sim, osim in ((ssj.SSJ_SIM_JACCARD, oracle.JACCARD), (ssj.SSJ_SIM_DICE, oracle.DICE),
                          (ssj.SSJ_SIM_COSINE, oracle.COSINE)):
            for p, q in ((1, 2), (7, 10), (4, 5), (9, 10), (19, 20)):
                st, got = _lib_cutoff(b, method, sim, p, q)
                assert st == ssj.SSJ_OK
                want = oracle.cutoff(om, b, oracle.normalized_threshold(osim, p, q))
                assert got == want, (b, method, sim, p, q, got, want)
    # Bitmap-Combined: the cutoff of the generator Alg. 6 picks for the
    # function's normalized threshold (for Dice and Cosine t, which is the
    # normalized value of the Jaccard threshold t / (2 - t))
    from fractions import Fraction
    for sim, osim in ((ssj.SSJ_SIM_JACCARD, oracle.JACCARD), (ssj.SSJ_SIM_DICE, oracle.DICE),
                      (ssj.SSJ_SIM_COSINE, oracle.COSINE)):
        for p, q in ((1, 5), (1, 3), (1, 2), (3, 5), (7, 10), (4, 5), (9, 10)):
            tau = oracle.normalized_threshold(osim, p, q)
            tj = tau / (2 - tau)
            om = oracle.combined_method(tj.numerator, tj.denominator)
            st, got = _lib_cutoff(b, ssj.SSJ_BM_COMBINED, sim, p, q)
            assert st == ssj.SSJ_OK and got == oracle.cutoff(om, b, tau), (b, sim, p, q)
            assert 2 * tj / (1 + tj) == tau and isinstance(tj, Fraction)
    # Overlap has no normalized threshold: the filter is never cut off
    st, got = _lib_cutoff(b, ssj.SSJ_BM_XOR, ssj.SSJ_SIM_OVERLAP, 3, 1)
    assert st == ssj.SSJ_OK and got == 0xFFFFFFFF
    assert _lib_cutoff(b, 7, ssj.SSJ_SIM_JACCARD, 1, 2)[0] == ssj.SSJ_E_UNSUPPORTED
    assert _lib_cutoff(100, ssj.SSJ_BM_XOR, ssj.SSJ_SIM_JACCARD, 1, 2)[0] == ssj.SSJ_E_INVALID


def test_exact_bound_matches_the_term_by_term_sum():
    """The exact Eq. 5 (through the odd-term identity) against the printed
    sum in rationals, and against the floating evaluation."""
    from fractions import Fraction
    from math import comb
    for b in (64, 100, 256):
        for n in (1, 2, 9, 40):
            s = sum(Fraction(comb(2 * n, k) * (b - 1) ** (2 * n - k), b ** (2 * n))
                    for k in range(1, 2 * n + 1, 2))
            want = n - Fraction(b, 2) * s
            assert oracle.expected_bound_exact(oracle.BM_XOR, b, n) == want
            assert abs(float(want) - oracle.expected_bound(oracle.BM_XOR, b, n)) < 1e-9 * n


def test_tie_at_an_integer_crossing():
    """Xor: E/n = 1 - b/(4n) + (b/4n)(1 - 2/b)^(2n) meets t exactly up to a
    tiny positive term when n = b / (4 (1 - t)) is an integer; that n is not
    within the threshold."""
    from fractions import Fraction
    t = oracle.normalized_threshold(oracle.JACCARD, 19, 20)   # 38/39
    assert t == Fraction(38, 39)
    n = 64 * 39 // 4                                            # 624
    assert oracle.expected_bound_exact(oracle.BM_XOR, 64, n) / n > t
    assert oracle.cutoff(oracle.BM_XOR, 64, t) == n - 1
