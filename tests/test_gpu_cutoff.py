"""GPU parity of the cutoff point (Section 3.4): with SSJ_FLAG_CUTOFF the
rows past the cutoff of their widest width skip the bitmap filter and take
prefix-filtered candidates.  The pairs must not change.  Bit-exact against
the oracle."""
import numpy as np
import pytest

import gen
import oracle
import paper_1711_07295_amd as ssj

pytestmark = pytest.mark.gpu

CUT = ssj.SSJ_FLAG_CUTOFF


def _dev(c):
    return ssj.to_device(c.offsets, c.tokens)


def _wide(seed, n, universe=3000, median=80.0, hi=1500, planted=0.25):
    """Sizes well past the cutoff of narrow bitmaps (about 45-300 at b = 64)."""
    return gen.generate(n_sets=n, universe=universe, zipf_s=1.0, size_dist=gen.SIZE_LOGNORMAL,
                        size_a=median, size_b=0.9, size_lo=1, size_hi=hi, planted_frac=planted,
                        seed=seed)


@pytest.mark.parametrize("b", [0, 64, 256])
@pytest.mark.parametrize("pq", [(1, 2), (7, 10), (9, 10)])
def test_self_join_with_cutoff_matches_oracle(b, pq):
    p, q = pq
    c = _wide(1000 + b + p, 1200)
    d = _dev(c)
    want = oracle.self_join(c.offsets, c.tokens, p, q)
    plain, st0 = ssj.ssj_self_join(d, p, q, b_bits=b)
    got, st = ssj.ssj_self_join(d, p, q, b_bits=b, flags=CUT)
    assert np.array_equal(plain, want)
    assert np.array_equal(got, want), (b, p, q, len(got), len(want))
    # the band is the same; the bitmap filter does less work
    assert st["band_pairs"] == st0["band_pairs"] == oracle.band_pairs(c.sizes(), p, q)
    # the widest width the automatic mode chose: its cutoff point
    omega = ssj.ssj_cutoff(b or st0["class_bits"][st0["n_classes"] - 1], p, q)
    if c.sizes().max() > omega:
        assert st["filter_ops"] < st0["filter_ops"]


@pytest.mark.parametrize("sim,osim", [(ssj.SSJ_SIM_DICE, oracle.DICE),
                                      (ssj.SSJ_SIM_COSINE, oracle.COSINE),
                                      (ssj.SSJ_SIM_OVERLAP, oracle.OVERLAP)])
def test_other_functions_and_rs_join_with_cutoff(sim, osim):
    r, s = _wide(1100 + sim, 700), _wide(1200 + sim, 900)
    pq = [(3, 5), (4, 5)] if sim != ssj.SSJ_SIM_OVERLAP else [(20, 1), (60, 1)]
    for p, q in pq:
        want = oracle.rs_join(r.offsets, r.tokens, s.offsets, s.tokens, p, q, sim=osim)
        got, _ = ssj.ssj_rs_join(_dev(r), _dev(s), p, q, b_bits=64, sim=sim, flags=CUT)
        assert np.array_equal(got, want), (sim, p, q)
        want = oracle.self_join(s.offsets, s.tokens, p, q, sim=osim)
        got, _ = ssj.ssj_self_join(_dev(s), p, q, b_bits=0, sim=sim, flags=CUT)
        assert np.array_equal(got, want), (sim, p, q)


def test_cutoff_chunks_and_survivors():
    """A small queue splits the prefix candidates into many chunks; the
    prefix candidates (reported with SSJ_FLAG_SURVIVORS_ONLY) cover every
    result."""
    c = _wide(1300, 1500, universe=800, planted=0.4)
    d = _dev(c)
    want = oracle.self_join(c.offsets, c.tokens, 1, 2)
    for cap in (1, 20_000):
        got, st = ssj.ssj_self_join(d, 1, 2, b_bits=64, flags=CUT, queue_capacity=cap)
        assert np.array_equal(got, want), cap
    surv, _ = ssj.ssj_self_join(d, 1, 2, b_bits=64, flags=CUT | ssj.SSJ_FLAG_SURVIVORS_ONLY)
    sk = surv[:, 0].astype(np.int64) << 32 | surv[:, 1]
    wk = want[:, 0].astype(np.int64) << 32 | want[:, 1]
    assert np.isin(wk, sk).all()
    assert len(np.unique(sk)) == len(sk)


def test_batch_and_index_with_cutoff():
    cols = [_wide(1400 + k, n) for k, n in enumerate((300, 900, 40))]
    pq = [(1, 2), (7, 10), (4, 5)]
    got, _ = ssj.ssj_self_join_batch([_dev(c) for c in cols], [p for p, _ in pq],
                                     [q for _, q in pq], b_bits=0, flags=CUT)
    for c, (p, q), g in zip(cols, pq, got):
        assert np.array_equal(g, oracle.self_join(c.offsets, c.tokens, p, q))
    res = cols[1]
    with ssj.Index(_dev(res)) as idx:
        got, _ = idx.query([_dev(cols[0]), _dev(cols[2])], [1, 7], [2, 10], flags=CUT)
        for x, (p, q), g in zip((cols[0], cols[2]), [(1, 2), (7, 10)], got):
            want = oracle.rs_join(x.offsets, x.tokens, res.offsets, res.tokens, p, q)
            assert np.array_equal(g, want)


def test_every_row_past_the_cutoff():
    """b = 64 at 1/2 cuts off at 45 tokens; sets of 60-200 tokens all take
    the prefix path."""
    c = gen.generate(n_sets=800, universe=2000, zipf_s=0.9, size_dist=gen.SIZE_UNIFORM,
                     size_lo=60, size_hi=200, planted_frac=0.3, seed=1500)
    assert ssj.ssj_cutoff(64, 1, 2) < 60
    want = oracle.self_join(c.offsets, c.tokens, 1, 2)
    got, st = ssj.ssj_self_join(_dev(c), 1, 2, b_bits=64, flags=CUT)
    assert np.array_equal(got, want)
    assert st["filter_ops"] == 0 and st["band_pairs"] == oracle.band_pairs(c.sizes(), 1, 2)


@pytest.mark.parametrize("pq", [(1, 2), (7, 10), (4, 5)])
def test_wide_bitmaps_for_large_sets(pq):
    """Sets of 200-1500 tokens: pairs of sets above 256 tokens take a second
    test at 4096 bits in verification (automatic widths), with and without
    the cutoff.  The pairs must not change."""
    p, q = pq
    c = gen.generate(n_sets=1500, universe=4000, zipf_s=1.0, size_dist=gen.SIZE_UNIFORM,
                     size_lo=200, size_hi=1500, planted_frac=0.4, seed=1600 + p)
    r = gen.generate(n_sets=400, universe=4000, zipf_s=1.0, size_dist=gen.SIZE_UNIFORM,
                     size_lo=200, size_hi=1500, planted_frac=0.4, seed=1700 + p)
    want = oracle.self_join(c.offsets, c.tokens, p, q)
    assert len(want) > 50
    for fl in (0, CUT):
        got, _ = ssj.ssj_self_join(_dev(c), p, q, b_bits=0, flags=fl)
        assert np.array_equal(got, want), (p, q, fl)
    want = oracle.rs_join(r.offsets, r.tokens, c.offsets, c.tokens, p, q)
    for fl in (0, CUT):
        got, _ = ssj.ssj_rs_join(_dev(r), _dev(c), p, q, b_bits=0, flags=fl)
        assert np.array_equal(got, want), (p, q, fl)
    with ssj.Index(_dev(c)) as idx:
        got, _ = idx.query([_dev(r)], [p], [q])
        assert np.array_equal(got[0], want)
