"""The matrix-core filter (b = 64, 128, 256) against the oracle and the
vector-ALU kernel (SSJ_FLAG_VALU).  The matrix cores score the Hamming
distance of Theorem 1 as a dot product of +-1 vectors, exact in fp32, so
both kernels must keep exactly the same pairs: the survivor sets
(SSJ_FLAG_SURVIVORS_ONLY) are compared whole, also through queue drains
that resume inside a step.  These inputs are small, so SSJ_FLAG_MFMA puts
every width class on the matrix cores (by default a b = 256 class this
small runs on the vector ALUs, whose launch costs less); one test also
checks that default."""
import numpy as np
import pytest

import gen
import oracle
import paper_1711_07295_amd as ssj

pytestmark = pytest.mark.gpu

SURV = ssj.SSJ_FLAG_SURVIVORS_ONLY
VALU = ssj.SSJ_FLAG_VALU
MF = ssj.SSJ_FLAG_MFMA


def _dev(c):
    return ssj.to_device(c.offsets, c.tokens)


def _coll(seed, n, universe, lo=1, hi=120, median=25.0, planted=0.2):
    return gen.generate(n_sets=n, universe=universe, zipf_s=1.0, size_dist=gen.SIZE_LOGNORMAL,
                        size_a=median, size_b=0.8, size_lo=lo, size_hi=hi, planted_frac=planted,
                        seed=seed)


@pytest.mark.parametrize("b", [64, 128, 256, 512])
@pytest.mark.parametrize("pq", [(1, 2), (7, 10), (9, 10)])
def test_self_join_survivors_equal_oracle_and_valu(b, pq):
    p, q = pq
    c = _coll(2000 + b + p, 3000, 1500)
    d = _dev(c)
    mf, st = ssj.ssj_self_join(d, p, q, b_bits=b, flags=SURV | MF)
    va, st2 = ssj.ssj_self_join(d, p, q, b_bits=b, flags=SURV | VALU)
    bm = oracle.bitmaps(c.offsets, c.tokens, b, oracle.BM_XOR)
    cnt, band, surv = oracle.survivors(c.offsets, bm, b, p, q, listing=True)
    assert np.array_equal(mf, surv), (b, p, q, len(mf), len(surv))
    assert np.array_equal(va, surv)
    assert st["survivors"] == st2["survivors"] == cnt and st["band_pairs"] == band
    # and the join itself
    want = oracle.self_join(c.offsets, c.tokens, p, q)
    got, _ = ssj.ssj_self_join(d, p, q, b_bits=b, flags=MF)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("b", [0, 64, 512])
def test_rs_join_both_kernels(b):
    r, s = _coll(2100, 900, 1200), _coll(2101, 2500, 1200)
    for p, q in [(1, 2), (4, 5)]:
        want = oracle.rs_join(r.offsets, r.tokens, s.offsets, s.tokens, p, q)
        for fl in (0, MF, VALU):
            got, _ = ssj.ssj_rs_join(_dev(r), _dev(s), p, q, b_bits=b, flags=fl)
            assert np.array_equal(got, want), (b, p, q, fl)
        mf, _ = ssj.ssj_rs_join(_dev(r), _dev(s), p, q, b_bits=b, flags=SURV | MF)
        va, _ = ssj.ssj_rs_join(_dev(r), _dev(s), p, q, b_bits=b, flags=SURV | VALU)
        assert np.array_equal(mf, va), (b, p, q)


@pytest.mark.parametrize("sim,osim", [(ssj.SSJ_SIM_DICE, oracle.DICE),
                                      (ssj.SSJ_SIM_COSINE, oracle.COSINE),
                                      (ssj.SSJ_SIM_OVERLAP, oracle.OVERLAP)])
def test_other_functions_both_kernels(sim, osim):
    """Dice, Cosine and Overlap: both kernels keep exactly the survivors of
    the oracle's filter (Table 2 length band, Alg. 7's decision against the
    function's Table 1 overlap threshold) at fixed widths, and agree with
    each other at automatic widths; the joins equal the oracle's."""
    c = _coll(2200 + sim, 2500, 1500)
    pq = [(3, 5), (4, 5)] if sim != ssj.SSJ_SIM_OVERLAP else [(5, 1), (12, 1)]
    for p, q in pq:
        want = oracle.self_join(c.offsets, c.tokens, p, q, sim=osim)
        for b in (0, 64, 128, 256):
            got, _ = ssj.ssj_self_join(_dev(c), p, q, b_bits=b, sim=sim, flags=MF)
            assert np.array_equal(got, want), (sim, p, q, b)
            mf, st = ssj.ssj_self_join(_dev(c), p, q, b_bits=b, sim=sim, flags=SURV | MF)
            va, _ = ssj.ssj_self_join(_dev(c), p, q, b_bits=b, sim=sim, flags=SURV | VALU)
            assert np.array_equal(mf, va), (sim, p, q, b)
            if b:
                bm = oracle.bitmaps(c.offsets, c.tokens, b, oracle.BM_XOR)
                cnt, band, surv = oracle.survivors(c.offsets, bm, b, p, q, listing=True,
                                                   sim=osim)
                assert np.array_equal(mf, surv), (sim, p, q, b, len(mf), len(surv))
                assert st["survivors"] == cnt and st["band_pairs"] == band


@pytest.mark.parametrize("b", [64, 256])
def test_drains_resume_inside_steps(b):
    """Near-duplicate clusters at a low threshold keep hundreds of pairs per
    step of 32 columns; the smallest queue (4096 entries) fills many times,
    often in the middle of a step, and every survivor must still come out
    exactly once."""
    c = _coll(2300 + b, 5000, 400, hi=60, planted=0.5)
    d = _dev(c)
    full, st0 = ssj.ssj_self_join(d, 1, 3, b_bits=b, flags=SURV | MF)
    assert st0["filter_launches"] == 1 and len(full) > 50_000
    small, st = ssj.ssj_self_join(d, 1, 3, b_bits=b, flags=SURV | MF, queue_capacity=1)
    assert st["filter_launches"] > 10
    assert np.array_equal(small, full)
    va, _ = ssj.ssj_self_join(d, 1, 3, b_bits=b, flags=SURV | VALU, queue_capacity=1)
    assert np.array_equal(va, full)
    want = oracle.self_join(c.offsets, c.tokens, 1, 3)
    got, _ = ssj.ssj_self_join(d, 1, 3, b_bits=b, flags=MF, queue_capacity=1)
    assert np.array_equal(got, want)


def test_batch_and_index_both_kernels():
    cols = [_coll(2400 + k, n, 800) for k, n in enumerate((50, 700, 2000, 1))]
    pq = [(1, 2), (7, 10), (4, 5), (1, 2)]
    a, _ = ssj.ssj_self_join_batch([_dev(c) for c in cols], [p for p, _ in pq],
                                   [q for _, q in pq], b_bits=0, flags=MF)
    b, _ = ssj.ssj_self_join_batch([_dev(c) for c in cols], [p for p, _ in pq],
                                   [q for _, q in pq], b_bits=0, flags=VALU)
    for c, (p, q), x, y in zip(cols, pq, a, b):
        want = oracle.self_join(c.offsets, c.tokens, p, q)
        assert np.array_equal(x, want) and np.array_equal(y, want)
    res = _coll(2500, 20_000, 3000)
    qs = [_coll(2501, 300, 3000), _coll(2502, 40, 3000)]
    with ssj.Index(_dev(res)) as idx:
        for fl in (0, MF, VALU):
            got, _ = idx.query([_dev(x) for x in qs], [7, 1], [10, 2], flags=fl)
            for x, (p, q), g in zip(qs, [(7, 10), (1, 2)], got):
                want = oracle.rs_join(x.offsets, x.tokens, res.offsets, res.tokens, p, q)
                assert np.array_equal(g, want), fl


def test_small_classes_take_the_vector_alus_and_flags_conflict():
    """By default a b = 256 class below 2^26 band pairs runs on the vector
    ALUs: the survivor set is the same either way, and SSJ_FLAG_MFMA with
    SSJ_FLAG_VALU is rejected."""
    c = _coll(2600, 3000, 1500)
    d = _dev(c)
    dflt, st = ssj.ssj_self_join(d, 1, 2, b_bits=256, flags=SURV)
    mf, st_mf = ssj.ssj_self_join(d, 1, 2, b_bits=256, flags=SURV | MF)
    assert st["band_pairs"] < 1 << 26
    assert np.array_equal(dflt, mf) and st["survivors"] == st_mf["survivors"]
    with pytest.raises(ssj.SsjError) as e:
        ssj.ssj_self_join(d, 1, 2, flags=MF | VALU)
    assert e.value.status == ssj.SSJ_E_INVALID
