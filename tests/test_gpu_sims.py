"""GPU parity of the Dice, Cosine and Overlap joins (Table 1 functions with
their Table 2 length filters) against the CPU oracle, bit-exact."""
import numpy as np
import pytest

import gen
import oracle
import paper_1711_07295_amd as ssj

pytestmark = pytest.mark.gpu

SIMS = [(ssj.SSJ_SIM_DICE, oracle.DICE), (ssj.SSJ_SIM_COSINE, oracle.COSINE),
        (ssj.SSJ_SIM_OVERLAP, oracle.OVERLAP), (ssj.SSJ_SIM_JACCARD, oracle.JACCARD)]


def _dev(c):
    return ssj.to_device(c.offsets, c.tokens)


def _col(seed, n, universe=300, hi=80, median=12.0, planted=0.2):
    return gen.generate(n_sets=n, universe=universe, zipf_s=1.0, size_dist=gen.SIZE_LOGNORMAL,
                        size_a=median, size_b=0.9, size_lo=1, size_hi=hi,
                        planted_frac=planted, seed=seed)


def _thresholds(sim):
    if sim == ssj.SSJ_SIM_OVERLAP:
        return [(1, 1), (3, 1), (5, 2), (12, 1)]
    return [(1, 2), (7, 10), (4, 5), (9, 10), (1, 1)]


@pytest.mark.parametrize("sim,osim", SIMS)
@pytest.mark.parametrize("b", [0, 64, 192])
def test_self_join_matches_oracle(sim, osim, b):
    c = _col(900 + sim, 1500)
    d = _dev(c)
    for p, q in _thresholds(sim):
        want = oracle.self_join(c.offsets, c.tokens, p, q, sim=osim)
        got, st = ssj.ssj_self_join(d, p, q, b_bits=b, sim=sim)
        assert np.array_equal(got, want), (sim, p, q, b, len(got), len(want))
        assert st["band_pairs"] == oracle.band_pairs(c.sizes(), p, q, sim=osim)


@pytest.mark.parametrize("sim,osim", SIMS)
def test_rs_join_and_survivors(sim, osim):
    r, s = _col(910 + sim, 700, hi=200, median=30.0), _col(920 + sim, 1100, hi=200, median=30.0)
    for p, q in _thresholds(sim)[:3]:
        want = oracle.rs_join(r.offsets, r.tokens, s.offsets, s.tokens, p, q, sim=osim)
        got, _ = ssj.ssj_rs_join(_dev(r), _dev(s), p, q, b_bits=0, sim=sim)
        assert np.array_equal(got, want), (sim, p, q)
    # survivors are a superset of the result: no false negatives (Theorem 1)
    p, q = _thresholds(sim)[1]
    c = _col(930 + sim, 1200)
    d = _dev(c)
    surv, _ = ssj.ssj_self_join(d, p, q, b_bits=64, sim=sim, flags=ssj.SSJ_FLAG_SURVIVORS_ONLY)
    res, _ = ssj.ssj_self_join(d, p, q, b_bits=64, sim=sim)
    sk = surv[:, 0].astype(np.int64) << 32 | surv[:, 1]
    rk = res[:, 0].astype(np.int64) << 32 | res[:, 1]
    assert np.isin(rk, sk).all()


def test_cosine_thresholds_exactly_on_the_boundary():
    """Sets built so that cosine equals p/q exactly: included at p/q,
    excluded just above."""
    # |r| = 9, |s| = 4, o = 3: cos = 3 / 6 = 1/2; |r| = 16, |s| = 4, o = 4: cos = 4/8
    base = list(range(100, 109))
    sets = [base, base[:3] + [500], list(range(200, 216)), list(range(200, 204))]
    c = gen.from_lists([sorted(x) for x in sets])
    d = _dev(c)
    got, _ = ssj.ssj_self_join(d, 1, 2, b_bits=64, sim=ssj.SSJ_SIM_COSINE)
    assert got.tolist() == [[0, 1], [2, 3]]
    got, _ = ssj.ssj_self_join(d, 501, 1000, b_bits=64, sim=ssj.SSJ_SIM_COSINE)
    assert len(got) == 0
    want = oracle.self_join(c.offsets, c.tokens, 1, 2, sim=oracle.COSINE)
    assert want.tolist() == [[0, 1], [2, 3]]


def test_batch_and_index_with_other_functions():
    cols = [_col(940 + k, n) for k, n in enumerate((400, 1300, 60))]
    for sim, osim in SIMS[:3]:
        pq = _thresholds(sim)[:3]
        got, _ = ssj.ssj_self_join_batch([_dev(c) for c in cols], [p for p, _ in pq],
                                         [q for _, q in pq], sim=sim)
        for c, (p, q), g in zip(cols, pq, got):
            assert np.array_equal(g, oracle.self_join(c.offsets, c.tokens, p, q, sim=osim))
        res = cols[1]
        with ssj.Index(_dev(res)) as idx:
            got, _ = idx.query([_dev(cols[0]), _dev(cols[2])], [pq[0][0], pq[1][0]],
                               [pq[0][1], pq[1][1]], sim=sim)
            for x, (p, q), g in zip((cols[0], cols[2]), pq[:2], got):
                want = oracle.rs_join(x.offsets, x.tokens, res.offsets, res.tokens, p, q,
                                      sim=osim)
                assert np.array_equal(g, want)


def test_overlap_threshold_validation():
    d = _dev(gen.from_lists([[1, 2, 3], [1, 2, 3, 4]]))
    got, _ = ssj.ssj_self_join(d, 3, 1, sim=ssj.SSJ_SIM_OVERLAP)
    assert got.tolist() == [[0, 1]]
    got, _ = ssj.ssj_self_join(d, 4, 1, sim=ssj.SSJ_SIM_OVERLAP)
    assert len(got) == 0
    for sim in (ssj.SSJ_SIM_JACCARD, ssj.SSJ_SIM_DICE, ssj.SSJ_SIM_COSINE):
        with pytest.raises(ssj.SsjError) as e:
            ssj.ssj_self_join(d, 3, 1, sim=sim)
        assert e.value.status == ssj.SSJ_E_INVALID
