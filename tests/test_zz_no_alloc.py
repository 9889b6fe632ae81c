"""ssj_build_bitmaps_noalloc, the bitmap build that allocates no memory,
against ssj_build_bitmaps (which takes its working memory from the library's
chunk cache): the same bitmaps word for word, through the C ABI, on calls in
a row whose later inputs are smaller than the earlier ones (the fixed
working array keeps the previous call's contents), for every generator.
Both are checked against the oracle's bitmaps (Alg. 3/4/5/6)."""
import numpy as np
import pytest

import gen
import oracle
import paper_1711_07295_amd as ssj

pytestmark = pytest.mark.gpu

METHODS = [(ssj.SSJ_BM_XOR, oracle.BM_XOR), (ssj.SSJ_BM_SET, oracle.BM_SET),
           (ssj.SSJ_BM_NEXT, oracle.BM_NEXT)]


def _coll(seed, n, universe=5000, hi=300):
    return gen.generate(n_sets=n, universe=universe, zipf_s=1.0, size_dist=gen.SIZE_LOGNORMAL,
                        size_a=20.0, size_b=0.9, size_lo=0, size_hi=hi, planted_frac=0.1,
                        seed=seed)


def _both(d, b, method, p=0, q=0):
    import torch
    want = ssj.ssj_build_bitmaps(d, b, method, p, q)
    got = torch.full_like(want, -1)  # stale contents must all be overwritten
    ssj.ssj_build_bitmaps_noalloc(d, b, got, method, p, q)
    torch.cuda.synchronize()
    return got.cpu().numpy().view(np.uint64), want.cpu().numpy().view(np.uint64)


@pytest.mark.parametrize("b", [64, 192, 4096])
def test_noalloc_equals_build_bitmaps_on_shrinking_inputs(b):
    big, small = _coll(51, 30_000), _coll(52, 700)
    for method, om in METHODS:
        for c in (big, small):  # the second call's input is smaller
            d = ssj.to_device(c.offsets, c.tokens)
            got, want = _both(d, b, method)
            assert np.array_equal(got, want), (b, method, c.n_sets)
            assert np.array_equal(got, oracle.bitmaps(c.offsets, c.tokens, b, om))


def test_noalloc_combined_picks_the_same_generator():
    c = _coll(53, 4000)
    d = ssj.to_device(c.offsets, c.tokens)
    for p, q in [(1, 2), (7, 10), (4, 5), (9, 10), (38, 62), (39, 61)]:
        got, want = _both(d, 128, ssj.SSJ_BM_COMBINED, p, q)
        assert np.array_equal(got, want), (p, q)
        ref = oracle.bitmaps(c.offsets, c.tokens, 128, oracle.BM_COMBINED, p=p, q=q)
        assert np.array_equal(got, ref), (p, q)


def test_noalloc_errors_leave_no_trace():
    """Unsorted input and bad offsets are reported; the next call on the same
    working array still builds the right bitmaps (counters are cleared at
    the start of every call)."""
    import torch
    bad = gen.from_lists([[1, 2, 3], [5, 4], [7]])
    d = ssj.to_device(bad.offsets, bad.tokens)
    out = torch.zeros((3, 1), dtype=torch.int64, device="cuda")
    with pytest.raises(ssj.SsjError) as e:
        ssj.ssj_build_bitmaps_noalloc(d, 64, out)
    assert e.value.status == ssj.SSJ_E_UNSORTED
    off = bad.offsets.copy()
    off[-1] += 1  # offsets[n] != n_tokens
    d2 = ssj.DeviceSets(torch.from_numpy(off.view(np.int64)).cuda(), d.tokens)
    with pytest.raises(ssj.SsjError) as e:
        ssj.ssj_build_bitmaps_noalloc(d2, 64, out)
    assert e.value.status == ssj.SSJ_E_INVALID
    good = _coll(54, 300)
    dg = ssj.to_device(good.offsets, good.tokens)
    got, want = _both(dg, 64, ssj.SSJ_BM_XOR)
    assert np.array_equal(got, want)


def test_noalloc_rejects_more_sets_than_its_array_holds():
    import torch
    n = ssj.SSJ_NOALLOC_MAX_SETS + 1
    offsets = torch.zeros(n + 1, dtype=torch.int64, device="cuda")  # n empty sets
    tokens = torch.zeros(0, dtype=torch.int32, device="cuda")
    d = ssj.DeviceSets(offsets, tokens)
    out = torch.zeros((n, 1), dtype=torch.int64, device="cuda")
    with pytest.raises(ssj.SsjError) as e:
        ssj.ssj_build_bitmaps_noalloc(d, 64, out)
    assert e.value.status == ssj.SSJ_E_UNSUPPORTED
    # at the limit it runs: every bitmap of an empty set is zero
    d = ssj.DeviceSets(offsets[:n], tokens)
    out = torch.full((n - 1, 1), -1, dtype=torch.int64, device="cuda")
    ssj.ssj_build_bitmaps_noalloc(d, 64, out)
    assert int(out.abs().sum()) == 0
