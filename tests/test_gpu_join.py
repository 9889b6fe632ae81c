"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Integer work throughout, so every comparison is bit-exact: bitmaps word for
word, survivor sets and counts, and the sorted pair lists of the joins."""
import numpy as np
import pytest

import gen
import oracle
import paper_1711_07295_amd as ssj

pytestmark = pytest.mark.gpu


def _dev(c):
    return ssj.to_device(c.offsets, c.tokens)


def _bm_np(t):
    return t.cpu().numpy().view(np.uint64)


def _ragged(seed, n=1500, universe=300, hi=60, planted=0.15):
    return gen.generate(n_sets=n, universe=universe, zipf_s=1.0, size_dist=gen.SIZE_LOGNORMAL,
                        size_a=10.0, size_b=0.8, size_lo=1, size_hi=hi, planted_frac=planted,
                        seed=seed)


@pytest.mark.parametrize("method", [ssj.SSJ_BM_XOR, ssj.SSJ_BM_SET, ssj.SSJ_BM_NEXT])
@pytest.mark.parametrize("b", [64, 128, 192, 256, 4096])
def test_bitmaps_match_oracle(method, b):
    c = gen.generate(n_sets=3000, universe=20000, zipf_s=0.9, size_dist=gen.SIZE_LOGNORMAL,
                     size_a=40.0, size_b=1.0, size_lo=0, size_hi=5000, seed=b + method)
    got = _bm_np(ssj.ssj_build_bitmaps(_dev(c), b, method))
    want = oracle.bitmaps(c.offsets, c.tokens, b, method)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("pq", [(1, 5), (7, 18), (1, 2), (73, 127), (4, 5)])
@pytest.mark.parametrize("b", [64, 192, 4096])
def test_combined_bitmaps_match_oracle(pq, b):
    """Bitmap-Combined (Alg. 6): the generator picked by the threshold,
    bit-exact against the oracle's Combined, on both sides of the printed
    range edges (7/18 and 73/127 sit exactly on 0.56 and 0.73)."""
    p, q = pq
    c = gen.generate(n_sets=2000, universe=20000, zipf_s=0.9, size_dist=gen.SIZE_LOGNORMAL,
                     size_a=40.0, size_b=1.0, size_lo=0, size_hi=5000, seed=b + p)
    got = _bm_np(ssj.ssj_build_bitmaps(_dev(c), b, ssj.SSJ_BM_COMBINED, p, q))
    want = oracle.bitmaps(c.offsets, c.tokens, b, oracle.BM_COMBINED, p, q)
    assert np.array_equal(got, want)


def test_combined_bitmaps_join_unchanged_and_bad_threshold():
    c = _ragged(77)
    d = _dev(c)
    for p, q in ((1, 2), (4, 5)):
        bm = ssj.ssj_build_bitmaps(d, 128, ssj.SSJ_BM_COMBINED, p, q)
        got, _ = ssj.ssj_self_join(d, p, q, b_bits=128, bitmaps=bm)
        assert np.array_equal(got, oracle.self_join(c.offsets, c.tokens, p, q))
    for p, q in ((0, 1), (3, 2), (1, 0)):
        with pytest.raises(ssj.SsjError) as e:
            ssj.ssj_build_bitmaps(d, 64, ssj.SSJ_BM_COMBINED, p, q)
        assert e.value.status == ssj.SSJ_E_INVALID
    with pytest.raises(ssj.SsjError) as e:
        ssj.ssj_build_bitmaps(d, 64, 4)
    assert e.value.status == ssj.SSJ_E_UNSUPPORTED


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("pq", [(1, 2), (7, 10), (4, 5), (9, 10), (1, 1)])
def test_self_join_matches_oracle(seed, pq):
    p, q = pq
    c = _ragged(100 + seed)
    want = oracle.self_join(c.offsets, c.tokens, p, q)
    b = (64, 128, 192)[seed % 3]
    got, st = ssj.ssj_self_join(_dev(c), p, q, b_bits=b)
    assert np.array_equal(got, want), (len(got), len(want))
    assert st["results"] == len(want)
    assert st["band_pairs"] == oracle.band_pairs(c.sizes(), p, q)


def test_selfjoin_10k_workload():
    c = gen.workload("selfjoin-10k")
    for p, q in [(4, 5), (1, 2), (3, 10)]:
        want = oracle.self_join(c.offsets, c.tokens, p, q)
        got, st = ssj.ssj_self_join(_dev(c), p, q, b_bits=64)
        assert np.array_equal(got, want)
        assert st["band_pairs"] == oracle.band_pairs(c.sizes(), p, q)


@pytest.mark.parametrize("b", [64, 128, 192, 256, 512])
@pytest.mark.parametrize("pq", [(1, 2), (4, 5)])
def test_survivors_match_oracle(b, pq):
    p, q = pq
    c = _ragged(7, n=2500, universe=2000, hi=120)
    d = _dev(c)
    got, st = ssj.ssj_self_join(d, p, q, b_bits=b, flags=ssj.SSJ_FLAG_SURVIVORS_ONLY)
    bm = oracle.bitmaps(c.offsets, c.tokens, b, oracle.BM_XOR)
    cnt, band, surv = oracle.survivors(c.offsets, bm, b, p, q, listing=True)
    assert np.array_equal(got, surv)
    assert st["survivors"] == cnt and st["band_pairs"] == band


def test_queue_overflow_resume_gives_same_pairs():
    """A queue far smaller than the ~1e5 survivors forces many drain/resume
    rounds; capacities below the library's floor (4096) are raised to it."""
    c = _ragged(11, n=6000, universe=500, hi=60, planted=0.3)
    d = _dev(c)
    want = oracle.self_join(c.offsets, c.tokens, 1, 2)
    base, st0 = ssj.ssj_self_join(d, 1, 2, b_bits=64)
    assert np.array_equal(base, want) and st0["filter_launches"] == 1
    assert st0["survivors"] > 50_000
    for cap in (1, 5000, 30_000):
        got, st = ssj.ssj_self_join(d, 1, 2, b_bits=64, queue_capacity=cap)
        assert np.array_equal(got, want)
        assert st["filter_launches"] > 1
        assert st["survivors"] == st0["survivors"]


@pytest.mark.parametrize("pq", [(1, 2), (4, 5), (9, 10)])
def test_rs_join_matches_oracle_and_transpose(pq):
    p, q = pq
    r = _ragged(21, n=900, universe=250, hi=50)
    s = _ragged(22, n=1700, universe=250, hi=70)
    want = oracle.rs_join(r.offsets, r.tokens, s.offsets, s.tokens, p, q)
    got, st = ssj.ssj_rs_join(_dev(r), _dev(s), p, q, b_bits=128)
    assert np.array_equal(got, want)
    back, _ = ssj.ssj_rs_join(_dev(s), _dev(r), p, q, b_bits=64)
    assert np.array_equal(back[np.lexsort((back[:, 0], back[:, 1]))][:, ::-1], want)


def test_self_join_is_triangle_of_rs_join():
    c = _ragged(31, n=800)
    d = _dev(c)
    full, _ = ssj.ssj_rs_join(d, d, 3, 5, b_bits=64)
    tri = full[full[:, 0] < full[:, 1]]
    got, _ = ssj.ssj_self_join(d, 3, 5, b_bits=64)
    assert np.array_equal(got, tri)


def test_result_independent_of_width_tiling_and_generator():
    c = _ragged(41, n=2000, universe=400, hi=90)
    d = _dev(c)
    want = oracle.self_join(c.offsets, c.tokens, 3, 5)
    for b in (64, 128, 192, 320, 512, 1024, 4096):
        got, _ = ssj.ssj_self_join(d, 3, 5, b_bits=b)
        assert np.array_equal(got, want), b
    for tc in (1, 5, 64, 1000):
        got, _ = ssj.ssj_self_join(d, 3, 5, b_bits=64, tile_cols=tc)
        assert np.array_equal(got, want), tc
    for method in (ssj.SSJ_BM_SET, ssj.SSJ_BM_NEXT, ssj.SSJ_BM_XOR):
        bm = ssj.ssj_build_bitmaps(d, 128, method)
        got, _ = ssj.ssj_self_join(d, 3, 5, b_bits=128, bitmaps=bm)
        assert np.array_equal(got, want), method


def test_degenerate_inputs():
    cases = [
        [],                                   # no sets
        [[1, 2, 3]],                          # one set
        [[], [], []],                         # only empty sets
        [[5], [5], [6], []],                  # singletons, duplicates, empty
        [[1, 2, 3], [1, 2, 3], [1, 2, 3]],    # identical sets
        [list(range(0, 3000, 3)), list(range(0, 3000, 3)), list(range(1, 3001, 3))],
    ]
    for sets in cases:
        c = gen.from_lists(sets)
        for p, q in [(1, 2), (1, 1), (1, 1000)]:
            want = oracle.self_join(c.offsets, c.tokens, p, q)
            got, _ = ssj.ssj_self_join(_dev(c), p, q, b_bits=64)
            assert np.array_equal(got, want), (sets[:2], p, q)


def test_errors_are_reported_without_output():
    good = gen.from_lists([[1, 2], [2, 3]])
    d = _dev(good)
    with pytest.raises(ssj.SsjError) as e:
        ssj.ssj_self_join(d, 1, 2, b_bits=100)
    assert e.value.status == ssj.SSJ_E_INVALID
    for p, q in [(0, 1), (3, 2), (1, 0)]:
        with pytest.raises(ssj.SsjError) as e:
            ssj.ssj_self_join(d, p, q)
        assert e.value.status == ssj.SSJ_E_INVALID
    with pytest.raises(ssj.SsjError) as e:
        ssj.ssj_self_join(d, 1, 2, sim=7)
    assert e.value.status == ssj.SSJ_E_INVALID
    bad = gen.from_lists([[1, 2], [3, 3], [9, 4]])        # repeated and decreasing tokens
    with pytest.raises(ssj.SsjError) as e:
        ssj.ssj_self_join(_dev(bad), 1, 2)
    assert e.value.status == ssj.SSJ_E_UNSORTED
    with pytest.raises(ssj.SsjError) as e:
        ssj.ssj_build_bitmaps(_dev(bad), 64)
    assert e.value.status == ssj.SSJ_E_UNSORTED
    # offsets that do not end at n_tokens, and decreasing offsets
    import torch
    off = torch.tensor([0, 2, 5], dtype=torch.int64, device="cuda")
    tok = torch.tensor([1, 2, 3, 4], dtype=torch.int32, device="cuda")
    with pytest.raises(ssj.SsjError) as e:
        ssj.ssj_self_join(ssj.DeviceSets(off, tok), 1, 2)
    assert e.value.status == ssj.SSJ_E_INVALID
    off = torch.tensor([0, 3, 2, 4], dtype=torch.int64, device="cuda")
    with pytest.raises(ssj.SsjError) as e:
        ssj.ssj_self_join(ssj.DeviceSets(off, tok), 1, 2)
    assert e.value.status == ssj.SSJ_E_INVALID


def test_selfjoin_1m_sampled():
    """The 1,000,000-set workload at t = 4/5, b = 128 (the benchmark's
    configuration): every pair that involves one of 300 sampled sets must
    match the oracle, and every reported pair must pass the oracle's check."""
    c = gen.workload("selfjoin-1m")
    got, st = ssj.ssj_self_join(_dev(c), 4, 5, b_bits=128)
    assert st["band_pairs"] == oracle.band_pairs(c.sizes(), 4, 5)
    assert len(got) > 1000
    assert np.all(got[:, 0] < got[:, 1])
    assert np.all(np.diff(got[:, 0].astype(np.int64) * (1 << 32) + got[:, 1]) > 0)
    assert oracle.check_pairs(c.offsets, c.tokens, c.offsets, c.tokens, got, 4, 5).all()
    rng = np.random.default_rng(2024)
    rows = rng.choice(c.n_sets, size=300, replace=False)
    # include sets that are known to pair
    rows = np.unique(np.concatenate([rows, got[rng.choice(len(got), 50, replace=False), 0]]))
    want = oracle.self_join_rows(c.offsets, c.tokens, rows, 4, 5)
    mask = np.isin(got[:, 0], rows) | np.isin(got[:, 1], rows)
    assert np.array_equal(got[mask], want)


@pytest.mark.parametrize("pq", [(1, 2), (7, 10), (4, 5), (9, 10)])
def test_automatic_width_classes_match_oracle(pq):
    """b_bits = 0: row-size classes with their own widths, exact result."""
    p, q = pq
    c = gen.generate(n_sets=4000, universe=3000, zipf_s=1.0, size_dist=gen.SIZE_LOGNORMAL,
                     size_a=40.0, size_b=1.0, size_lo=1, size_hi=600, planted_frac=0.2,
                     seed=300 + p)
    want = oracle.self_join(c.offsets, c.tokens, p, q)
    got, st = ssj.ssj_self_join(_dev(c), p, q, b_bits=0)
    assert np.array_equal(got, want)
    # a workload this small may take one class: each class costs a launch
    assert st["b_bits"] == 0 and st["n_classes"] >= 1
    assert st["band_pairs"] == oracle.band_pairs(c.sizes(), p, q)
    bits = st["class_bits"][:st["n_classes"]]
    assert bits == sorted(bits) and set(bits) <= {64, 128, 256, 512, 1024, 2048}
    sizes = st["class_max_size"][:st["n_classes"]]
    assert sizes == sorted(sizes) and sizes[-1] == int(c.sizes().max())
    # the filter's algorithmic work lies between the narrowest and widest class
    assert st["band_pairs"] * (bits[0] // 16 + 1) <= st["filter_ops"]
    assert st["filter_ops"] <= st["band_pairs"] * (bits[-1] // 16 + 1)
    r, s = _ragged(51, n=700, universe=900, hi=300), _ragged(52, n=900, universe=900, hi=300)
    want = oracle.rs_join(r.offsets, r.tokens, s.offsets, s.tokens, p, q)
    got, _ = ssj.ssj_rs_join(_dev(r), _dev(s), p, q, b_bits=0)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("flags", [0, ssj.SSJ_FLAG_SURVIVORS_ONLY])
def test_width_classes_drain_together(flags):
    """Automatic widths with a small queue on the 1,000,000-set workload (its
    width classes: 64 bits for small sets, wider ones for larger): the queue
    fills in the launches of several classes, each resuming from its own
    tiles in later rounds.  Pairs and survivor sets equal those of one pass
    with the library's queue."""
    c = gen.workload("selfjoin-1m")
    d = _dev(c)
    one, s1 = ssj.ssj_self_join(d, 4, 5, b_bits=0, flags=flags)
    got, st = ssj.ssj_self_join(d, 4, 5, b_bits=0, flags=flags, queue_capacity=1 << 14)
    assert st["n_classes"] >= 2 and s1["n_classes"] == st["n_classes"]
    assert s1["filter_launches"] == s1["n_classes"]
    assert s1["survivors"] > 4 * (1 << 14) and st["filter_launches"] >= 3 * st["n_classes"]
    assert st["survivors"] == s1["survivors"] and st["results"] == s1["results"]
    assert np.array_equal(got, one)


def test_automatic_width_rejects_caller_bitmaps():
    c = _ragged(61, n=100)
    d = _dev(c)
    bm = ssj.ssj_build_bitmaps(d, 64)
    with pytest.raises(ssj.SsjError) as e:
        ssj.ssj_self_join(d, 1, 2, b_bits=0, bitmaps=bm)
    assert e.value.status == ssj.SSJ_E_INVALID


def test_selfjoin_1m_sampled_automatic_width():
    c = gen.workload("selfjoin-1m")
    got, st = ssj.ssj_self_join(_dev(c), 4, 5, b_bits=0)
    fixed, _ = ssj.ssj_self_join(_dev(c), 4, 5, b_bits=128)
    assert np.array_equal(got, fixed)
    assert st["n_classes"] >= 2
    rng = np.random.default_rng(77)
    rows = rng.choice(c.n_sets, size=200, replace=False)
    want = oracle.self_join_rows(c.offsets, c.tokens, rows, 4, 5)
    mask = np.isin(got[:, 0], rows) | np.isin(got[:, 1], rows)
    assert np.array_equal(got[mask], want)


def test_selfjoin_10m_row_sample():
    """The 10,000,000-set workload at t = 4/5 (automatic widths): every pair
    that involves one of 40 sampled sets matches the oracle, and a sample of
    the reported pairs passes the oracle's check."""
    c = gen.workload("selfjoin-10m")
    got, st = ssj.ssj_self_join(_dev(c), 4, 5, b_bits=0)
    assert st["band_pairs"] == oracle.band_pairs(c.sizes(), 4, 5)
    assert len(got) > 10_000 and np.all(got[:, 0] < got[:, 1])
    rng = np.random.default_rng(10)
    pick = got[rng.choice(len(got), size=min(len(got), 200_000), replace=False)]
    assert oracle.check_pairs(c.offsets, c.tokens, c.offsets, c.tokens, pick, 4, 5).all()
    rows = np.unique(np.concatenate([rng.choice(c.n_sets, size=30, replace=False),
                                     got[rng.choice(len(got), 10, replace=False), 1]]))
    want = oracle.self_join_rows(c.offsets, c.tokens, rows, 4, 5)
    mask = np.isin(got[:, 0], rows) | np.isin(got[:, 1], rows)
    assert np.array_equal(got[mask], want)


@pytest.mark.parametrize("pq", [(1, 2), (4, 5)])
def test_survivors_automatic_widths_match_oracle(pq):
    """b_bits = 0: every band pair is tested at the width of its row's class
    (the row is the later set in size order); the bitmaps of the narrower
    widths are folded from the widest one on the GPU.  The survivor set must
    equal a brute force over the band with the oracle's bitmaps."""
    p, q = pq
    c = gen.generate(n_sets=1500, universe=4000, zipf_s=1.0, size_dist=gen.SIZE_LOGNORMAL,
                     size_a=60.0, size_b=1.0, size_lo=1, size_hi=700, planted_frac=0.2,
                     seed=77 + p)
    got, st = ssj.ssj_self_join(_dev(c), p, q, b_bits=0, flags=ssj.SSJ_FLAG_SURVIVORS_ONLY)
    ncls = st["n_classes"]
    # the classes are the autotuner's (a workload this small may take one);
    # the brute force below follows whatever widths the call reports
    assert ncls >= 1
    bounds, widths = st["class_max_size"][:ncls], st["class_bits"][:ncls]
    sizes = c.sizes()
    order = np.lexsort((np.arange(c.n_sets), sizes))     # size order, ties by caller index
    pos = np.empty(c.n_sets, dtype=np.int64)
    pos[order] = np.arange(c.n_sets)
    bms = {b: oracle.bitmaps(c.offsets, c.tokens, b, oracle.BM_XOR) for b in set(widths)}
    wid = np.array(widths)
    want = []
    for i in range(c.n_sets):
        js = np.arange(i + 1, c.n_sets)
        a, s = int(sizes[i]), sizes[js]
        ok = np.array([a > 0 and int(x) > 0 and oracle.length_ok(oracle.JACCARD, a, int(x), p, q)
                       for x in s], dtype=bool)
        js = js[ok]
        if js.size == 0:
            continue
        rows = np.where(pos[i] > pos[js], i, js)
        bw = wid[np.searchsorted(np.array(bounds), sizes[rows])]
        for b in np.unique(bw):
            jb = js[bw == b]
            x = np.bitwise_xor(bms[int(b)][i][None, :], bms[int(b)][jb])
            h = np.unpackbits(x.view(np.uint8), axis=1).sum(axis=1)
            for j, hj in zip(jb, h):
                if oracle.bitmap_survives(a, int(sizes[j]), int(hj), p, q):
                    want.append((i, int(j)))
    want.sort()
    want = np.array(want, dtype=np.uint32).reshape(-1, 2)
    assert np.array_equal(got, want)
    assert st["survivors"] == len(want)


def test_memory_limit_fails_with_nomem_and_no_partial_output():
    """A cap on the library's working memory below what a call needs: the
    call fails with SSJ_E_NOMEM, leaves *out = {NULL, 0} (filled with junk
    before the call), and the library works again once the cap is lifted."""
    import ctypes
    c = _ragged(5)
    d = _dev(c)
    want = oracle.self_join(c.offsets, c.tokens, 1, 2)
    lib = ssj.load()
    cs = d.c()
    out = ssj.ssj_pairs()
    out.pairs = ctypes.cast(ctypes.c_void_p(0x1234), ctypes.POINTER(ssj.ssj_pair))
    out.count = 77
    try:
        ssj.ssj_memory_limit(1)
        st = lib.ssj_self_join(ctypes.byref(cs), None, 64, ssj.SSJ_SIM_JACCARD, 1, 2, None,
                               ctypes.byref(out), None, ssj._stream(None))
        assert st == ssj.SSJ_E_NOMEM
        assert not out.pairs and out.count == 0
        with pytest.raises(ssj.SsjError) as e:
            ssj.ssj_self_join(d, 1, 2, b_bits=0)
        assert e.value.status == ssj.SSJ_E_NOMEM
    finally:
        held = ssj.ssj_memory_limit(0)
    assert held == 0  # the cap freed every idle chunk
    got, _ = ssj.ssj_self_join(d, 1, 2, b_bits=64)
    assert np.array_equal(got, want)
    assert ssj.ssj_memory_limit(0) > 0  # chunks are cached again
