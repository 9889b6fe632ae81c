"""The bitmap build's handling of the token array (Section 3.2's bitmaps of
strictly increasing token sets).  The segmented build reads four tokens per
thread from the 16-byte boundary at or before a run of sets, finds the set
of the first by binary search and steps across set ends, and checks every
token against the one before it in its set.  So a strict-order violation
must be reported wherever it sits (any place in a four-token group, a set's
first or last pair, on either side of a 256-set segment, in any side of a
batch), and the bitmaps and pairs must equal the oracle's whatever the
alignment of the token array (unaligned arrays take scalar loads)."""
import numpy as np
import pytest
import torch

import gen
import oracle
import paper_1711_07295_amd as ssj

pytestmark = pytest.mark.gpu


def _col(seed, n=1500):
    """Ragged sets of 1..300 tokens with a few empty ones among them."""
    c = gen.generate(n_sets=n, universe=4000, zipf_s=1.0, size_dist=gen.SIZE_LOGNORMAL,
                     size_a=12.0, size_b=1.0, size_lo=1, size_hi=300, planted_frac=0.2,
                     seed=seed)
    sets = [c.set(k).tolist() for k in range(c.n_sets)]
    for k in (3, 255, 256, 700):
        sets.insert(k, [])
    return gen.from_lists(sets)


def _dev_shifted(c, shift):
    """c on the device with its token array starting `shift` tokens past a
    16-byte boundary."""
    tok = np.concatenate([np.zeros(shift, np.uint32), c.tokens]).view(np.int32)
    t = torch.from_numpy(tok.copy()).to("cuda")[shift:]
    off = torch.from_numpy(c.offsets.view(np.int64).copy()).to("cuda")
    assert t.data_ptr() % 16 == 4 * shift
    return ssj.DeviceSets(off, t)


@pytest.mark.parametrize("shift", [0, 1, 2, 3])
def test_bitmaps_and_pairs_at_any_alignment(shift):
    c = _col(61)
    d = _dev_shifted(c, shift)
    for b in (64, 512, 2048):
        got = ssj.ssj_build_bitmaps(d, b).cpu().numpy().view(np.uint64)
        want = oracle.bitmaps(c.offsets, c.tokens, b, oracle.BM_XOR)
        assert np.array_equal(got, want), b
    pairs, _ = ssj.ssj_self_join(d, 1, 2, b_bits=0)
    assert np.array_equal(pairs, oracle.self_join(c.offsets, c.tokens, 1, 2))


def _violations(c):
    """(set, place) pairs: the first, a middle and the last pair of sets
    around the 256-set segment boundaries and at the end, so that the
    broken pair falls at every place in a four-token group."""
    sizes = c.sizes()
    out = []
    for k in (0, 254, 255, 257, 258, 511, 512, c.n_sets - 2, c.n_sets - 1):
        n = int(sizes[k])
        if n >= 2:
            out += [(k, 0), (k, n - 2), (k, n // 2 - 1 if n >= 4 else 0)]
    return sorted(set(out))


def test_strict_order_violations_are_reported_wherever_they_sit():
    c = _col(62)
    places = _violations(c)
    seen = set()
    for k, i in places:
        a = int(c.offsets[k]) + i
        seen.add(a % 4)
        for kind in ("swap", "repeat"):
            bad = c.tokens.copy()
            if kind == "swap":
                bad[a], bad[a + 1] = bad[a + 1], bad[a]
            else:
                bad[a + 1] = bad[a]
            cb = gen.Collection(offsets=c.offsets, tokens=bad)
            for shift in (0, 3):
                d = _dev_shifted(cb, shift)
                with pytest.raises(ssj.SsjError) as e:
                    ssj.ssj_build_bitmaps(d, 64)
                assert e.value.status == ssj.SSJ_E_UNSORTED, (k, i, kind, shift)
                with pytest.raises(ssj.SsjError) as e:
                    ssj.ssj_self_join(d, 4, 5, b_bits=0)
                assert e.value.status == ssj.SSJ_E_UNSORTED, (k, i, kind, shift)
    assert seen == {0, 1, 2, 3}  # the broken pair started at every place in a group
    # the intact collection passes
    ssj.ssj_build_bitmaps(_dev_shifted(c, 0), 64)


def test_a_violation_in_one_side_of_a_batch_is_reported():
    cols = [_col(63 + k, n=600) for k in range(3)]
    for side in range(3):
        devs = []
        for k, c in enumerate(cols):
            if k == side:
                bad = c.tokens.copy()
                a = int(c.offsets[c.n_sets // 2]) + 1
                while a + 1 >= int(c.offsets[c.n_sets // 2 + 1]):
                    a -= 1
                bad[a], bad[a + 1] = bad[a + 1], bad[a]
                c = gen.Collection(offsets=c.offsets, tokens=bad)
            devs.append(ssj.to_device(c.offsets, c.tokens))
        with pytest.raises(ssj.SsjError) as e:
            ssj.ssj_self_join_batch(devs, [1, 4, 7], [2, 5, 10])
        assert e.value.status == ssj.SSJ_E_UNSORTED, side
    got, _ = ssj.ssj_self_join_batch([ssj.to_device(c.offsets, c.tokens) for c in cols],
                                     [1, 4, 7], [2, 5, 10])
    for c, g, (p, q) in zip(cols, got, [(1, 2), (4, 5), (7, 10)]):
        assert np.array_equal(g, oracle.self_join(c.offsets, c.tokens, p, q))
