"""GPU parity at full size, element by element, against pair lists that the
oracle alone wrote (tests/golden/make_full_golden.py; the manifest
full_golden.json holds the input checksums and the SHA-256 of every list).

  selfjoin-1m   every similar pair (Eq. 1, Table 1 predicate) at Jaccard
                1/2, 7/10, 4/5 and 9/10, at automatic widths and at fixed
                b = 64, 128 and 256: the pair set is the same at every
                width, only the work differs
  selfjoin-10m  every similar pair whose larger size-order position is a
                sampled row (every 100th position from 50: a 1% row
                sample), at 4/5 and 19/20, automatic widths and b = 128; and
                every pair the library reports passes the oracle's
                predicate

  served-5m     the smallest query batches of the served form that hold a
                perturbed copy, against the 5,000,000-set index, against
                the oracle's R-S join over each batch's length band

A fixed b = 64 at t = 1/2 is left out: about a tenth of the 2.4e11 band
pairs survive a 64-bit bitmap at that threshold, and the test would spend
minutes draining the survivor queue; the automatic widths cover that
threshold."""
import importlib.util
import json
import os

import numpy as np
import pytest

import gen
import oracle
import paper_1711_07295_amd as ssj

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden")


def _golden_module():
    spec = importlib.util.spec_from_file_location(
        "make_full_golden", os.path.join(GOLDEN, "make_full_golden.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


MG = _golden_module()
MANIFEST = MG.load_manifest()


def _entry(name):
    e = MANIFEST.get(name)
    if e is None or not os.path.exists(os.path.join(GOLDEN, e["file"])):
        pytest.skip(f"no expected pair lists for {name}")
    return e


def _lists(name):
    e = _entry(name)
    base, higher = MG.load(os.path.join(GOLDEN, e["file"]))
    lo = tuple(int(x) for x in e["base_threshold"].split("/"))
    out = {lo: base, **higher}
    # the stored lists are the ones the manifest describes
    for (p, q), v in out.items():
        t = e["thresholds"][f"{p}/{q}"]
        assert v.shape[0] == t["pairs"] and MG.pairs_sha256(v) == t["sha256"]
    return e, out


@pytest.fixture(scope="module")
def c1m():
    e, lists = _lists("selfjoin-1m")
    col = gen.workload("selfjoin-1m")
    assert f"{col.checksum():#x}" == e["checksum"]
    return col, ssj.to_device(col.offsets, col.tokens), lists


@pytest.mark.parametrize("pq", [(1, 2), (7, 10), (4, 5), (9, 10)])
@pytest.mark.parametrize("b", [0, 64, 128, 256])
def test_selfjoin_1m_whole_pair_list(c1m, b, pq):
    if b == 64 and pq == (1, 2):
        pytest.skip("fixed b = 64 at t = 1/2: see the module docstring")
    col, dev, lists = c1m
    p, q = pq
    got, st = ssj.ssj_self_join(dev, p, q, b_bits=b)
    want = lists[pq]
    assert got.shape == want.shape, (b, pq, got.shape, want.shape)
    assert np.array_equal(got, want), (b, pq)
    assert st["results"] == len(want)
    assert st["band_pairs"] == oracle.band_pairs(col.sizes(), p, q)


@pytest.fixture(scope="module")
def c10m():
    e, lists = _lists("selfjoin-10m")
    col = gen.workload("selfjoin-10m")
    assert f"{col.checksum():#x}" == e["checksum"]
    order = oracle.size_order(col.offsets)
    rank = np.empty(col.n_sets, dtype=np.int64)
    rank[order] = np.arange(col.n_sets, dtype=np.int64)
    return col, ssj.to_device(col.offsets, col.tokens), lists, rank, e


@pytest.mark.parametrize("pq", [(4, 5), (19, 20)])
@pytest.mark.parametrize("b", [0, 128])
def test_selfjoin_10m_row_sample(c10m, b, pq):
    col, dev, lists, rank, e = c10m
    p, q = pq
    got, st = ssj.ssj_self_join(dev, p, q, b_bits=b)
    # precision: every reported pair is similar
    assert oracle.check_pairs(col.offsets, col.tokens, col.offsets, col.tokens, got, p, q).all()
    # recall on the sampled rows: the pairs whose larger size-order position
    # is a sampled row are exactly the oracle's
    step, first = e["rows"]["step"], e["rows"]["first"]
    top = np.maximum(rank[got[:, 0]], rank[got[:, 1]]) if len(got) else np.zeros(0, np.int64)
    mine = got[(top % step) == first]
    want = lists[pq]
    assert np.array_equal(mine, want), (b, pq, len(mine), len(want))
    assert st["results"] == len(got)


@pytest.fixture(scope="module")
def served5m():
    sw = gen.served_workload(60)  # the served form's 5,000,000-set index
    res = sw.resident
    idx = ssj.Index(ssj.to_device(res.offsets, res.tokens))
    yield sw, idx
    idx.close()


def _band_subset(res, r_sizes, p, q):
    """The resident sets a batch of sizes r_sizes can pair with (Table 2's
    length filter, the oracle's predicate): their indices and a CSR copy."""
    sizes = np.diff(res.offsets).astype(np.int64)
    ok = np.zeros(int(sizes.max()) + 1, dtype=bool)
    for c in np.unique(sizes):
        ok[c] = any(oracle.length_ok(oracle.JACCARD, int(a), int(c), p, q)
                    for a in np.unique(r_sizes))
    keep = np.nonzero(ok[sizes])[0]
    n = sizes[keep]
    off = np.zeros(keep.shape[0] + 1, dtype=np.uint64)
    np.cumsum(n, out=off[1:])
    starts = res.offsets[:-1][keep].astype(np.int64)
    gather = np.repeat(starts - off[:-1].astype(np.int64), n) + np.arange(int(off[-1]))
    return keep, off, res.tokens[gather]


def test_served_batches_against_the_5m_index_match_the_oracle(served5m):
    """The four smallest query batches of the served workload that hold a
    perturbed copy of a resident set, against the real 5,000,000-set index
    in one call: pairs element by element equal to
    the oracle's R-S join (Eq. 1) over the resident sets inside each batch's
    length band (sets outside it cannot reach the threshold, Table 2)."""
    sw, idx = served5m
    by_size = np.argsort([b.n_sets for b in sw.batches], kind="stable")
    order = [k for k in by_size if sw.copies[k].any()][:4]  # each holds a perturbed copy
    batches = [sw.batches[k] for k in order]
    ps, qs = [sw.thresholds[k][0] for k in order], [sw.thresholds[k][1] for k in order]
    got, st = idx.query([ssj.to_device(b.offsets, b.tokens) for b in batches], ps, qs)
    found = 0
    for b, p, q, g in zip(batches, ps, qs, got):
        keep, off, tok = _band_subset(sw.resident, b.sizes(), p, q)
        w = oracle.rs_join(b.offsets, b.tokens, off, tok, p, q)
        want = np.stack([w[:, 0], keep[w[:, 1]].astype(np.uint32)], axis=1) if len(w) else w
        assert np.array_equal(g, want), (b.n_sets, p, q, len(g), len(want))
        found += len(want)
    assert found > 0  # the perturbed copies find their sources
    assert st["results"] == found
