"""Host arithmetic of bench.py (no GPU): the roofline entry of the dominant
filter launch for the matrix-core and the vector-ALU kernel."""
import math

import bench


def _stats(bits, ops, ms, launches=1):
    n = len(bits)
    return {"n_classes": n, "class_bits": list(bits) + [0] * (4 - n),
            "class_ops": list(ops) + [0] * (4 - n), "class_ms": list(ms) + [0.0] * (4 - n),
            "filter_launches": launches * n, "filter_ops": sum(ops), "ms_filter": sum(ms)}


def test_mfma_roofline_counts_2b_flops_per_band_pair():
    band64 = 1_000_000_000
    st = _stats([64, 128], [band64 * 5, 10 * 9], [2.0, 0.1])
    r = bench.roofline_of([st, st], 2)
    assert r["bound"] == "mfma" and r["unit"] == "TFLOP/s"
    want = band64 * 128 / 2.0e-3
    assert math.isclose(r["achieved"] * 1e12, want, rel_tol=1e-12)
    assert math.isclose(r["frac"], want / bench.PEAK_FP4, rel_tol=1e-12)
    assert math.isclose(r["band_pairs_per_launch"], band64)


def test_valu_roofline_and_odd_widths():
    st = _stats([192], [1000 * 13], [1.0])           # b = 192 runs on the vector ALU
    r = bench.roofline_of([st], 1)
    assert r["bound"] == "alu" and math.isclose(r["achieved"] * 1e12, 13000 / 1e-3)
    st = _stats([64], [1000 * 5], [1.0], launches=2)   # --valu at b = 64, two launches
    r = bench.roofline_of([st], 1, valu=True)
    assert r["bound"] == "alu" and math.isclose(r["ops_per_launch"], 2500)
    assert math.isclose(r["frac"], 5000 / 1e-3 / bench.PEAK_INT_OPS)


def test_zero_event_timings_give_no_roofline_entry():
    st = _stats([64], [5000], [0.0])
    assert bench.roofline_of([st], 1) is None


def test_golden_parity_compares_the_pair_list_hash():
    import json
    import os

    import numpy as np
    path = os.path.join(bench.ROOT, "tests", "golden", "full_golden.json")
    if not os.path.exists(path):
        import pytest
        pytest.skip("no full-size golden pair lists")
    with open(path) as fh:
        entry = json.load(fh)["selfjoin-1m"]
    ck = int(entry["checksum"], 16)
    pairs = np.zeros((3, 2), dtype=np.uint32)
    r = bench.golden_parity("selfjoin-1m", ck, "jaccard", 4, 5, pairs)
    assert r["sha256_equal"] is False and r["expected_pairs"] == entry["thresholds"]["4/5"]["pairs"]
    assert bench.golden_parity("selfjoin-1m", ck + 1, "jaccard", 4, 5, pairs) is None
    assert bench.golden_parity("selfjoin-1m", ck, "dice", 4, 5, pairs) is None
    assert bench.golden_parity("selfjoin-1m", ck, "jaccard", 3, 5, pairs) is None
