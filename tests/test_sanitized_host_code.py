"""The oracle and the input generator (plain C) built with AddressSanitizer
and UndefinedBehaviorSanitizer, and driven through their Python wrappers in
a child process: every call must finish without a sanitizer report, and
give the same results as the regular build."""
import os
import subprocess
import sys
import textwrap

import pytest

from gen import build as gen_build
from oracle import build as oracle_build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# The same calls in the child (sanitized libraries) and here (regular ones):
# every generator, every join form and similarity function, the bitmap
# generators at several widths, the survivor filter and the pair check.
EXERCISE = textwrap.dedent("""
    import hashlib
    import numpy as np
    import gen, oracle

    def exercise():
        h = hashlib.sha256()
        def add(a):
            h.update(np.ascontiguousarray(a).tobytes())
        c = gen.generate(n_sets=700, universe=400, zipf_s=1.0, size_dist=gen.SIZE_LOGNORMAL,
                         size_a=9.0, size_b=0.8, size_lo=0, size_hi=70, planted_frac=0.2, seed=5)
        add(c.offsets); add(c.tokens)
        u = gen.generate(n_sets=300, universe=200, zipf_s=0.8, size_dist=gen.SIZE_UNIFORM,
                         size_a=1, size_b=30, seed=6)
        add(u.offsets); add(u.tokens)
        for inst, (p, q) in gen.batched_instances(3, n_min=100, n_max=400):
            add(inst.tokens); add(np.array([p, q]))
        sw = gen.served_workload(3, resident_sets=500, max_batch=40)
        add(sw.resident.tokens)
        for sim in (oracle.JACCARD, oracle.DICE, oracle.COSINE, oracle.OVERLAP):
            p, q = (3, 1) if sim == oracle.OVERLAP else (7, 10)
            pr = oracle.self_join(c.offsets, c.tokens, p, q, sim=sim, threads=3)
            add(pr)
            bp, ev = oracle.self_join_banded(c.offsets, c.tokens, p, q, sim=sim, threads=3)
            add(bp); add(np.array([ev]))
            add(oracle.rs_join(u.offsets, u.tokens, c.offsets, c.tokens, p, q, sim=sim, threads=2))
            add(oracle.check_pairs(c.offsets, c.tokens, c.offsets, c.tokens, pr, p, q, sim=sim))
        for b in (64, 192, 4096):
            for m in (oracle.BM_XOR, oracle.BM_SET, oracle.BM_NEXT):
                bm = oracle.bitmaps(c.offsets, c.tokens, b, m)
                add(bm)
            add(oracle.bitmaps(c.offsets, c.tokens, b, oracle.BM_COMBINED, 4, 5))
            bm = oracle.bitmaps(c.offsets, c.tokens, b, oracle.BM_XOR)
            for sim in (oracle.JACCARD, oracle.DICE, oracle.COSINE, oracle.OVERLAP):
                p, q = (2, 1) if sim == oracle.OVERLAP else (1, 2)
                cnt, band, _ = oracle.survivors(c.offsets, bm, b, p, q, sim=sim)
                add(np.array([cnt, band], dtype=np.int64))
        add(np.array([oracle.cutoff(oracle.BM_XOR, 64, 0.72)]))
        return h.hexdigest()
""")


def _child_script(lo, lg):
    return EXERCISE + textwrap.dedent(f"""
        oracle._LIB_PATH = {lo!r}
        gen._LIB_PATH = {lg!r}
        print("DIGEST", exercise(), flush=True)
    """)


def test_oracle_and_generator_under_asan_and_ubsan(tmp_path):
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                          text=True).stdout.strip()
    if not asan or not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("libasan is not installed")
    lo = oracle_build.build(out=str(tmp_path / "liboracle_san.so"), sanitize=True)
    lg = gen_build.build(out=str(tmp_path / "libssjgen_san.so"), sanitize=True)
    env = dict(os.environ, LD_PRELOAD=asan, PYTHONPATH=ROOT,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-c", _child_script(lo, lg)], capture_output=True,
                       text=True, env=env, cwd=ROOT, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, \
        r.stderr[-4000:]
    got = [ln.split()[1] for ln in r.stdout.splitlines() if ln.startswith("DIGEST")]
    ns = {}
    exec(EXERCISE, ns)
    assert got == [ns["exercise"]()]
