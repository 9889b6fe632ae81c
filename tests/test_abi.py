"""The C-ABI library loads and exports every entry point its header declares.
No compute call is made here (no GPU needed)."""
import os
import re
import subprocess

import pytest

import paper_1711_07295_amd as ssj

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ssj.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ssj_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("ssj_build_bitmaps", "ssj_self_join", "ssj_rs_join", "ssj_free_pairs"):
        assert n in names
    assert set(names) == set(ssj.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = ssj.load()
    for name in _declared():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", ssj.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(line.split()[-1] for line in out.splitlines() if line.strip())
    for name in _declared():
        assert name in exported, name


def test_abi_version_and_status_strings():
    assert ssj.ssj_abi_version() == ssj.ABI_VERSION == 4
    assert ssj.status_string(0) == "ok"
    assert "strictly increasing" in ssj.status_string(ssj.SSJ_E_UNSORTED)
    assert ssj.status_string(12345) == "unknown status"


def test_free_pairs_is_null_safe():
    ssj.load().ssj_free_pairs(None)
    p = ssj.ssj_pairs()
    ssj.ssj_free_pairs(p)
    ssj.ssj_free_pairs(p)
    assert p.count == 0


def test_struct_layouts_match_header():
    import ctypes
    assert ctypes.sizeof(ssj.ssj_sets) == 32
    assert ctypes.sizeof(ssj.ssj_pair) == 8
    assert ctypes.sizeof(ssj.ssj_pairs) == 16
    assert ctypes.sizeof(ssj.ssj_options) == 16
    assert ctypes.sizeof(ssj.ssj_stats) == 8 * 5 + 4 * 3 + 4 * 16 + 4 + 8 * 8 + 8 * 8 + 4 * 8 + 4 * 5 + 4


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(ssj, "_lib", None)
    monkeypatch.setattr(ssj, "LIB_PATH", str(tmp_path / "absent.so"))
    with pytest.raises(RuntimeError, match="missing"):
        ssj.load()
