"""The C-ABI library loads and exports every function include/cgb.h declares
(no device calls: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared(header):
    src = open(os.path.join(ROOT, "include", header)).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cgb_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_1005_2594_amd import cgb
    lib = ctypes.CDLL(cgb.LIB_PATH)
    names = declared("cgb.h")
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_params_default_matches_paper_values():
    from paper_1005_2594_amd import cgb
    p = cgb.make_params({})
    assert p.tau == 1.0 and p.rho0 == 1.0 and p.sig_w == 0.5 and p.eps == 0.05


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    from paper_1005_2594_amd import cgb
    monkeypatch.setattr(cgb, "_lib", None)
    monkeypatch.setattr(cgb, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(ImportError):
        cgb.lib()
