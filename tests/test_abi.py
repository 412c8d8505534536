"""The C-ABI library loads and exports every function include/cgb.h declares
(no device calls: runs without a GPU)."""
import ctypes
import os
import re

import numpy as np
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


def test_estimators_match_the_oracle():
    # host-side estimator functions of the library against the oracle's
    from oracle import oracle as O
    from paper_1005_2594_amd import cgb
    rng = np.random.default_rng(3)
    A = 1e-6 * (1.0 + 0.1 * rng.random(50))
    assert cgb.mu_rel_kolmogorov(A, 1e-6, 1.0, 64, 7) == pytest.approx(O.mu_rel_kolmogorov(A, 1e-6, 1.0, 64, 7), rel=1e-13)
    u = 1e-4 * (1.0 + 0.1 * rng.random(50))
    for tau in (1.0, 0.8):
        assert cgb.mu_rel_slit(u, 1e-6, tau, 40, 9) == pytest.approx(O.mu_rel_slit(u, 1e-6, tau, 40, 9), rel=1e-13)
