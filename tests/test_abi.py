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


def test_query_sizes_without_a_device():
    # cgb_query_sizes is host arithmetic: the arena grows with the cell
    # capacity and the track record, staging holds 19 FP64 per site
    import synth
    from paper_1005_2594_amd import cgb
    p = synth.params(32, 24, 40)
    s0 = cgb.query_sizes(p, None, 0, 0, precision="pmx16s")
    s1 = cgb.query_sizes(p, None, 1000, 0, precision="pmx16s")
    s2 = cgb.query_sizes(p, None, 2000, 0, precision="pmx16s")
    s3 = cgb.query_sizes(p, None, 2000, 500, precision="pmx16s")
    assert s0.staging_bytes == 19 * 32 * 24 * 40 * 8
    assert s0.arena_bytes > 19 * 2 * 2 * 32 * 24 * 40
    assert s0.arena_bytes < s1.arena_bytes < s2.arena_bytes
    # at least the per-cell state: X, q, V, L, forces, kinematics, list of covered nodes
    assert s2.arena_bytes - s1.arena_bytes >= 1000 * (8 * (3 + 4 + 3 + 3 + 6 + 6 + 12) + 4 * 154)
    # 16 bytes per recorded step, in 256-byte pieces (one piece without a record)
    assert s3.arena_bytes - s2.arena_bytes == (500 * 16 + 255) // 256 * 256 - 256
    # FP64 storage needs more than FP16
    assert cgb.query_sizes(p, None, 0, 0, precision="p64").arena_bytes > s0.arena_bytes
    with pytest.raises(cgb.CgbError):
        cgb.query_sizes(dict(p, tau=0.4), None, 0, 0)


def test_viscometer_estimator_matches_the_oracle():
    from oracle import oracle as O
    from paper_1005_2594_amd import cgb
    rng = np.random.default_rng(5)
    flux = 1e-3 * (1 + 0.05 * rng.random(40))
    prof = 0.01 * np.arange(32) / 32 + 1e-5 * rng.standard_normal(32)
    for tau in (1.0, 0.8):
        assert cgb.mu_app_le(flux, 10, prof, 8, 9, 1.0, tau) == pytest.approx(
            O.mu_app_le(flux, 10, prof, 8, 9, 1.0, tau), rel=1e-12)


def test_indexed_layout_needs_less_memory():
    # sparse geometry: the indexed layout stores populations and link data
    # for the non-wall nodes only
    import synth
    from paper_1005_2594_amd import cgb
    m = synth.bifurcation_mask(5, 4, 5, 64)
    p = synth.vessel_params(m, force_mode=1, g=(0.0, 0.0, 1e-4))
    ns, nc = m.size, int((1 - m).sum())
    dense = cgb.query_sizes(p, wall_mask=m, cell_cap=10, precision="pmx16s").arena_bytes
    idx = cgb.query_sizes(dict(p, indexed=1), wall_mask=m, cell_cap=10, precision="pmx16s").arena_bytes
    # per stored node: populations A, B (2 x 19 x 2 B), densities (2 x 2 B),
    # link moments (4 x 4 B), node momenta (24 B); plus the 4 B index map per site
    want = (ns - nc) * (76 + 4 + 16 + 24) - 4 * ns
    assert abs((dense - idx) - want) < 0.01 * want + 16 * 256
    with pytest.raises(cgb.CgbError):
        cgb.query_sizes(dict(p, indexed=1, tau=0.8), wall_mask=m, cell_cap=10, precision="pmx16s")
