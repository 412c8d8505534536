"""The lattice-unit parameters used by the workloads follow from the
physical values the paper prints (Sec. IV); tests/golden/paper_units.txt
holds them with their citations."""
import os

import numpy as np

import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def _golden():
    out = {}
    for line in open(os.path.join(HERE, "golden", "paper_units.txt")):
        line = line.split("#")[0].strip()
        if line:
            name, val, _ = line.split()[:3]
            out[name] = float(val)
    return out


def test_time_and_mass_units():
    g = _golden()
    nu_lattice = (2 * g["tau"] - 1) / 6          # Sec. II
    dt = nu_lattice * g["dx"] ** 2 / g["nu_plasma"]
    assert abs(dt / g["dt"] - 1) < 5e-3
    dm = g["rho_plasma"] * g["dx"] ** 3
    assert abs(dm / g["dm"] - 1) < 5e-3


def test_potential_strength_in_lattice_units():
    g = _golden()
    energy_unit = g["dm"] * g["dx"] ** 2 / g["dt"] ** 2
    assert abs(g["eps_cell"] / energy_unit / synth.EPS_LU - 1) < 5e-3


def test_shape_aspect_ratio():
    # sigma_perp / sigma_par = 3 for the paper's cells; the workload cells keep
    # R_perp/R_par = 2.5 and sigma = (12/11) R (ratio R_par/sigma_par = 11/12)
    g = _golden()
    assert np.isclose(g["sig_perp"] / g["sig_par"], 3.0)
    p = synth.params(8, 8, 8)
    assert np.isclose(p["R_par"] / p["sig_par"], 11 / 12)
