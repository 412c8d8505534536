"""Failure detection of the oracle: non-finite or runaway states must be
reported as instability, deterministically."""
import numpy as np
import pytest

import synth
from oracle import oracle as O


def test_nan_population_trips_instability():
    p = synth.params(8, 8, 8)
    o = O.Oracle(p)
    o.set_particles(np.zeros((0, 3)), np.zeros((0, 4)))
    o.init_fluid()
    d = o.deviations()
    d[3, 100] = np.nan
    o.set_deviations(d)
    with pytest.raises(O.OracleError) as e:
        o.step(1)
    assert e.value.code == -4


def test_huge_force_trips_instability():
    p = synth.params(1, 10, 1, wall_y=1, force_mode=1, g=(0, 0, 0.05))
    o = O.Oracle(p)
    o.set_particles(np.zeros((0, 3)), np.zeros((0, 4)))
    o.init_fluid()
    with pytest.raises(O.OracleError) as e:
        o.step(200)
    assert e.value.code == -4


def test_flat_cell_at_fluid_density_is_unstable_under_explicit_coupling():
    # documents the measured limit: a (2.5, 1.0) disc moving broadside at
    # rho_p = rho0 (added mass ~ (8/3) a^3 > M) grows without bound, while
    # rho_p = 4 rho0 decays
    def run(rho_p):
        p = synth.params(20, 20, 20, eps=0.0, rho_p=rho_p)
        o = O.Oracle(p)
        o.set_particles([[10.0, 10.0, 10.0]], [[1.0, 0, 0, 0]], [[0, 0, 1e-3]], [[0, 0, 0]])
        o.init_fluid()
        try:
            o.step(120)
        except O.OracleError:
            return np.inf
        return np.linalg.norm(o.particles()[2])
    assert run(1.0) > 1e-2
    assert run(4.0) < 1e-3
