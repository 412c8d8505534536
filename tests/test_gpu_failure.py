"""Failure handling on the GPU, forced from the host: a runaway state must be
reported as instability at the next synchronisation, every kernel must keep
its accesses inside the lattice, and cells must stay inside the box."""
import numpy as np
import pytest

import synth
from parity_util import say

pytestmark = pytest.mark.gpu


def test_runaway_cell_reported_and_kept_in_box():
    from paper_1005_2594_amd import CgbError, Sim
    p = synth.params(32, 32, 32, force_mode=1, g=(2e-2, 0, 0), force_on_particles=1, rho_p=16.0)
    rng = np.random.default_rng(1)
    X = rng.random((8, 3)) * 32
    say("case: runaway cells under a large body force, p32")
    s = Sim(p, precision="p32")
    s.set_particles(X, synth.random_quaternions(rng, 8), V=np.full((8, 3), 0.45))
    s.init_fluid()
    s.step(40)
    with pytest.raises(CgbError) as e:
        s.sync()
    assert e.value.code == -4
    Xg = s.particles()[0]
    assert np.all(np.isfinite(Xg)) and np.all(Xg >= 0) and np.all(Xg < 32)
    assert s.observables()["bad_step"] >= 0


def test_nan_population_reported():
    from paper_1005_2594_amd import CgbError, Sim
    p = synth.params(16, 16, 16)
    say("case: NaN population, pmx16")
    s = Sim(p, precision="pmx16")
    s.set_particles(np.zeros((0, 3)), np.zeros((0, 4)))
    d = np.zeros((19, 16 ** 3))
    d[5, 77] = np.nan
    s.set_populations(d)
    s.step(2)
    with pytest.raises(CgbError) as e:
        s.sync()
    assert e.value.code == -4
