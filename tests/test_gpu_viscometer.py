"""The plane-Couette viscometer (Sec. IV, Eq. 23) on the GPU against the
oracle: the Lees-Edwards seam of x, the reflective boundary of the cells and
the per-step momentum transfer Delta p_LE,z behind mu_app."""
import numpy as np
import pytest

import synth
from oracle import oracle as O
from parity_util import compare_state, make_pair, oracle_sensitivity, rel_inf, say

pytestmark = pytest.mark.gpu


def test_plasma_couette_on_gpu():
    nx, ny, nz, U = 16, 3, 5, 0.02
    p = synth.params(nx, ny, nz, le_u=U)
    say("case: viscometer, plasma 16x3x5, U 0.02, p64, 3000 steps")
    g, o = make_pair(p)
    g.track(3000)
    g.step(2999); o.step(2999)
    g.step(1); o.step(1)
    rep = compare_state(g, o, 1e-12, 1e-12)
    say(rep)
    fl = g.le_flux()
    assert len(fl) == 3000 and rel_inf(fl[-1:], np.array([o.le_flux()])) < 1e-12
    assert abs(g.mu_rel(2999) - 1) < 1e-10
    prof = g.plane_profile(0)
    assert abs(np.polyfit(np.arange(nx), prof, 1)[0] / (U / nx) - 1) < 1e-11


def _suspension(prec, steps_per_check=5, checks=8, seed=8):
    nx, ny, nz, U = 24, 14, 14, 0.024
    p = synth.params(nx, ny, nz, le_u=U, rho_p=synth.RHO_P_DENSE, force_on_particles=0)
    rng = np.random.default_rng(seed)
    n = 30
    X = rng.uniform([4.0, 0, 0], [nx - 5.0, ny, nz], (n, 3))
    q = synth.random_quaternions(rng, n)
    # cells drifting towards the sheared planes, so that reflections happen
    V = np.zeros((n, 3))
    V[:, 0] = np.where(X[:, 0] < nx / 2, -0.05, 0.05)
    return p, X, q, V


def test_suspension_parity_p64():
    p, X, q, V = _suspension("p64")
    sens = oracle_sensitivity(p, X, q, 40, V=V)
    tol = max(1e-12, 10 * max(sens.values()))
    say(f"case: viscometer suspension 24x14x14, 30 cells moving to the sheared planes, p64, 40 steps, tol {tol:.2e}")
    g, o = make_pair(p, X, q, V=V)
    g.track(40)
    flux_o = []
    flips = 0
    v0 = np.sign(V[:, 0])
    for t in range(8):
        for _ in range(5):
            g.step(1); o.step(1)
            flux_o.append(o.le_flux())
        say(compare_state(g, o, tol, tol))
        flips = int((np.sign(o.particles()[2][:, 0]) != v0).sum())
    assert flips > 0  # cells were reflected
    assert rel_inf(g.le_flux(), np.array(flux_o)) < max(tol, 1e-12)


def test_suspension_parity_p32():
    p, X, q, V = _suspension("p32")
    say("case: viscometer suspension, p32, 40 steps")
    g, o = make_pair(p, X, q, V=V, precision="p32")
    g.track(40)
    flux_o = []
    for _ in range(40):
        g.step(1); o.step(1)
        flux_o.append(o.le_flux())
    assert np.array_equal(g.owner(), o.owner())
    fl = o.owner() == -1
    err = rel_inf(g.fields()[1][fl], o.fields()[1][fl])
    say("  p32 velocity rel err", err)
    assert err < 1e-5
    assert rel_inf(g.le_flux(), np.array(flux_o)) < 1e-5


def test_viscometer_refusals():
    from paper_1005_2594_amd import Sim
    from paper_1005_2594_amd.cgb import CgbError
    for extra, prec in ((dict(wall_y=1), "p64"), ({}, "pmx16s")):
        with pytest.raises(CgbError):
            Sim(synth.params(16, 12, 12, le_u=0.01, **extra), precision=prec)
    # a cell on a sheared plane is refused when it is rasterised
    g = Sim(synth.params(16, 12, 12, R_perp=2.5, R_par=2.5, eps=0.0, le_u=1e-3), precision="p64")
    with pytest.raises(CgbError) as e:
        g.set_particles([[1.0, 6.0, 6.0]], [[1.0, 0, 0, 0]])
    assert "sheared plane" in str(e.value)
