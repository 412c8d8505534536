"""Pins of the leap-frog / unit-quaternion integrator (Sec. II)."""
import numpy as np
import pytest

import synth
from oracle import oracle as O


def test_free_symmetric_top_precession_second_order():
    # torque-free symmetric top: the axis precesses about the constant L at
    # angular rate |L| / I_perp, keeping o . L fixed.  Error must fall as dt^2.
    Ipar, Iperp = 2.0, 1.3
    rng = np.random.default_rng(1)
    q0 = rng.standard_normal(4); q0 /= np.linalg.norm(q0)
    L = np.array([0.0, 0.0, 0.4])
    o0 = O.axis(q0)
    T = 10.0
    errs = []
    for dt in (0.1, 0.05, 0.025):
        q = q0.copy()
        for _ in range(int(round(T / dt))):
            q = O.rotate(q, L, Ipar, Iperp, dt)
        assert abs(np.linalg.norm(q) - 1) < 1e-14
        ang = np.linalg.norm(L) / Iperp * T
        c, s = np.cos(ang), np.sin(ang)
        R = np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]])
        errs.append(np.linalg.norm(O.axis(q) - R @ o0))
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5


def test_rotation_about_symmetry_axis_keeps_axis():
    q = np.array([np.cos(0.3), np.sin(0.3), 0, 0])
    o = O.axis(q)
    q2 = O.rotate(q, 0.7 * o, 2.0, 1.0, 1.0)
    assert np.allclose(O.axis(q2), o, atol=1e-15)


def test_free_cell_constant_force_exact_leapfrog():
    # a cell too small to cover any node feels no fluid: under the body force
    # g it follows the exact leap-frog quadratic, L stays constant
    g = np.array([1e-4, -2e-4, 3e-4])
    p = synth.params(16, 16, 16, R_perp=0.1, R_par=0.05, force_mode=1, g=tuple(g), eps=0.0)
    o = O.Oracle(p)
    X0 = np.array([[8.5, 8.5, 8.5]]); V0 = np.array([[1e-3, 0, -2e-3]])
    L0 = np.array([[0, 1e-6, 0]])
    o.set_particles(X0, [[1.0, 0, 0, 0]], V0, L0)
    o.init_fluid()
    n = 25
    o.step(n)
    X, q, V, L = o.particles()
    assert (o.owner() == 0).sum() == 0
    assert np.allclose(V, V0 + n * g, rtol=0, atol=1e-15)
    assert np.allclose(X, X0 + n * V0 + n * (n + 1) / 2 * g, rtol=0, atol=1e-12)
    assert np.array_equal(L, L0)
    assert abs(np.linalg.norm(q) - 1) < 1e-14
