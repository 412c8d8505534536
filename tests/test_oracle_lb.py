"""Pins of the oracle's lattice-Boltzmann core (Sec. II, Eqs. 1-11) against
closed forms that do not come from the oracle itself."""
import numpy as np
import pytest

import synth
from oracle import oracle as O


def _run(p, steps, X=None, q=None, walls=None, rho=None, u=None):
    o = O.Oracle(p, walls)
    o.set_particles(np.zeros((0, 3)) if X is None else X, np.zeros((0, 4)) if q is None else q)
    o.init_fluid(rho, u)
    o.step(steps)
    return o


def test_d3q19_lattice_moments():
    # Sec. II: weights 1/3, 1/18, 1/36 by |c|; isotropy up to 4th order
    c, w, opp = O.d3q19()
    assert np.isclose(w.sum(), 1.0, rtol=0, atol=1e-15)
    for r in range(19):
        n2 = int((c[r] ** 2).sum())
        assert np.isclose(w[r], {0: 1 / 3, 1: 1 / 18, 2: 1 / 36}[n2], rtol=0, atol=1e-16)
        assert (c[opp[r]] == -c[r]).all()
    assert np.allclose(np.einsum("r,ra->a", w, c), 0, atol=1e-16)
    assert np.allclose(np.einsum("r,ra,rb->ab", w, c, c), np.eye(3) / 3, atol=1e-16)
    m4 = np.einsum("r,ra,rb,rc,rd->abcd", w, c, c, c, c)
    d = np.eye(3)
    iso = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d) + np.einsum("ad,bc->abcd", d, d)) / 9
    assert np.allclose(m4, iso, atol=1e-16)


@pytest.mark.parametrize("u", [(0.0, 0.0, 0.0), (0.01, -0.02, 0.03), (0.1, 0.05, -0.07)])
def test_equilibrium_moments(u):
    # Eqs. 7-8: density and momentum of n^eq are rho and rho u exactly; the
    # second moment is rho (u u + I/3)
    c, w, _ = O.d3q19()
    rho = 1.037
    f = O.equilibrium(rho, u)
    u = np.asarray(u)
    assert np.isclose(f.sum(), rho, rtol=1e-15)
    assert np.allclose(f @ c, rho * u, atol=1e-16)
    assert np.allclose(np.einsum("r,ra,rb->ab", f, c, c), rho * (np.outer(u, u) + np.eye(3) / 3), atol=1e-15)


def test_moving_bounce_back_consistency():
    # Eq. 11: n^eq_rbar(rho, v) + C - n^eq_r(rho, v) leaves only the cubic
    # remainder -9 rho w [(c v)^3 - v^2 (c v)] (second-order consistency)
    c, w, opp = O.d3q19()
    rho, v = 1.02, np.array([0.013, -0.007, 0.021])
    f = O.equilibrium(rho, v)
    for r in range(1, 19):
        cv = c[r] @ v
        C = 2 * w[r] / (1 / 3) * rho * cv
        lhs = f[opp[r]] + C - f[r]
        rhs = -9 * rho * w[r] * (cv ** 3 - (v @ v) * cv)
        assert abs(lhs - rhs) < 1e-17


@pytest.mark.parametrize("tau", [0.8, 1.0, 1.5])
def test_poiseuille_exact_discrete(tau):
    # Plane Poiseuille between mid-link walls: the discrete steady state is the
    # parabola with wall slip (g/2nu)(16 L - 3)/12, L = (tau-1/2)^2, and
    # nu = (2 tau - 1)/6 (Sec. II)
    N, g = 8, 1e-6
    p = synth.params(1, N + 2, 1, tau=tau, wall_y=1, force_mode=1, g=(0, 0, g))
    o = _run(p, 3000 if tau == 1.0 else 20000)
    _, u = o.fields()
    nu = (2 * tau - 1) / 6
    lam = (tau - 0.5) ** 2
    y = np.arange(1, N + 1)
    exact = g / (2 * nu) * (N * N / 4 + (16 * lam - 3) / 12 - (y - (N + 1) / 2) ** 2)
    assert np.max(np.abs(u[1:N + 1, 2] - exact)) < 1e-11 * exact.max()
    assert np.allclose(u[1:N + 1, :2], 0, atol=1e-20)


def test_couette_moving_wall_exact():
    # Eq. 10 moving wall: linear profile u_z = V (y - 1/2)/N between the
    # mid-link planes, exact in the discrete steady state
    N, V = 6, 1e-3
    p = synth.params(1, N + 2, 1, wall_y=1, wall_v_top=(0, 0, V))
    o = _run(p, 6000)
    _, u = o.fields()
    y = np.arange(1, N + 1)
    assert np.max(np.abs(u[1:N + 1, 2] - V * (y - 0.5) / N)) < 1e-9 * V


@pytest.mark.parametrize("steps", [1, 2, 7, 200])
def test_kolmogorov_transient_exact(steps):
    # Periodic shear flow under f_z = f0 sin(k y) at tau = 1: each step maps
    # the amplitude A -> lam A + f0 (5 + cos k)/6 with lam = (2 + cos k)/3;
    # the first collision from rest gives A = f0/2.
    L, f0 = 16, 1e-6
    p = synth.params(1, L, 1, force_mode=2, f0=f0)
    o = _run(p, steps)
    _, u = o.fields()
    k = 2 * np.pi / L
    lam = (2 + np.cos(k)) / 3
    Ad = f0 * (5 + np.cos(k)) / (2 * (1 - np.cos(k)))
    A = Ad + (f0 / 2 - Ad) * lam ** (steps - 1)
    assert np.max(np.abs(u[:, 2] - A * np.sin(k * np.arange(L)))) < 1e-12 * A


def test_mass_conserved_with_walls_and_resting_cells():
    # Bounce-back at rest conserves mass exactly; no cover/uncover happens for
    # fixed cells.
    rng = np.random.default_rng(5)
    p = synth.params(12, 14, 10, wall_y=1, force_mode=1, g=(1e-5, 0, 2e-5))
    X = np.array([[4.3, 5.2, 3.1], [8.6, 9.4, 6.7]])
    q = synth.random_quaternions(rng, 2)
    u0 = 1e-3 * rng.standard_normal((12 * 14 * 10, 3))
    o = O.Oracle(p)
    o.set_particles(X, q, fixed=np.ones(2, np.uint8))
    o.init_fluid(None, u0)
    m0 = o.observables()["mass"]
    o.step(50)
    assert abs(o.observables()["mass"] - m0) < 1e-12 * m0


def test_viscosity_from_shear_wave_decay():
    # nu = (2 tau - 1)/6 (Sec. II): a small shear wave u_z = U sin(k y)
    # relaxes; at tau = 1 the discrete decay factor per step is (2 + cos k)/3
    # which matches exp(-nu k^2) to O(k^4).
    L = 64
    p = synth.params(1, L, 1)
    k = 2 * np.pi / L
    u0 = np.zeros((L, 3)); u0[:, 2] = 1e-5 * np.sin(k * np.arange(L))
    o = _run(p, 100, u=u0)
    _, u = o.fields()
    A = (u[:, 2] @ np.sin(k * np.arange(L))) * 2 / L
    # the amplitude of the first read-out after t steps is U lam^t
    lam = (2 + np.cos(k)) / 3
    assert abs(A - 1e-5 * lam ** 100) < 1e-12 * 1e-5
    assert abs(np.log(lam) + k * k / 6) < k ** 4
