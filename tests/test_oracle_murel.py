"""Pins of the apparent-viscosity estimators and the mixture-velocity
observable they read (oracle only)."""
import numpy as np
import pytest

import synth
from oracle import oracle as O


def test_kolmogorov_amplitude_follows_the_mode_recursion():
    # tau = 1, pure shear mode from rest: the first collision gives A = f0/2,
    # each further step A -> lam A + f0 (5 + cos k)/6, lam = (2 + cos k)/3
    L, f0 = 32, 1e-6
    o = O.Oracle(synth.params(1, L, 1, force_mode=2, f0=f0))
    o.init_fluid()
    tr = o.track(40)
    k = 2 * np.pi / L
    lam = (2 + np.cos(k)) / 3
    A = np.empty(40)
    A[0] = f0 / 2
    for t in range(1, 40):
        A[t] = lam * A[t - 1] + f0 * (5 + np.cos(k)) / 6
    assert np.max(np.abs(tr[:, 0] - A)) < 1e-12 * A.max()
    assert np.max(np.abs(tr[:, 1])) < 1e-20  # the sine mode has zero mean


def test_kolmogorov_estimator_is_one_for_the_plasma():
    # every per-step value of the estimator is 1 for the particle-free fluid,
    # during the transient from rest as at late times
    L, f0 = 32, 1e-6
    o = O.Oracle(synth.params(1, L, 1, force_mode=2, f0=f0))
    o.init_fluid()
    A = o.track(60)[:, 0]
    for first in (0, 1, 10, 50):
        assert O.mu_rel_kolmogorov(A, f0, 1.0, L, first) == pytest.approx(1.0, abs=1e-9)
    # a mode that decays twice as fast reads as twice the viscosity
    k = 2 * np.pi / L
    lam2 = 1 - 2 * (1 - np.cos(k)) / 3
    B = np.empty(60)
    B[0] = f0 / 2
    for t in range(1, 60):
        B[t] = lam2 * B[t - 1] + f0 * (5 + np.cos(k)) / 6
    assert O.mu_rel_kolmogorov(B, f0, 1.0, L, 1) == pytest.approx(2.0, rel=1e-9)


@pytest.mark.parametrize("tau,steps", [(1.0, 3000), (1.5, 4000)])
def test_slit_estimator_is_one_for_the_plasma(tau, steps):
    N, g = 8, 1e-6
    o = O.Oracle(synth.params(1, N + 2, 1, tau=tau, wall_y=1, force_mode=1, g=(0, 0, g)))
    o.init_fluid()
    o.step(steps - 50)
    ub = o.track(50)[:, 1]
    assert O.mu_rel_slit(ub, g, tau, N + 2, 0) == pytest.approx(1.0, abs=1e-9)


def test_mixture_counts_cell_nodes_at_the_cell_velocity():
    # one cell moving with V (no rotation): the mixture sum minus the fluid
    # nodes' velocities is the number of cell nodes times V_z of the step
    p = synth.params(16, 16, 16)
    V = np.array([[0.0, 0.0, 2e-3]])
    o = O.Oracle(p)
    o.set_particles([[7.3, 8.1, 7.7]], [[0.9, 0.1, -0.3, 0.2] / np.linalg.norm([0.9, 0.1, -0.3, 0.2])], V=V)
    o.init_fluid()
    o.step(1)
    A, ub = o.mixture()
    own = o.owner()
    _, u = o.fields()
    N = 16 ** 3
    ncell = int((own >= 0).sum())
    assert ncell > 20
    assert ub * N - u[own == -1, 2].sum() == pytest.approx(ncell * V[0, 2], rel=1e-12)


def test_fixed_cells_raise_the_slit_viscosity():
    # resting obstacles in a body-force driven slit can only lower the flux:
    # against the particle-free channel after the same number of steps from
    # rest, the apparent viscosity rises
    rng = np.random.default_rng(11)
    W, g = 16, 1e-5
    p = synth.params(16, W, 16, wall_y=1, force_mode=1, g=(0, 0, g))
    X = np.array([[4.0, 5.0, 4.0], [11.5, 10.5, 9.0], [5.0, 11.0, 12.5]])
    q = synth.random_quaternions(rng, 3)
    mus = []
    for cells in (False, True):
        o = O.Oracle(p)
        if cells:
            o.set_particles(X, q, fixed=np.ones(3, np.uint8))
        o.init_fluid()
        o.step(2400)
        mus.append(O.mu_rel_slit(o.track(100)[:, 1], g, 1.0, W, 0))
    assert 0.95 < mus[0] < 1.05
    assert mus[1] > 1.1 * mus[0]
