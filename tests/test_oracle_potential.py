"""Pins of the Berne-Pechukas pair and wall potentials (Sec. III, Eqs. 15-20)."""
import numpy as np
import pytest

import synth
from oracle import oracle as O


def _rot(axis, ang):
    axis = np.asarray(axis, float) / np.linalg.norm(axis)
    K = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
    return np.eye(3) + np.sin(ang) * K + (1 - np.cos(ang)) * K @ K


def _unit(v):
    v = np.asarray(v, float)
    return v / np.linalg.norm(v)


PAPER = synth.params(64, 64, 64, R_perp=5.5, R_par=11 / 6, sig_perp=6.0, sig_par=2.0, r_cut=100.0)
BJ = synth.params(64, 64, 64, r_cut=100.0)


@pytest.mark.parametrize("P", [PAPER, BJ])
def test_contact_distances(P):
    # zero-energy surface: face-to-face 2 sig_par, edge-to-edge 2 sig_perp
    # (= sigma-bar), T-shape sqrt(2 (sig_perp^2 + sig_par^2)) from Eq. 17 with
    # (a, b, g) = (1, 1, 1), (0, 0, 1), (1, 0, 0)
    sp, sl = P["sig_perp"], P["sig_par"]
    z, x = np.array([0, 0, 1.0]), np.array([1.0, 0, 0])
    cases = [(z, z, z, 2 * sl), (z, x, x, 2 * sp), (z, z, x, np.sqrt(2 * (sp * sp + sl * sl)))]
    for rhat, oi, oj, dist in cases:
        U_in, _, _, _ = O.bp_pair(P, rhat * dist * (1 - 1e-9), oi, oj)
        U_out, _, _, _ = O.bp_pair(P, rhat * dist * (1 + 1e-9), oi, oj)
        assert U_in > 0 and U_out == 0


def test_paper_shape_contact_values():
    # sigma_perp = 6, sigma_par = 2 (the paper's Sec. IV values): chi = -0.8,
    # face 4, edge 12, T-shape 8.944
    sp, sl = 6.0, 2.0
    assert np.isclose((sl ** 2 - sp ** 2) / (sl ** 2 + sp ** 2), -0.8)
    assert np.isclose(np.sqrt(2 * (sp ** 2 + sl ** 2)), 8.94427191, atol=1e-8)


def test_wall_contact_distances():
    # Eqs. 19-20: facing the wall sqrt(sig_par^2 + sig_w^2), edge-on
    # sqrt(sig_perp^2 + sig_w^2)
    P = BJ
    sp, sl, sw = P["sig_perp"], P["sig_par"], P["sig_w"]
    y = np.array([0, 1.0, 0])
    for o, dist in [(y, np.hypot(sl, sw)), (np.array([1.0, 0, 0]), np.hypot(sp, sw))]:
        assert O.bp_wall(P, y * dist * (1 - 1e-9), o)[0] > 0
        assert O.bp_wall(P, y * dist * (1 + 1e-9), o)[0] == 0


def test_strength_scaling_parallel_vs_crossed():
    # Eq. 16: eps = eps-bar / sqrt(1 - chi^2 g^2): parallel cells are stiffer by
    # 1/sqrt(1 - chi^2); crossed cells (g = 0) have eps-bar.  At equal
    # sigma (edge approach, sigma = sigma-bar for both) compare U.
    P = BJ
    chi = (P["sig_par"] ** 2 - P["sig_perp"] ** 2) / (P["sig_par"] ** 2 + P["sig_perp"] ** 2)
    r = np.array([2.0, 0, 0])
    z, y = np.array([0, 0, 1.0]), np.array([0, 1.0, 0])
    Upar = O.bp_pair(P, r, z, z)[0]
    Ux = O.bp_pair(P, r, z, y)[0]
    s = 1 - 2.0 / (2 * P["sig_perp"])
    assert np.isclose(Ux, P["eps"] * s * s, rtol=1e-14)
    assert np.isclose(Upar, P["eps"] / np.sqrt(1 - chi * chi) * s * s, rtol=1e-14)


def _random_config(rng, P, scale):
    oi, oj = _unit(rng.standard_normal(3)), _unit(rng.standard_normal(3))
    for _ in range(1000):
        r = rng.standard_normal(3)
        r = _unit(r) * scale * rng.uniform(0.3, 1.0)
        if O.bp_pair(P, r, oi, oj)[0] > 1e-6:
            return r, oi, oj
    raise RuntimeError


@pytest.mark.parametrize("seed", range(8))
def test_pair_force_and_torque_are_gradients(seed):
    # F_i = -dU/dX_i and tau_i . n = -dU/dtheta for rotations of o_i about n
    rng = np.random.default_rng(seed)
    P = BJ
    r, oi, oj = _random_config(rng, P, 2 * P["sig_perp"])
    U, Fi, ti, tj = O.bp_pair(P, r, oi, oj)
    h = 1e-6
    for a in range(3):
        e = np.zeros(3); e[a] = h
        dU = (O.bp_pair(P, r + e, oi, oj)[0] - O.bp_pair(P, r - e, oi, oj)[0]) / (2 * h)
        assert abs(Fi[a] + dU) < 1e-8 * P["eps"]
        Rp, Rm = _rot(np.eye(3)[a], h), _rot(np.eye(3)[a], -h)
        dUi = (O.bp_pair(P, r, Rp @ oi, oj)[0] - O.bp_pair(P, r, Rm @ oi, oj)[0]) / (2 * h)
        dUj = (O.bp_pair(P, r, oi, Rp @ oj)[0] - O.bp_pair(P, r, oi, Rm @ oj)[0]) / (2 * h)
        assert abs(ti[a] + dUi) < 1e-8 * P["eps"]
        assert abs(tj[a] + dUj) < 1e-8 * P["eps"]


@pytest.mark.parametrize("seed", range(8))
def test_pair_conservation_and_symmetry(seed):
    # Newton's third law; total angular momentum: tau_i + tau_j + r x F_i = 0;
    # swapping i and j; flipping o -> -o (the disc has no head or tail)
    rng = np.random.default_rng(100 + seed)
    P = BJ
    r, oi, oj = _random_config(rng, P, 2 * P["sig_perp"])
    U, Fi, ti, tj = O.bp_pair(P, r, oi, oj)
    assert np.abs(ti + tj + np.cross(r, Fi)).max() < 1e-15
    U2, Fj, tj2, ti2 = O.bp_pair(P, -r, oj, oi)
    assert np.isclose(U, U2, rtol=1e-14)
    assert np.allclose(Fj, -Fi, rtol=0, atol=1e-16)
    assert np.allclose(ti2, ti, atol=1e-16) and np.allclose(tj2, tj, atol=1e-16)
    U3, Fi3, ti3, tj3 = O.bp_pair(P, r, -oi, oj)
    assert np.isclose(U, U3, rtol=1e-14) and np.allclose(Fi, Fi3, atol=1e-16)


@pytest.mark.parametrize("seed", range(6))
def test_wall_force_and_torque_are_gradients(seed):
    rng = np.random.default_rng(200 + seed)
    P = BJ
    o = _unit(rng.standard_normal(3))
    while True:
        r = _unit(rng.standard_normal(3)) * rng.uniform(0.5, 2.7)
        if O.bp_wall(P, r, o)[0] > 1e-6:
            break
    U, F, t = O.bp_wall(P, r, o)
    h = 1e-6
    for a in range(3):
        e = np.zeros(3); e[a] = h
        dU = (O.bp_wall(P, r + e, o)[0] - O.bp_wall(P, r - e, o)[0]) / (2 * h)
        assert abs(F[a] + dU) < 1e-8 * P["eps_w"]
        dUo = (O.bp_wall(P, r, _rot(np.eye(3)[a], h) @ o)[0] - O.bp_wall(P, r, _rot(np.eye(3)[a], -h) @ o)[0]) / (2 * h)
        assert abs(t[a] + dUo) < 1e-8 * P["eps_w"]


def test_hard_cutoff():
    # pairs at or beyond r_cut do not interact, even inside sigma (the cut-off
    # truncates Eq. 15)
    P = dict(BJ, r_cut=3.75)
    rng = np.random.default_rng(0)
    p = synth.params(30, 30, 30)
    o = O.Oracle(p)
    X = np.array([[10.0, 10, 10], [14.5, 10, 10], [10, 13.0, 10]])
    q = np.array([[1.0, 0, 0, 0]] * 3)
    o.set_particles(X, q)
    o.init_fluid()
    o.step(1)
    _, _, Fp, _ = o.forces()
    # particle 1 at distance 4.5 > 3.75 from 0 is edge-to-edge inside sigma-bar
    assert O.bp_pair(P, X[1] - X[0], [0, 0, 1], [0, 0, 1])[0] > 0
    assert np.abs(Fp[1]).max() == 0.0
    assert np.abs(Fp[0]).max() > 0 and np.abs(Fp[2]).max() > 0
    del rng
