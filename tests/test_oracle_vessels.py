"""Pins of the oracle on the paper's vessel geometries (Sec. IV): a
staircase cylinder driven by a uniform body force, and a bifurcation of
cylindrical capillaries driven by a body force in the entrance region only,
with and without a stenosis in one branch."""
import numpy as np
import pytest

import synth
from oracle import oracle as O

EMPTY = (np.zeros((0, 3)), np.zeros((0, 4)))


def _plasma(mask, steps, **kw):
    p = synth.vessel_params(mask, **kw)
    o = O.Oracle(p, wall_mask=mask)
    o.set_particles(*EMPTY)
    o.init_fluid()
    o.step(steps)
    return o


@pytest.mark.parametrize("R", [4, 8, 12])
def test_cylinder_hagen_poiseuille(R):
    # Steady plasma flow in the staircase cylinder against the Hagen-Poiseuille
    # law Q = pi R^4 rho0 g / (8 mu): with mid-link bounce-back each fluid
    # node stands for a unit square of the cross-section, so the radius is
    # the one of the fluid area, R_eff = sqrt(N_fluid / pi); the remaining
    # difference is the staircase wall (a few per cent, shrinking with R).
    # The cross-section keeps the square lattice's eight symmetries.
    m = synth.cylinder_mask(R, 3)
    g = 1e-5
    o = _plasma(m, int(3.5 * R * R * 6), force_mode=1, g=(0.0, 0.0, g))
    u = o.mixture_field().reshape(3, m.shape[1], m.shape[2], 3)
    uz = u[1, :, :, 2]
    Q = uz.sum()
    reff = np.sqrt((1 - m[1]).sum() / np.pi)
    nu = 1.0 / 6.0
    mu_rel = np.pi * reff ** 4 * g / (8.0 * Q * nu)
    assert abs(mu_rel - 1.0) < 0.035, mu_rel
    scale = np.abs(uz).max()
    for img in (uz[::-1], uz[:, ::-1], uz.T):
        assert np.abs(uz - img).max() < 1e-13 * scale
    assert np.abs(u[..., :2]).max() < 1e-5 * scale   # the transient's remains
    # and the law's own scaling: doubling the force doubles the flow
    o2 = _plasma(m, int(3.5 * R * R * 6), force_mode=1, g=(0.0, 0.0, 2 * g))
    Q2 = o2.mixture_field().reshape(3, m.shape[1], m.shape[2], 3)[1, :, :, 2].sum()
    assert abs(Q2 / Q - 2.0) < 1e-3


def _split(sten, steps=2000):
    m = synth.bifurcation_mask(4, 3, 4, 48, stenosis=sten)
    L, ny, nx = m.shape
    o = _plasma(m, steps, force_mode=1, g=(0.0, 0.0, 1e-4), force_zlo=0, force_zhi=6)
    u = o.mixture_field().reshape(L, ny, nx, 3)
    rho, _ = o.fields()
    rho = rho.reshape(L, ny, nx)
    xs = np.arange(nx)
    cx = (nx - 1) / 2.0
    ql = u[L // 2][:, xs < cx, 2].sum()
    qr = u[L // 2][:, xs > cx, 2].sum()
    flux = (rho * u[..., 2]).sum(axis=(1, 2))
    return qr / (ql + qr), flux, u, m, o


def test_symmetric_bifurcation_splits_evenly_and_conserves_mass():
    # equal branches: the mirror-symmetric mask gives a mirror-symmetric
    # flow, half of it through each branch; at steady state the same mass
    # flows through every cross-section
    q, flux, u, m, o = _split(None)
    assert abs(q - 0.5) < 1e-13
    assert np.abs(u[..., 2] - u[:, :, ::-1, 2]).max() < 1e-13 * np.abs(u[..., 2]).max()
    assert np.abs(u[..., 0] + u[:, :, ::-1, 0]).max() < 1e-13 * np.abs(u[..., 2]).max()
    assert np.abs(flux - flux.mean()).max() < 1e-8 * flux.mean()
    assert (np.asarray(u)[m.astype(bool)] == 0).all()


def test_stenosis_lowers_the_flow_fraction_monotonically():
    # a narrower stenosis in the +x branch takes a smaller share of the flow
    # (the paper: the flow fraction is monotonic in the stenosis radius)
    qs = [_split((rs, 6))[0] for rs in (3.0, 2.0, 1.2)]
    assert abs(qs[0] - 0.5) < 1e-13   # radius 3 is the branch's own radius
    assert 0.5 > qs[1] > qs[2] > 0.0


def test_entrance_region_force():
    # the constant force acts on the fluid nodes of the region only: the
    # momentum it adds per step is g times their number
    m = synth.bifurcation_mask(4, 3, 4, 48)
    o = _plasma(m, 3, force_mode=1, g=(0.0, 0.0, 1e-4), force_zlo=0, force_zhi=6)
    obs = o.observables()
    nreg = (1 - m[:6]).sum()
    assert abs(obs["body_force_last"][2] - 1e-4 * nreg) < 1e-16 * nreg
    assert obs["body_force_last"][0] == 0.0 and obs["body_force_last"][1] == 0.0
