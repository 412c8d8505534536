"""Pins of the oracle's plane-Couette viscometer (Sec. IV, Eq. 23): the
Lees-Edwards seam of x for the LB, the reflective boundary for the cells,
and the apparent viscosity mu_app = Delta p_LE,z / (l_y l_z gammadot)."""
import numpy as np
import pytest

import synth
from oracle import oracle as O

EMPTY = (np.zeros((0, 3)), np.zeros((0, 4)))


def _plasma(nx, ny, nz, U, steps, tau=1.0, u0=None):
    p = synth.params(nx, ny, nz, le_u=U, tau=tau)
    o = O.Oracle(p)
    o.set_particles(*EMPTY)
    o.init_fluid(None, u0)
    o.step(steps)
    return o


@pytest.mark.parametrize("tau", [1.0, 0.8])
def test_plasma_couette_is_exact_and_mu_app_is_one(tau):
    # The plasma alone between the sheared images relaxes to plane Couette
    # flow: v_z(x) linear with slope U / l_x (the image beyond the seam moves
    # at +U), uniform in y and z, so the interpolation across the seam is
    # exact and so is the discrete steady state; the momentum carried across
    # the seam per step is then mu gammadot l_y l_z, i.e. Eq. 23 gives mu_app
    # = mu (rho0 nu, nu = (2 tau - 1)/6) exactly.  Mass is conserved.
    nx, ny, nz, U = 16, 3, 5, 0.02
    o = _plasma(nx, ny, nz, U, 3000, tau)
    rho, u = o.fields()
    uz = u[:, 2].reshape(nz, ny, nx)
    assert np.abs(uz - uz[0, 0]).max() < 1e-16
    prof = uz[0, 0]
    slope = np.polyfit(np.arange(nx), prof, 1)[0]
    assert abs(slope / (U / nx) - 1) < 1e-11
    assert np.abs(prof - (prof[0] + slope * np.arange(nx))).max() < 1e-13
    mu_rel = O.mu_app_le([o.le_flux()], 0, prof, ny, nz, 1.0, tau)
    assert abs(mu_rel - 1) < 1e-10
    assert abs(rho.sum() - nx * ny * nz) < 1e-11
    assert np.abs(u[:, :2]).max() < 1e-17


def test_cells_are_reflected_at_the_sheared_planes():
    # A heavy sphere moving towards the plane x = 0 has its normal velocity
    # negated in the step where its centre comes closer than sigma_perp to
    # the plane, and only then; the same at x = nx - 1.
    nx, a = 20, 2.5
    p = synth.params(nx, 12, 12, R_perp=a, R_par=a, eps=0.0, eps_w=0.0, rho_p=1e10, le_u=1e-3)
    sig = p["sig_perp"]
    for x0, v in ((4.0, -0.1), (nx - 5.0, 0.1)):
        o = O.Oracle(p)
        o.set_particles([[x0, 6.0, 6.0]], [[1.0, 0, 0, 0]], V=[[v, 0, 0]])
        o.init_fluid()
        flipped = None
        for t in range(40):
            X0 = o.particles()[0][0, 0]
            o.step(1)
            X1, _, V1, _ = o.particles()
            dist = X1[0, 0] if v < 0 else nx - 1 - X1[0, 0]
            if flipped is None and np.sign(V1[0, 0]) != np.sign(v):
                flipped = t
                assert dist < sig and (X0 if v < 0 else nx - 1 - X0) >= sig
            if flipped is not None:
                break
        assert flipped is not None
        # it moves away afterwards and never covers a sheared plane
        o.step(20)
        own = o.owner().reshape(12, 12, nx)
        assert (own[:, :, 0] == -1).all() and (own[:, :, nx - 1] == -1).all()


def test_a_cell_on_a_sheared_plane_is_refused():
    p = synth.params(16, 12, 12, R_perp=2.5, R_par=2.5, eps=0.0, le_u=1e-3)
    o = O.Oracle(p)
    o.set_particles([[1.0, 6.0, 6.0]], [[1.0, 0, 0, 0]])
    o.init_fluid()
    with pytest.raises(O.OracleError):
        o.step(1)


def test_suspension_mu_app_exceeds_plasma():
    # cells raise the apparent viscosity of the sheared suspension above the
    # plasma's (Sec. IV measures mu_app / mu > 1 throughout)
    nx, ny, nz, U = 24, 14, 14, 0.024
    p = synth.params(nx, ny, nz, le_u=U, rho_p=synth.RHO_P_DENSE, force_on_particles=0)
    rng = np.random.default_rng(8)
    n = 30
    X = rng.uniform([4.0, 0, 0], [nx - 5.0, ny, nz], (n, 3))
    o = O.Oracle(p)
    o.set_particles(X, synth.random_quaternions(rng, n))
    o.init_fluid()
    o.step(600)
    flux = []
    for _ in range(200):
        o.step(1)
        flux.append(o.le_flux())
    rho, u = o.fields()
    own = o.owner()
    uz = np.where(own == -1, u[:, 2], np.nan).reshape(nz, ny, nx)
    prof = np.nanmean(uz, axis=(0, 1))
    mu = O.mu_app_le(flux, 0, prof, ny, nz, 1.0, 1.0)
    assert mu > 1.05


def _d3q19():
    # the textbook D3Q19 set (Sec. II, Eq. 6): rest 1/3, axes 1/18, face diagonals 1/36
    c = [(0, 0, 0)]
    for a in range(3):
        for s in (1, -1):
            v = [0, 0, 0]
            v[a] = s
            c.append(tuple(v))
    for a, b in ((0, 1), (0, 2), (1, 2)):
        for sa in (1, -1):
            for sb in (1, -1):
                v = [0, 0, 0]
                v[a], v[b] = sa, sb
                c.append(tuple(v))
    w = [1 / 3] + [1 / 18] * 6 + [1 / 36] * 12
    return np.array(c), np.array(w)


def test_seam_interpolates_a_field_varying_in_z():
    # Pins the seam's linear interpolation and Galilean shift (reading R29)
    # where the field varies in z.  A fluid at rest whose density is a
    # triangle wave in z with its kinks on nodes has populations w_r rho(z),
    # linear between any two neighbouring nodes, so interpolating them at
    # the sheared offset is exact: the population pulled across the seam
    # must be w_r rho_s shifted by the equilibrium change for the image's
    # velocity -/+ U e_z (Eq. 6 with u = -/+U e_z, u = 0),
    #   d_r = w_r (rho_s - rho0) + w_r rho_s (3 c.u + 4.5 (c.u)^2 - 1.5 u^2),
    # with rho_s the triangle wave at z - c_z +/- Delta, Delta = U t for
    # t steps completed.  After one step at tau = 1 the density and z
    # momentum of every node are these pulled sums (the collision keeps
    # them).  A wrong offset (its sign, t + 1 for t, the interpolation
    # weights swapped) or a wrong shift fails this at 1e-14.
    nx, ny, nz, U, k, A, rho0 = 6, 3, 8, 0.05, 7, 1e-2, 1.0
    p = synth.params(nx, ny, nz, le_u=U, tau=1.0)
    o = O.Oracle(p)
    o.set_particles(*EMPTY)
    o.init_fluid()
    o.step(k)  # Delta = U k = 0.35 at the next step

    def g(z):  # triangle wave of period nz, kinks at 0 and nz/2
        t = np.mod(z, nz) / nz
        return 1.0 - np.abs(2.0 * t - 1.0)

    z = np.arange(nz)
    rho_z = rho0 + A * g(z)
    rho = np.broadcast_to(rho_z[:, None, None], (nz, ny, nx)).reshape(-1)
    o.init_fluid(rho, np.zeros((nx * ny * nz, 3)))
    o.step(1)
    r_o, u_o = o.fields()
    r_o = r_o.reshape(nz, ny, nx)
    jz_o = (r_o.reshape(-1) * u_o[:, 2]).reshape(nz, ny, nx)
    c, w = _d3q19()
    delta = U * k
    for x, sign in ((0, +1), (nx - 1, -1)):  # into x = 0 along c_x = +1; into nx - 1 along c_x = -1
        rho_e = np.full(nz, rho0)
        jz_e = np.zeros(nz)
        for cr, wr in zip(c, w):
            if cr[0] == sign:
                rs = rho0 + A * g(z - cr[2] + sign * delta)
                uz = -sign * U
                cu = cr[2] * uz
                d = wr * (rs - rho0) + wr * rs * (3 * cu + 4.5 * cu * cu - 1.5 * uz * uz)
            else:
                d = wr * A * g(z - cr[2])
            rho_e += d
            jz_e += d * cr[2]
        for y in range(ny):
            assert np.abs(r_o[:, y, x] - rho_e).max() < 1e-14
            assert np.abs(jz_o[:, y, x] - jz_e).max() < 1e-14
    # interior columns: plain streaming of the density wave
    for x in range(1, nx - 1):
        rho_i = rho0 + sum(wr * A * g(z - cr[2]) for cr, wr in zip(c, w))
        assert np.abs(r_o[:, 0, x] - rho_i).max() < 1e-14
    o.close()
