"""The vessel geometries of the paper (Sec. IV) on the GPU against the
oracle: a bifurcation of cylindrical capillaries with a stenosis in one
branch, driven by a body force in the entrance region only, with cells
moving through it (arbitrary wall surfaces: curved-wall links and the
cell-wall potential over surface wall nodes), and a straight cylinder."""
import numpy as np
import pytest

import synth
from parity_util import compare_state, make_pair, oracle_sensitivity, rel_inf, say

pytestmark = pytest.mark.gpu


def _bifurcation_case(seed=41, n=6):
    m = synth.bifurcation_mask(5, 4, 5, 48, stenosis=(2.0, 6))
    p = synth.vessel_params(m, force_mode=1, g=(0.0, 0.0, 1e-4), force_zlo=0, force_zhi=6, rho_p=16.0,
                            force_on_particles=0)
    X, q = synth.vessel_cells(m, n, p["R_perp"], seed, clear=0.0)
    # one more cell flat against the parent's wall, inside the range of the
    # cell-wall potential (its axis normal to the wall)
    L_, ny, nx = m.shape
    c = np.sqrt(0.5)
    X = np.vstack([X, [[(nx - 1) / 2.0, (ny - 1) / 2.0 + 3.7, 3.0]]])
    q = np.vstack([q, [[c, -c, 0.0, 0.0]]])
    rng = np.random.default_rng(seed)
    V = 2e-3 * rng.standard_normal((n + 1, 3))
    L = 0.05 * rng.standard_normal((n + 1, 3))
    return m, p, X, q, V, L


def test_bifurcation_with_cells_p64():
    m, p, X, q, V, L = _bifurcation_case()
    steps = 40
    sens = oracle_sensitivity(p, X, q, steps, walls=m, V=V, L=L)
    tol = max(1e-12, 10 * max(sens.values()))
    say(f"case: bifurcation with stenosis 21x13x48, {len(X)} cells, entrance force, p64, {steps} steps, tol {tol:.2e}")
    g, o = make_pair(p, X, q, "p64", walls=m, V=V, L=L)
    g.step(steps)
    o.step(steps)
    compare_state(g, o, tol, tol)
    assert np.abs(o.forces()[2]).max() > 0.0   # the wall potential acted
    # the mixture velocity (the flow rates of the branches sum it over planes)
    L_, ny, nx = m.shape
    ug = g.mixture_box((0, 0, 0), (nx, ny, L_)).reshape(-1, 3)
    uo = o.mixture_field()
    assert rel_inf(ug, uo) <= tol
    g.close()


def test_bifurcation_flow_fraction_pmx16s():
    # the plasma's split between the branches, the observable of the
    # bifurcation runs, from the mixture velocity on the middle plane
    m = synth.bifurcation_mask(4, 3, 4, 48, stenosis=(2.0, 6))
    p = synth.vessel_params(m, force_mode=1, g=(0.0, 0.0, 1e-4), force_zlo=0, force_zhi=6)
    say("case: bifurcation plasma flow fraction, pmx16s and p32 against the oracle, 1500 steps")
    L_, ny, nx = m.shape
    xs = np.arange(nx)
    cx = (nx - 1) / 2.0
    fr = {}
    for prec in ("p32", "pmx16s"):
        g, o = make_pair(p, precision=prec, walls=m)
        g.step(1500)
        u = g.mixture_box((0, 0, L_ // 2), (nx, ny, 1))[0]
        fr[prec] = u[:, xs > cx, 2].sum() / u[:, xs != cx, 2].sum()
        g.close()
    o.step(1500)
    uo = o.mixture_field().reshape(L_, ny, nx, 3)[L_ // 2]
    ref = uo[:, xs > cx, 2].sum() / uo[:, xs != cx, 2].sum()
    assert 0.2 < ref < 0.35
    assert abs(fr["p32"] - ref) < 1e-5 * ref
    assert abs(fr["pmx16s"] - ref) < 1e-3 * ref


def test_cylinder_with_cells_p32():
    mk = synth.cylinder_mask(6, 40)
    p = synth.vessel_params(mk, force_mode=1, g=(0.0, 0.0, 2e-5), rho_p=16.0, force_on_particles=2)
    X, q = synth.vessel_cells(mk, 5, p["R_perp"], 42, clear=0.5)
    steps = 40
    say(f"case: cylinder R 6 x 40, {len(X)} cells, body force on plasma and cells, p32, {steps} steps")
    g, o = make_pair(p, X, q, "p32", walls=mk)
    g.step(steps)
    o.step(steps)
    compare_state(g, o, 1e-5, 1e-5)
    g.close()


@pytest.mark.parametrize("prec", ["p64", "p32", "pmx16s"])
def test_indexed_layout_matches_dense(prec):
    # the indexed layout stores the non-wall nodes only (27 % of this box);
    # every result equals the dense layout's bit for bit
    from paper_1005_2594_amd import Sim
    m, p, X, q, V, L = _bifurcation_case(seed=45)
    L_, ny, nx = m.shape
    say(f"case: indexed vs dense layout, bifurcation 21x13x48 with {len(X)} cells, {prec}, 30 steps")
    out = []
    for idx in (0, 1):
        g = Sim(dict(p, indexed=idx), m, precision=prec)
        g.set_particles(X, q, V, L)
        g.init_fluid()
        g.step(30)
        out.append((g.owner(), g.populations(), *g.particles(), *g.forces(),
                    g.mixture_box((0, 0, 0), (nx, ny, L_))))
        if idx:
            assert g.device_bytes < dense_bytes
        else:
            dense_bytes = g.device_bytes
        g.close()
    for x, y in zip(*out):
        assert np.array_equal(x, y)
