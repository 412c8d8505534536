"""Helpers shared by the GPU parity tests: run the same seeded case through
the HIP path (C ABI) and the oracle, and compare."""
import sys

import numpy as np

from oracle import oracle as O


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def make_pair(params, X=None, q=None, precision="p64", walls=None, V=None, L=None, fixed=None, u0=None):
    from paper_1005_2594_amd import Sim
    g = Sim(params, walls, precision=precision)
    o = O.Oracle(params, walls)
    if X is None:
        X, q = np.zeros((0, 3)), np.zeros((0, 4))
    g.set_particles(X, q, V, L, fixed)
    o.set_particles(X, q, V, L, fixed)
    g.init_fluid(None, u0)
    o.init_fluid(None, u0)
    return g, o


def rel_inf(a, b):
    """||a - b||_inf / ||b||_inf (absolute when b is zero)."""
    den = np.max(np.abs(b))
    num = np.max(np.abs(a - b)) if a.size else 0.0
    return num / den if den > 0 else num


def oracle_sensitivity(params, X, q, steps, walls=None, V=None, L=None, u0=None):
    """Conditioning of the problem itself: how far the oracle's own state
    moves after ``steps`` when every initial x coordinate is perturbed by one
    unit in the last place.  Two correct FP64 implementations that round
    differently cannot agree better than this."""
    runs = []
    for eps in (0.0, 2.2e-16):
        o = O.Oracle(params, walls)
        Xp = np.array(X, dtype=np.float64).copy()
        Xp[:, 0] *= 1.0 + eps
        o.set_particles(Xp, q, V, L)
        o.init_fluid(None, u0)
        o.step(steps)
        runs.append(o)
    a, b = runs
    fl = a.owner() == -1
    out = {"pop": rel_inf(a.deviations()[:, fl], b.deviations()[:, fl]),
           "u": rel_inf(a.fields()[1][fl], b.fields()[1][fl])}
    if a.n:
        for name, x, y in zip(("Fh", "Th", "Fp", "Tp"), a.forces(), b.forces()):
            out[name] = rel_inf(y, x)
        for name, x, y in zip(("X", "q", "V", "L"), a.particles(), b.particles()):
            out[name] = rel_inf(y, x)
    return out


def compare_state(g, o, tol_pop, tol_part, check_geometry=True):
    """Element-wise comparison of the whole state; returns a report dict."""
    rep = {}
    og, oo = g.owner(), o.owner()
    if check_geometry:
        assert np.array_equal(og, oo), f"owner maps differ at {np.count_nonzero(og != oo)} nodes"
        assert np.array_equal(g.link_mask(), o.link_mask()), "link masks differ"
    fluid = oo == -1
    dg, do = g.populations(), o.deviations()
    rep["pop"] = rel_inf(dg[:, fluid], do[:, fluid])
    rg, ug = g.fields()
    ro, uo = o.fields()
    rep["u"] = rel_inf(ug[fluid], uo[fluid])
    rep["rho"] = rel_inf(rg[fluid] - 1.0, ro[fluid] - 1.0)
    assert rep["pop"] <= tol_pop, rep
    assert rep["u"] <= tol_pop, rep
    if o.n:
        Xg, qg, Vg, Lg = g.particles()
        Xo, qo, Vo, Lo = o.particles()
        rep["X"] = np.max(np.abs(Xg - Xo)) / np.max(np.abs(Xo))
        rep["q"] = np.max(np.abs(qg - qo))
        rep["V"] = rel_inf(Vg, Vo)
        rep["L"] = rel_inf(Lg, Lo)
        Fg = g.forces(); Fo = o.forces()
        for name, a, b in zip(("Fh", "Th", "Fp", "Tp"), Fg, Fo):
            rep[name] = rel_inf(a, b)
        for k in ("X", "q", "V", "L", "Fh", "Th", "Fp", "Tp"):
            assert rep[k] <= tol_part, (k, rep)
    return rep
