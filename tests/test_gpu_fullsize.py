"""Full-size parity: the 256^3 Kolmogorov suspension at Ht 0.4 (256,337 cells,
the benchmark's workload) through the HIP path in the launch configuration
the benchmark times (default tiles, the independent phases on side streams),
against the oracle started from the same state.  Every site and every cell is
compared: the oracle steps the whole lattice on the host cores (seconds per
step).  The start has moving, spinning cells and a random velocity field, so
that the moving-boundary terms, transitions and pair forces all act."""
import numpy as np
import pytest

import synth
from oracle import oracle as O
from parity_util import compare_state, make_pair, rel_inf, say

pytestmark = pytest.mark.gpu

W = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)


def _start(precision, seed=12):
    cfg = synth.config3()
    p, X, q = cfg["params"], cfg["X"], cfg["q"]
    rng = np.random.default_rng(seed)
    n = len(X)
    V = 1e-3 * rng.standard_normal((n, 3))
    L = 1e-2 * rng.standard_normal((n, 3))
    u0 = 2e-3 * rng.standard_normal((p["nx"] * p["ny"] * p["nz"], 3))
    say("case: 256^3 Ht 0.4,", n, "cells,", precision, "seed", seed)
    g, o = make_pair(p, X, q, precision=precision, V=V, L=L, u0=u0)
    # the oracle starts from the populations as stored on the device (the
    # FP16 codecs round the initial state)
    o.set_deviations(g.populations())
    return g, o


def _rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


# FP64 to the parity bar (1e-12 relative; measured ~2e-15 over these two
# steps); FP32 storage and collision to the velocity bound stated for FP32
# (1e-5 relative)
@pytest.mark.parametrize("precision,tol_pop,tol_part", [("p64", 1e-12, 1e-12), ("p32", 1e-5, 1e-5)])
def test_fullsize_matches_oracle(precision, tol_pop, tol_part):
    g, o = _start(precision)
    for t in range(2):
        g.step(1)
        o.step(1)
        rep = compare_state(g, o, tol_pop=tol_pop, tol_part=tol_part)
        say(" ", precision, "step", t + 1, {k: float(f"{v:.3g}") for k, v in rep.items()})
    g.close()


def test_fullsize_pmx16s_matches_oracle():
    g, o = _start("pmx16s")
    g.step(1)
    o.step(1)
    # one step from the same state: the occupancy is rasterised from the same
    # cells, so it must agree exactly
    og, oo = g.owner(), o.owner()
    assert np.array_equal(og, oo), f"owner maps differ at {np.count_nonzero(og != oo)} nodes"
    assert np.array_equal(g.link_mask(), o.link_mask())
    fl = oo == -1
    dg, do = g.populations()[:, fl], o.deviations()[:, fl]
    # each stored population is w_r (D + h / S): the residual h carries FP16's
    # relative rounding (2^-11) of delta_r / w_r - D, the node's density
    # deviation D its own; the FP32 collision adds ~1e-7 of rho0 w_r
    D = do.sum(axis=0)
    bound = W[:, None] * (2.0 ** -11 * (np.abs(do / W[:, None] - D) + 2.0 ** -11 * np.abs(D)) + 1e-6)
    ratio = float(np.max(np.abs(dg - do) / bound))
    say("  pmx16s step 1: max |error| / codec bound", ratio)
    assert ratio <= 1.0
    rg, ug = g.fields()
    ro, uo = o.fields()
    e1 = _rel_l2(ug[fl], uo[fl])
    say("  pmx16s step 1: velocity rel L2", e1)
    assert e1 <= 1e-3
    Fg, Fo = g.forces(), o.forces()
    ef = {k: rel_inf(a, b) for k, a, b in zip(("Fh", "Th", "Fp", "Tp"), Fg, Fo)}
    say("  pmx16s step 1: force rel inf", ef)
    # pair forces come from identical positions and axes, in FP64 on both
    # sides: the FP64 parity bar (measured ~1e-15)
    assert ef["Fp"] <= 1e-12 and ef["Tp"] <= 1e-12
    # hydrodynamic forces are sums over links of FP16-stored populations
    assert _rel_l2(Fg[0], Fo[0]) <= 1e-3 and _rel_l2(Fg[1], Fo[1]) <= 1e-3
    # two more steps: positions now differ by rounding, so a node at the
    # boundary of a cell's inside test may change owner one step apart; the
    # velocity is compared where both hold fluid
    g.step(2)
    o.step(2)
    og, oo = g.owner(), o.owner()
    nflip = int(np.count_nonzero(og != oo))
    fl = (og == -1) & (oo == -1)
    e3 = _rel_l2(g.fields()[1][fl], o.fields()[1][fl])
    Xg, Xo = g.particles()[0], o.particles()[0]
    pos = float(np.sqrt(np.mean(np.sum((Xg - Xo) ** 2, axis=1))))
    say("  pmx16s step 3: owner differences", nflip, "velocity rel L2", e3, "position rms", pos)
    assert nflip <= 16
    assert e3 <= 1e-3
    assert pos <= 1e-6
    g.close()


def test_fullsize_batch_channels_match_oracle():
    """The 64-channel ensemble at its full size (FP16 deviations per
    direction, autotuned tiles, one replayed graph of two steps); the
    smallest, the largest and the densest channel against the oracle."""
    from paper_1005_2594_amd import Batch
    chans = synth.config4()
    sites = [c["params"]["nx"] * c["params"]["ny"] * c["params"]["nz"] for c in chans]
    pick = sorted({int(np.argmin(sites)), int(np.argmax(sites)), int(np.argmax([c["hematocrit"] for c in chans]))})
    say("batch 64 channels,", sum(sites), "sites; compared:", [(c, chans[c]["width"], chans[c]["length"]) for c in pick])
    b = Batch([c["params"] for c in chans], precision="pmx16")
    rng = np.random.default_rng(13)
    start = {}
    try:
        for c, (s, ch) in enumerate(zip(b.channels, chans)):
            n = len(ch["X"])
            V = 1e-3 * rng.standard_normal((n, 3))
            L = 1e-2 * rng.standard_normal((n, 3))
            s.set_particles(ch["X"], ch["q"], V, L)
            s.init_fluid(None, 2e-3 * rng.standard_normal((sites[c], 3)))
            if c in pick:
                start[c] = (V, L, s.populations())
        b.autotune(reps=2)
        b.capture(2)
        b.run(2)
        b.sync()
        for c in pick:
            ch, (V, L, d0) = chans[c], start[c]
            o = O.Oracle(ch["params"])
            o.set_particles(ch["X"], ch["q"], V, L)
            o.init_fluid()
            o.set_deviations(d0)
            o.step(2)
            g = b.channels[c]
            np.testing.assert_array_equal(g.owner(), o.owner())
            fl = o.owner() == -1
            # two steps of per-direction FP16 storage (each stored value
            # rounded to 2^-11 of itself, the first step's rounding carried
            # through the second): the mixed-precision bar of 1e-3 relative
            ep = _rel_l2(g.populations()[:, fl], o.deviations()[:, fl])
            eu = _rel_l2(g.fields()[1][fl], o.fields()[1][fl])
            ex = float(np.max(np.abs(g.particles()[0] - o.particles()[0])))
            say("  channel", c, "population rel L2", ep, "velocity rel L2", eu, "max position error", ex)
            assert ep <= 1e-3
            assert eu <= 1e-3
            assert ex <= 1e-8
    finally:
        b.close()
