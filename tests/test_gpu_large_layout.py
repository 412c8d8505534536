"""The large-lattice layout (64-bit lane addresses in the LB kernel, a cell
node's momentum kept in its own unused population slots) forced on small
lattices: every result equals the narrow layout's bit for bit, so its
indexing and slot packing are checked where the oracle parity tests run."""
import numpy as np
import pytest

import synth
from paper_1005_2594_amd import Sim
from paper_1005_2594_amd.cgb import CgbError
from parity_util import say

pytestmark = pytest.mark.gpu


def _moving(n, seed):
    c = synth.kolmogorov(n, seed, f0=1e-5)
    rng = np.random.default_rng(seed)
    N = len(c["X"])
    return c, 3e-3 * rng.standard_normal((N, 3)), 0.2 * rng.standard_normal((N, 3))


def _run(params, X, q, V, L, prec, layout, steps):
    g = Sim(dict(params, mem_layout=layout), precision=prec)
    g.set_particles(X, q, V, L)
    g.init_fluid()
    own0 = g.owner()
    g.step(steps)
    out = (g.owner(), g.populations(), *g.particles(), *g.forces(), g.pairs())
    moved = int((out[0] != own0).sum())
    g.close()
    return out, moved


@pytest.mark.parametrize("prec", ["p64", "p32", "pmx16", "pmx16s"])
def test_large_layout_matches_narrow(prec):
    c, V, L = _moving(32, 31)
    say(f"case: large-lattice layout vs narrow, {prec} 32^3, {len(c['X'])} moving cells, 20 steps")
    a, moved = _run(c["params"], c["X"], c["q"], V, L, prec, 0, 20)
    b, _ = _run(c["params"], c["X"], c["q"], V, L, prec, 1, 20)
    assert moved > 0
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_large_layout_ragged_box():
    # ragged sizes: rows and planes that do not fill the tiles, wrap at
    # every face
    p = synth.params(37, 29, 23, force_mode=1, g=(0.0, 0.0, 1e-5), rho_p=64.0, force_on_particles=2)
    rng = np.random.default_rng(32)
    N = 40
    X = synth.uniform_positions(rng, N, (37, 29, 23))
    q = synth.random_quaternions(rng, N)
    V = 3e-3 * rng.standard_normal((N, 3))
    L = 0.2 * rng.standard_normal((N, 3))
    say("case: large-lattice layout vs narrow, pmx16s ragged 37x29x23, 40 moving cells, 20 steps")
    a, _ = _run(p, X, q, V, L, "pmx16s", 0, 20)
    b, _ = _run(p, X, q, V, L, "pmx16s", 1, 20)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_box_getter_matches_whole_lattice():
    c, V, L = _moving(32, 33)
    say("case: sub-box getter against the whole-lattice getters, pmx16s 32^3, 5 steps")
    g = Sim(dict(c["params"], mem_layout=1), precision="pmx16s")
    g.set_particles(c["X"], c["q"], V, L)
    g.init_fluid()
    g.step(5)
    d = g.populations().reshape(19, 32, 32, 32)
    own = g.owner().reshape(32, 32, 32)
    lo, ext = (3, 0, 17), (29, 32, 15)
    db, ob = g.box(lo, ext)
    sl = (slice(lo[2], lo[2] + ext[2]), slice(lo[1], lo[1] + ext[1]), slice(lo[0], lo[0] + ext[0]))
    assert np.array_equal(db, d[(slice(None),) + sl])
    assert np.array_equal(ob, own[sl])
    with pytest.raises(CgbError):
        g.box((20, 0, 0), (13, 1, 1))
    g.close()


def test_large_layout_refusals():
    say("case: large-lattice layout refusals (tau != 1, viscometer, tile depth)")
    with pytest.raises(CgbError):
        Sim(synth.params(16, 16, 16, tau=0.8, mem_layout=1), precision="p32")
    with pytest.raises(CgbError):
        Sim(synth.params(16, 16, 16, le_u=0.01, mem_layout=1), precision="p32")
    g = Sim(synth.params(16, 16, 16, mem_layout=1), precision="p32")
    with pytest.raises(CgbError):
        g.set_tiles(16, 4, 8)
    g.close()
