"""Graph replay of the time step (cgb_capture / cgb_replay): the captured
sequence, side stream included, gives the eager step's results bit for bit,
replay after replay, with the program's own eager work and synchronisations
in between; the handle refuses a replay once its launches would differ."""
import numpy as np
import pytest

import synth
from paper_1005_2594_amd import Sim
from paper_1005_2594_amd.cgb import CgbError
from parity_util import say

pytestmark = pytest.mark.gpu


def _case(seed=51):
    c = synth.kolmogorov(32, seed, f0=1e-5)
    rng = np.random.default_rng(seed)
    N = len(c["X"])
    return c, 3e-3 * rng.standard_normal((N, 3)), 0.2 * rng.standard_normal((N, 3))


def _state(g):
    return (g.owner(), g.populations(), *g.particles(), *g.forces(), g.pairs())


@pytest.mark.parametrize("prec,concurrent", [("pmx16s", True), ("p64", False)])
def test_replay_matches_eager(prec, concurrent):
    c, V, L = _case()
    say(f"case: graph replay vs eager steps, {prec} 32^3, {len(c['X'])} moving cells, concurrency {concurrent}")
    sims = []
    for _ in range(2):
        g = Sim(c["params"], precision=prec)
        g.set_particles(c["X"], c["q"], V, L)
        g.init_fluid()
        g.set_concurrency(concurrent)
        g.track(40)
        sims.append(g)
    eager, rep = sims
    rep.capture(2)
    for chunk in (6, 4, 8, 6):
        eager.step(chunk)
        rep.replay(chunk)
        a, b = _state(eager), _state(rep)
        for x, y in zip(a, b):
            assert np.array_equal(x, y)
        # eager work of the program's own between the replays
        rep.observables()
        rep.fields()
    assert np.array_equal(eager.get_track(), rep.get_track())
    for g in sims:
        g.close()


def test_replay_refusals():
    c, V, L = _case(52)
    say("case: graph replay refusals (odd eager step, new tiles)")
    g = Sim(c["params"], precision="pmx16s")
    g.set_particles(c["X"], c["q"], V, L)
    g.init_fluid()
    g.capture(2)
    g.replay(4)
    g.step(1)
    with pytest.raises(CgbError):
        g.replay(2)
    g.step(1)
    g.replay(2)
    g.set_tiles(16, 4, 16)
    with pytest.raises(CgbError):
        g.replay(2)
    g.capture(2)
    g.replay(2)
    with pytest.raises(CgbError):
        g.replay(3)
    g.close()
