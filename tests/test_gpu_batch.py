"""Ensemble of uneven channels advanced by one replayed HIP graph: every
replay equals eager stepping of the same channels, the autotuned launch
shapes keep the results, and one channel agrees with the oracle."""
import numpy as np
import pytest

import synth
from oracle import oracle as O
from parity_util import rel_inf, say

pytestmark = pytest.mark.gpu

# A channel in the batch runs the same kernel bodies on the same data as the
# channel alone, and every reduction has a fixed order (the cover/uncover
# sums are fixed-point): replays equal eager stepping bit for bit.
TOL_REPLAY = 0.0


def small_channels(n=5, seed=41):
    return synth.config4(seed=seed, n_channels=n, w_range=(20, 40), lz_range=(24, 48))


def setup(sim, ch):
    sim.set_particles(ch["X"], ch["q"])
    sim.init_fluid()


def state(sim):
    X, q, V, L = sim.particles()
    return {"pop": sim.populations(), "X": X, "q": q, "V": V, "L": L, "owner": sim.owner(),
            "step": sim.observables()["step"]}


def compare(a, b, tol, tag):
    assert a["step"] == b["step"], (tag, a["step"], b["step"])
    np.testing.assert_array_equal(a["owner"], b["owner"], err_msg=tag)
    for k in ("pop", "X", "q", "V", "L"):
        e = rel_inf(a[k], b[k])
        assert e <= tol, (tag, k, e)


def make(chans, precision="p64"):
    from paper_1005_2594_amd import Batch, Sim
    b = Batch([c["params"] for c in chans], precision=precision)
    for s, c in zip(b.channels, chans):
        setup(s, c)
    ref = []
    for c in chans:
        s = Sim(c["params"], precision=precision)
        setup(s, c)
        ref.append(s)
    return b, ref


def test_batch_replays_match_eager():
    chans = small_channels()
    say("batch: channels", [(c["width"], c["length"], len(c["X"])) for c in chans])
    b, ref = make(chans)
    try:
        b.capture(2)
        for rep in range(3):
            b.run(2)
            for s in ref:
                s.step(2)
            b.sync()
            for c, (g, r) in enumerate(zip(b.channels, ref)):
                compare(state(g), state(r), TOL_REPLAY, f"replay {rep} channel {c}")
            say("batch: replay", rep, "ok")
        # an even number of eager steps between replays keeps the graph valid
        for g in b.channels:
            g.step(2)
        for s in ref:
            s.step(2)
        b.run(4)
        for s in ref:
            s.step(4)
        b.sync()
        for c, (g, r) in enumerate(zip(b.channels, ref)):
            compare(state(g), state(r), TOL_REPLAY, f"after eager channel {c}")
    finally:
        b.close()
        for s in ref:
            s.close()


def test_batch_refuses_stale_graph():
    from paper_1005_2594_amd import CgbError
    chans = small_channels(n=2, seed=42)
    b, ref = make(chans)
    try:
        with pytest.raises(CgbError, match="EINVAL"):
            b.capture(3)
        with pytest.raises(CgbError, match="ESTATE"):
            b.run(2)
        b.capture(2)
        with pytest.raises(CgbError, match="EINVAL"):
            b.run(3)
        b.channels[0].step(1)  # buffer roles swapped
        with pytest.raises(CgbError, match="ESTATE"):
            b.run(2)
        b.channels[0].step(1)
        b.run(2)
        b.sync()
    finally:
        b.close()
        for s in ref:
            s.close()


def test_batch_autotune_keeps_results():
    chans = small_channels(n=4, seed=43)
    b, ref = make(chans)
    try:
        tiles = b.autotune(reps=3)
        say("batch: tiles", tiles.tolist())
        for t, g in zip(tiles, b.channels):
            bx, by, tz = (int(x) for x in t)
            nt = bx if by == 0 else bx * by  # by = 0: plane-linear tiles of bx sites
            assert nt % 64 == 0 and 0 < nt <= 256 and tz in (4, 8, 16, 32)
            assert g.tiles() == (bx, by, tz)
        b.capture(2)
        b.run(6)
        for s in ref:
            s.step(6)
        b.sync()
        for c, (g, r) in enumerate(zip(b.channels, ref)):
            # the LB's launch shape changes no node's arithmetic, and the
            # per-cell sums run in list order: bit for bit
            compare(state(g), state(r), 0.0, f"autotuned channel {c}")
    finally:
        b.close()
        for s in ref:
            s.close()


def test_batch_mu_rel_and_oracle():
    chans = small_channels(n=3, seed=44)
    b, ref = make(chans)
    try:
        b.track(8)
        for s in ref:
            s.track(8)
        b.capture(2)
        b.run(8)
        for s in ref:
            s.step(8)
        b.sync()
        mu = b.mu_rel(first=2)
        for c, s in enumerate(ref):
            assert mu[c] == pytest.approx(s.mu_rel(first=2), rel=1e-9)
        c = 0
        o = O.Oracle(chans[c]["params"])
        o.set_particles(chans[c]["X"], chans[c]["q"])
        o.init_fluid()
        to = o.track(8)
        g = b.channels[c]
        fl = o.owner() == -1
        np.testing.assert_array_equal(g.owner(), o.owner())
        e = rel_inf(g.populations()[:, fl], o.deviations()[:, fl])
        say("batch: channel 0 vs oracle, pop", e)
        assert e <= 1e-11
        for name, x, y in zip(("X", "q", "V", "L"), g.particles(), o.particles()):
            assert rel_inf(x, y) <= 1e-11, name
        mo = O.mu_rel_slit(to[:, 1], chans[c]["params"]["g"][2], 1.0, chans[c]["params"]["ny"], 2)
        say("batch: channel 0 mu_rel", mu[0], "oracle", mo)
        assert mu[0] == pytest.approx(mo, rel=1e-8)
    finally:
        b.close()
        for s in ref:
            s.close()


def test_batch_unfused_channels_match_eager():
    # channels at tau = 0.8 cannot take the one-launch-per-kernel step (its
    # LB kernel is the tau = 1 one): each channel's step sequence runs on its
    # own stream between a fork and joins inside the graph; replays still
    # equal the channels stepped alone, bit for bit
    chans = small_channels(n=3, seed=43)
    for c in chans:
        c["params"] = dict(c["params"], tau=0.8)
    say("batch (tau 0.8, per-channel streams): channels", [(c["width"], c["length"], len(c["X"])) for c in chans])
    b, ref = make(chans, precision="p32")
    try:
        b.capture(2)
        for rep in range(2):
            b.run(4)
            for s in ref:
                s.step(4)
            b.sync()
            for c, (g, r) in enumerate(zip(b.channels, ref)):
                compare(state(g), state(r), 0.0, f"unfused replay {rep} channel {c}")
    finally:
        b.close()
        for s in ref:
            s.close()
