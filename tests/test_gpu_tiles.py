"""Launch shapes of the fused LB kernel, the plane-linear form (by = 0: bx
consecutive sites of the flattened x-y plane per block) among them: every
node's arithmetic is the same whatever the shape, so populations, owners,
particles and forces are bit-identical; the mixture record differs only in
the summation order of its per-block partials."""
import numpy as np
import pytest

import synth
from paper_1005_2594_amd import Sim
from paper_1005_2594_amd.cgb import CgbError
from parity_util import say

pytestmark = pytest.mark.gpu

STEPS = 12


def _ragged_channel():
    # 41 x 35 plane (1,435 sites: not a multiple of any block), 50 planes
    # (not a multiple of 4, 8 or 16), walls at y = 0 and 34, moving cells
    p = synth.params(41, 35, 50, wall_y=1, force_mode=1, g=(0.0, 0.0, 1e-5), rho_p=64.0, force_on_particles=2)
    rng = np.random.default_rng(71)
    N = 60
    X = synth.uniform_positions(rng, N, (41, 35, 50), y_range=(3.0, 31.0))
    q = synth.random_quaternions(rng, N)
    V = 3e-3 * rng.standard_normal((N, 3))
    L = 0.2 * rng.standard_normal((N, 3))
    return p, X, q, V, L


def _run(p, X, q, V, L, prec, tiles, layout=0):
    g = Sim(dict(p, mem_layout=layout), precision=prec)
    try:
        g.set_particles(X, q, V, L)
        g.init_fluid()
        if tiles is not None:
            g.set_tiles(*tiles)
        g.track(STEPS)
        g.step(STEPS)
        g.sync()
        state = (g.owner(), g.populations(), *g.particles(), *g.forces())
        return state, g.get_track(), g.tiles()
    finally:
        g.close()


@pytest.mark.parametrize("prec", ["p64", "pmx16s", "pmx16"])
def test_plane_linear_tiles_match_patches(prec):
    p, X, q, V, L = _ragged_channel()
    say(f"case: LB tiles, ragged 41x35x50 channel, {len(X)} moving cells, {prec}, {STEPS} steps")
    ref, tref, t0 = _run(p, X, q, V, L, prec, None)
    say("  default tiles", t0)
    for tiles in [(64, 0, 8), (256, 0, 4), (128, 0, 16), (192, 0, 32), (32, 8, 8)]:
        st, tr, used = _run(p, X, q, V, L, prec, tiles)
        assert used == tiles
        for a, b in zip(st, ref):
            assert np.array_equal(a, b), tiles
        # the record's partials are summed per block: another partition moves
        # it by rounding only (FP32 per-thread sums in the FP32 codecs)
        tol = 1e-12 if prec == "p64" else 1e-5
        e = float(np.max(np.abs(tr - tref)) / np.max(np.abs(tref[:, 1])))
        say(f"  {tiles}: state identical, record {e:.1e}")
        assert e <= tol


def test_plane_linear_tiles_large_layout():
    p, X, q, V, L = _ragged_channel()
    say("case: plane-linear tiles in the large-lattice layout, pmx16s ragged channel")
    ref, _, _ = _run(p, X, q, V, L, "pmx16s", None, layout=0)
    st, _, used = _run(p, X, q, V, L, "pmx16s", (256, 0, 16), layout=1)
    assert used == (256, 0, 16)
    for a, b in zip(st, ref):
        assert np.array_equal(a, b)


def test_tile_refusals():
    g = Sim(synth.params(16, 16, 16, tau=0.8), precision="p32")
    try:
        with pytest.raises(CgbError):
            g.set_tiles(256, 0, 8)  # plane-linear tiles need tau = 1
        with pytest.raises(CgbError):
            g.set_tiles(96, 0, 8)  # not a multiple of 64
        with pytest.raises(CgbError):
            g.set_tiles(64, 0, 12)
        g.set_tiles(32, 8, 8)
        assert g.tiles() == (32, 8, 8)
    finally:
        g.close()
