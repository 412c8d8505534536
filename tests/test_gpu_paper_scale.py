"""The paper's largest system on one GPU (Sec. IV: 1024^2 x 2048 sites,
4.1e6 cells), in the large-lattice layout.  The lattice is 16 x 16 x 32
copies of one periodic 64^3 tile of 500 cells (4,096,000 cells), so the
method's translation invariance fixes the whole run by a run of the tile:
after one step every copy's populations, owners and forces equal the tile's
bit for bit (positions are on a 2^-10 grid, so every copy's coordinates are
exact), and after three steps they agree to the rounding of the absolute
positions.  The tile itself is held to the oracle by the parity tests."""
import numpy as np
import pytest

import synth
from paper_1005_2594_amd import Sim
from parity_util import say

pytestmark = pytest.mark.gpu

# copies checked: corners (wrap in every direction), a middle copy and the
# last one in memory (the largest offsets)
COPIES = [(0, 0, 0), (15, 15, 31), (7, 3, 20), (15, 0, 0), (0, 15, 31), (8, 8, 16)]


def _free_bytes():
    import torch
    free, _ = torch.cuda.mem_get_info()
    return free


def test_paper_scale_equals_its_tile():
    nx, ny, nz = synth.PAPER_SCALE
    t = synth.PAPER_TILE
    reps = (nx // t, ny // t, nz // t)
    if _free_bytes() < 250e9:
        pytest.skip("needs about 250 GB of free device memory")
    tile = synth.paper_scale_tile()
    full = synth.tile_copies(tile, reps)
    n_t = len(tile["X"])
    say(f"case: paper scale {nx}x{ny}x{nz}, {len(full['X'])} cells, pmx16s, large-lattice layout, 1 + 2 steps")
    # the tile: narrow layout, 1 step then 2 more
    g = Sim(tile["params"], precision="pmx16s")
    g.set_particles(tile["X"], tile["q"], tile["V"], tile["L"])
    g.init_fluid()
    g.step(1)
    d1 = g.box((0, 0, 0), (t, t, t))
    f1 = g.forces()
    g.step(2)
    d3 = g.box((0, 0, 0), (t, t, t))
    X3 = g.particles()[0]
    g.close()
    G = Sim(full["params"], precision="pmx16s")
    assert G.ns == nx * ny * nz
    G.set_particles(full["X"], full["q"], full["V"], full["L"])
    G.init_fluid()
    G.step(1)
    say("  one step done")
    F1 = G.forces()
    for c in COPIES:
        k = c[0] + reps[0] * (c[1] + reps[1] * c[2])
        db, ob = G.box((t * c[0], t * c[1], t * c[2]), (t, t, t))
        # a node near a copy's face may be covered by the image of a tile
        # cell that belongs to the neighbouring copy: owners agree modulo
        # the tile's cell count
        assert np.array_equal(np.where(ob >= 0, ob % n_t, ob), d1[1]), c
        assert np.array_equal(db, d1[0]), c
        sl = slice(k * n_t, (k + 1) * n_t)
        for j in range(4):
            assert np.array_equal(F1[j][sl], f1[j]), c
    G.step(2)
    say("  three steps done")
    X = G.particles()[0]
    for c in COPIES:
        k = c[0] + reps[0] * (c[1] + reps[1] * c[2])
        db, ob = G.box((t * c[0], t * c[1], t * c[2]), (t, t, t))
        assert np.array_equal(np.where(ob >= 0, ob % n_t, ob), d3[1]), c
        # populations to one FP16 rounding step of the stored residuals
        # (the copies' positions differ by the rounding of their absolute
        # coordinates after the first step)
        assert np.abs(db - d3[0]).max() < 1e-5, c
        off = t * np.asarray(c, dtype=np.float64)
        dX = X[k * n_t:(k + 1) * n_t] - off - X3
        dX -= np.round(dX / np.array([nx, ny, nz], dtype=np.float64)) * np.array([nx, ny, nz])
        assert np.abs(dX).max() < 1e-10, c
    G.close()
