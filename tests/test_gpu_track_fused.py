"""Mixture record summed inside the tau = 1 LB kernel (one partial per LB
block) against the record of the separate pass over the stored state: the
same per-step sums of u_z sin(2 pi y/ny) and u_z over the non-wall nodes.
The separate pass runs where the LB blocks outnumber the partial slots of a
handle in caller-provided memory; a handle in its own memory grows its slots
when a tile with more blocks is set.  The oracle parity of the fused record
itself is covered by the apparent-viscosity tests."""
import numpy as np
import pytest

import synth
from paper_1005_2594_amd import Sim
from parity_util import say

pytestmark = pytest.mark.gpu

STEPS = 6


def _record(c, prec, tiles=None, arena=False):
    g = Sim(c["params"], precision=prec, cell_cap=len(c["X"]) + 64 if arena else None,
            track_cap=STEPS if arena else 0)
    try:
        g.set_particles(c["X"], c["q"])
        g.init_fluid()
        if tiles is not None:
            g.set_tiles(*tiles)
        g.track(STEPS)
        g.step(STEPS)
        g.sync()
        return g.get_track()
    finally:
        g.close()


def _err(a, b):
    # both columns against the velocity scale of the sin-weighted sum (the
    # plain sum of u_z of a Kolmogorov flow is near zero)
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b[:, 0])))


# tol_order: the same sums over another block partition.  p64 differs in
# rounding order only; the FP32 codecs sum each thread's sweep in FP32, so
# the partition moves the sums by FP32 rounding.  tol_sep: p64, rounding order
# (the separate pass forms u_z from the stored post-collision moments);
# split FP16 storage, the separate pass decodes the stored FP16 state while
# the fused sum takes the collision's velocity before storage: they differ by
# the storage rounding, which moves the series by about 5e-5 on these cases.
@pytest.mark.parametrize("prec,tol_order,tol_sep", [("p64", 1e-12, 1e-10), ("pmx16s", 1e-5, 5e-4)])
def test_fused_record_matches_separate_pass(prec, tol_order, tol_sep):
    c = synth.kolmogorov(96, seed=61, hematocrit=0.2, f0=1e-5)
    say(f"case: fused vs separate mixture record, {prec} 96^3, {len(c['X'])} cells")
    # default tiles (64x4x16: 288 blocks), fused
    base = _record(c, prec)
    assert base.shape == (STEPS, 2)
    # 64x1x4: 4,608 blocks; own memory grows the partial slots, still fused
    grown = _record(c, prec, tiles=(64, 1, 4))
    # caller-provided memory keeps its slots (sized for the default tiles):
    # the same tile falls back to the separate pass
    sep = _record(c, prec, tiles=(64, 1, 4), arena=True)
    fused_arena = _record(c, prec, arena=True)
    e1, e2, e3 = _err(grown, base), _err(sep, base), _err(fused_arena, base)
    say(f"  grown slots {e1:.2e}, separate pass {e2:.2e}, arena fused {e3:.2e}")
    assert e1 <= tol_order and e3 <= tol_order
    assert e2 <= tol_sep
    # a non-trivial record: the flow has spun up
    assert np.all(np.abs(base[1:, 0]) > 0)
