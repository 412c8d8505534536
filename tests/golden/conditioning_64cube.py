"""Writes conditioning_64cube.json: how far the FP64 oracle's own state moves
when the cell positions of the 64^3 Kolmogorov companion workload (Ht 0.4,
4,005 cells, seed 3, f0 = 1e-6) are perturbed by a relative eps, for eps from
one unit in the last place up to 1e-7 (the size of the position differences
that lower-precision arithmetic produces).  Calls only the oracle.

Reported per eps at steps 100, 250 and 500: the relative L2 difference of
the fluid velocity (over nodes fluid in both runs), the RMS difference of the
cell positions, and the number of (node, step) pairs at which the two owner
maps differed during the run (a node covered or freed one step apart).  The
rasterisation is a discrete event in time: once two runs are far enough
apart for a node to change owner at different steps, the node that was freed
first starts as fluid at rest density among neighbours whose density differs
by up to a few per cent, and the pressure pulse this sends out is large next
to the flow velocity of the early, slowly spinning-up shear flow.

Run from the repository root: python tests/golden/conditioning_64cube.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import oracle as O  # noqa: E402

EPS = [0.0, 2.2e-16, 1e-12, 1e-9, 1e-7]
HORIZONS = (100, 250, 500)


def main():
    cfg = synth.config3_companion()
    p, X, q = cfg["params"], cfg["X"], cfg["q"]
    runs = []
    for eps in EPS:
        o = O.Oracle(p)
        Xp = np.array(X, dtype=np.float64)
        Xp[:, 0] *= 1.0 + eps
        o.set_particles(Xp, q)
        o.init_fluid()
        runs.append(o)
    mism = [0] * len(EPS)
    out = {"workload": "kolmogorov 64^3 periodic, Ht 0.4, 4005 cells (2.5, 1.0), seed 3, f0 1e-6, tau 1, r_cut 3.75",
           "perturbation": "x coordinates of every cell multiplied by (1 + eps) before the first step",
           "eps": EPS[1:], "steps": {}}
    t0 = time.perf_counter()
    for t in range(1, HORIZONS[-1] + 1):
        for o in runs:
            o.step(1)
        own0 = runs[0].owner()
        for k in range(1, len(EPS)):
            mism[k] += int((runs[k].owner() != own0).sum())
        if t in HORIZONS:
            _, u0 = runs[0].fields()
            X0 = runs[0].particles()[0]
            rows = []
            for k in range(1, len(EPS)):
                own = runs[k].owner()
                _, u = runs[k].fields()
                m = (own == -1) & (own0 == -1)
                d = runs[k].particles()[0] - X0
                d -= 64.0 * np.round(d / 64.0)
                rows.append({"eps": EPS[k],
                             "rel_l2_u": float(np.linalg.norm(u[m] - u0[m]) / np.linalg.norm(u0[m])),
                             "pos_rms": float(np.sqrt(np.mean(np.sum(d * d, axis=1)))),
                             "owner_mismatch_node_steps": mism[k]})
            out["steps"][str(t)] = rows
            print(t, round(time.perf_counter() - t0, 1), rows, flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "conditioning_64cube.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
