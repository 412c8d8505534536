"""Throughput of the coupled LB / rigid-ellipsoid time step on one MI355X.

Workload: 256^3 periodic box, Kolmogorov body force f_z = 1e-6 sin(2 pi y/256),
hematocrit 0.4 (256,337 cells with half axes (2.5, 1.0)), tau = 1.  The
headline number is the mixed-precision path (populations stored as FP16
scaled deviations, FP32 collision, FP64 momentum exchange and integration);
the FP32-storage path runs beside it.  One step = every kernel of the time
step (rasterisation, cover/uncover, fused LB + momentum exchange, cell list,
pair and wall forces, integration).  Inputs are resident in HBM before the
timed region.

Prints one JSON line.  --gpus N > 1 exits: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

METRIC = "MLUPS at 256³ Ht=0.4, mixed vs FP32 at stated error; % of HBM peak"
HBM_PEAK_GBS = 8000.0
STORE_BYTES = {"p64": 8, "p32": 4, "pmx16": 2, "pmxbf16": 2}


def lb_algorithmic_bytes(n_fluid: int, n_sites: int, prec: str) -> float:
    """Bytes one LB launch must move: for every fluid node 19 populations read
    and written plus its density deviation written and read (for Eq. 10), and
    one 4-byte flag word per site."""
    s = STORE_BYTES[prec]
    return n_fluid * (2 * 19 * s + 2 * s) + 4.0 * n_sites


def run_gpu(cfg, prec, steps, warmup, profile=True):
    from paper_1005_2594_amd import Sim
    p = cfg["params"]
    sim = Sim(p, precision=prec)
    sim.set_particles(cfg["X"], cfg["q"])
    sim.init_fluid()
    sim.step(warmup)
    sim.sync()
    nf0 = sim.observables()["n_fluid"]
    if profile:
        sim.profile(True)
    sim.sync()
    t0 = time.perf_counter()
    sim.step(steps)
    sim.sync()
    t1 = time.perf_counter()
    kt = sim.kernel_times() if profile else {}
    if profile:
        sim.profile(False)
    ob = sim.observables()
    nf = 0.5 * (nf0 + ob["n_fluid"])
    out = dict(seconds=t1 - t0, n_fluid=nf, kernel_times=kt, obs=ob, sim=sim)
    return out


def velocity_error_64(seed=3, horizons=(100, 500)):
    """Mixed and FP32 paths against the FP64 path of the same kernels on the
    64^3 companion workload (same cell density; the FP64 path matches the
    oracle to ~1e-14 over 250 steps in the parity runs).  Pointwise errors are
    reported at a short horizon, before discrete events (a node changing
    owner, a pair crossing the cut-off) happen at different steps in different
    precisions; the mixture velocity profile u_z(y) is the long-horizon
    measure."""
    from paper_1005_2594_amd import Sim
    cfg = synth.config3_companion(seed=seed)
    sims = {p: Sim(cfg["params"], precision=p) for p in ("p64", "p32", "pmx16")}
    for s in sims.values():
        s.set_particles(cfg["X"], cfg["q"])
        s.init_fluid()
    res = {p: {} for p in ("p32", "pmx16")}
    done = 0
    for t in horizons:
        for s in sims.values():
            s.step(t - done)
        done = t
        own64 = sims["p64"].owner()
        _, u64 = sims["p64"].fields()
        X64 = sims["p64"].particles()[0]
        pr64 = sims["p64"].profile_z()
        for p in ("p32", "pmx16"):
            own = sims[p].owner()
            _, u = sims[p].fields()
            X = sims[p].particles()[0]
            m = (own == -1) & (own64 == -1)
            pr = sims[p].profile_z()
            res[p][f"step{t}"] = dict(
                rel_l2_u=float(np.linalg.norm(u[m] - u64[m]) / np.linalg.norm(u64[m])),
                rel_l2_profile=float(np.linalg.norm(pr - pr64) / np.linalg.norm(pr64)),
                pos_rms=float(np.sqrt(np.mean(np.sum((X - X64) ** 2, axis=1)))),
                owner_flips=int((own != own64).sum()))
    for s in sims.values():
        s.close()
    return res


def cpu_baseline(cfg, steps):
    """The FP64 oracle on the same 256^3 workload for a few steps (host cores)."""
    from oracle import oracle as O
    o = O.Oracle(cfg["params"])
    o.set_particles(cfg["X"], cfg["q"])
    o.init_fluid()
    t0 = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t0
    ns = cfg["params"]["nx"] * cfg["params"]["ny"] * cfg["params"]["nz"]
    return {"value": ns * steps / dt / 1e6, "unit": "MLUPS", "cores": O.num_threads(), "kind": "oracle",
            "sample": f"{steps} steps of the 256^3 Ht=0.4 workload in FP64 (all sites), set-up excluded",
            "seconds": dt}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=256, help="box edge")
    ap.add_argument("--cpu-steps", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-error", action="store_true")
    ap.add_argument("--only", default=None, help="run only this precision (profiling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; multi-GPU runs are not part of it",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    cfg = synth.config3(n=args.n)
    ns = args.n ** 3
    results = {}
    for prec in ([args.only] if args.only else ["pmx16", "p32"]):
        r = run_gpu(cfg, prec, args.steps, args.warmup)
        results[prec] = r
        print(f"# {prec}: {r['seconds'] * 1e3 / args.steps:.3f} ms/step, "
              f"{ns * args.steps / r['seconds'] / 1e6:.0f} MLUPS, kernels {r['kernel_times']}", flush=True)
        r["sim"].close()

    head = args.only or "pmx16"
    r = results[head]
    mlups = ns * args.steps / r["seconds"] / 1e6
    lb_ms, lb_cnt = r["kernel_times"].get("lb", (float("nan"), 1))
    lb_avg_s = lb_ms / max(lb_cnt, 1) / 1e3
    algo = lb_algorithmic_bytes(r["n_fluid"], ns, head)
    achieved = algo / lb_avg_s / 1e9
    line = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["seconds"] * 1e3 / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"kolmogorov {args.n}^3 periodic, Ht=0.4 ({len(cfg['X'])} cells (2.5,1.0)), tau=1, "
                        f"f0=1e-6; populations stored as {head}",
            "sites": ns, "cells": len(cfg["X"]), "precision": head,
            "kernel_ms_per_step": {k: round(v[0] / max(v[1], 1), 4) for k, v in r["kernel_times"].items()},
        },
        "roofline": {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "kernel": "lb_kernel", "algorithmic_bytes_per_launch": algo,
            "avg_launch_ms": round(lb_avg_s * 1e3, 5),
        },
    }
    if "p32" in results and head != "p32":
        r32 = results["p32"]
        line["config"]["p32_mlups"] = round(ns * args.steps / r32["seconds"] / 1e6, 1)
        line["config"]["p32_ms_per_step"] = round(r32["seconds"] * 1e3 / args.steps, 4)
        l32, c32 = r32["kernel_times"].get("lb", (float("nan"), 1))
        line["config"]["p32_lb_frac"] = round(lb_algorithmic_bytes(r32["n_fluid"], ns, "p32") /
                                              (l32 / max(c32, 1) / 1e3) / 1e9 / HBM_PEAK_GBS, 4)
    if not args.no_error:
        line["config"]["error_vs_p64_64cube"] = velocity_error_64()
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(cfg, args.cpu_steps)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
