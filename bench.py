"""Throughput of the coupled LB / rigid-ellipsoid time step on one MI355X.

Workload: 256^3 periodic box, Kolmogorov body force f_z = 1e-6 sin(2 pi y/256),
hematocrit 0.4 (256,337 cells with half axes (2.5, 1.0)), tau = 1.  The
headline number is the mixed-precision path that meets the 1e-3 velocity
error bar: the deviations n*_r - w_r rho0 stored in FP16 as a per-node part
(the density deviation) plus per-direction residuals, FP32 collision, FP64
momentum exchange and integration.  Beside it: FP16 deviations stored per
direction alone (the same storage size, ~8x the velocity error) and the
FP32-storage path.  One step = every kernel of the time
step (rasterisation, cover/uncover, fused LB, momentum-exchange reduction,
cell list, pair and wall forces, integration).  Inputs are resident in HBM
before the timed region.

Also reported (in "config"): the error of the mixed and FP32 paths against
the FP64 path on the 64^3 companion workload, the batched ensemble of 64
uneven channels (one replayed HIP graph, autotuned LB tiles, apparent
viscosity per channel), and the oracle on the host cores ("cpu_baseline").

Prints one JSON line.  --gpus N > 1 exits: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
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
STORE_BYTES = {"p64": 8, "p32": 4, "pmx16": 2, "pmxbf16": 2, "pmx16s": 2}
LB_SOURCE = os.path.join(ROOT, "paper_1005_2594_amd", "csrc", "lb.hip")
HEAD = "pmx16s"
STORE_DESC = {
    "pmx16s": "FP16 deviations n*_r - w_r rho0 split into a per-node FP16 density part and per-direction "
              "FP16 residuals (2 B per population), FP32 collision (pmx16s)",
    "pmx16": "FP16 deviations (n*_r - w_r rho0)/w_r per direction (2 B per population), FP32 collision (pmx16)",
    "p32": "FP32 deviations, FP32 collision (p32)",
}


def traffic_file(prec: str) -> str:
    return os.path.join(ROOT, "profiles", f"lb_traffic_{prec}_256.txt")


def lb_algorithmic_bytes(n_fluid: float, n_sites: int, prec: str) -> float:
    """Bytes one LB launch must move: for every fluid node 19 populations read
    and written plus its density deviation written and read (the density in
    the moving-boundary term of Eq. 10), and one 4-byte flag word per site."""
    s = STORE_BYTES[prec]
    return n_fluid * (2 * 19 * s + 2 * s) + 4.0 * n_sites


def measured_traffic(prec: str):
    """HBM bytes per LB launch from the committed rocprofv3 counter summary,
    or None when it was taken on another version of the kernel source."""
    if not os.path.exists(traffic_file(prec)):
        return None
    kv = {}
    for line in open(traffic_file(prec)):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    src = hashlib.sha256(open(LB_SOURCE, "rb").read()).hexdigest()
    if kv.get("lb_source_sha256") != src or "hbm_bytes_per_launch" not in kv:
        return None
    return float(kv["hbm_bytes_per_launch"])


def run_gpu(cfg, prec, steps, warmup, kernel_steps=50, serial=False):
    """Timed region: `steps` steps with no instrumentation (the independent
    phases of a step on side streams unless `serial`).  Then a kernel pass:
    `kernel_steps` more steps with every kernel in sequence on the handle's
    stream, each bracketed by HIP events (per-kernel times, and the LB launch
    time of the roofline)."""
    from paper_1005_2594_amd import Sim
    p = cfg["params"]
    sim = Sim(p, precision=prec)
    sim.set_particles(cfg["X"], cfg["q"])
    sim.init_fluid()
    sim.set_concurrency(not serial)
    sim.step(warmup)
    sim.sync()
    nf0 = sim.observables()["n_fluid"]
    t0 = time.perf_counter()
    sim.step(steps)
    sim.sync()
    t1 = time.perf_counter()
    kt = {}
    if kernel_steps > 0:
        sim.set_concurrency(False)
        sim.profile(True)
        sim.step(kernel_steps)
        sim.sync()
        kt = sim.kernel_times()
        sim.profile(False)
        sim.set_concurrency(not serial)
    ob = sim.observables()
    nf = 0.5 * (nf0 + ob["n_fluid"])
    return dict(seconds=t1 - t0, n_fluid=nf, kernel_times=kt, obs=ob, sim=sim)


def error_report_64(seed=3, horizons=(100, 250, 500)):
    """Mixed and FP32 paths against the FP64 path of the same kernels on the
    64^3 companion workload (same cell density; the FP64 path matches the
    oracle to ~1e-14 in the parity tests).  Pointwise velocity errors are
    taken at the first horizon, before discrete events (a node changing
    owner, a pair crossing the cut-off) happen at different steps in
    different precisions; the plane-averaged mixture velocity profile and
    the apparent viscosity (Kolmogorov estimator, last half of the run) are
    the long-horizon measures."""
    from paper_1005_2594_amd import Sim
    cfg = synth.config3_companion(seed=seed)
    precs = ("p64", "p32", "pmx16", "pmx16s")
    sims = {p: Sim(cfg["params"], precision=p) for p in precs}
    for s in sims.values():
        s.set_particles(cfg["X"], cfg["q"])
        s.init_fluid()
        s.track(horizons[-1])
    res = {p: {} for p in precs[1:]}
    done = 0
    for t in horizons:
        for s in sims.values():
            s.step(t - done)
        done = t
        own64 = sims["p64"].owner()
        _, u64 = sims["p64"].fields()
        X64 = sims["p64"].particles()[0]
        pr64 = sims["p64"].profile_z()
        for p in precs[1:]:
            own = sims[p].owner()
            _, u = sims[p].fields()
            X = sims[p].particles()[0]
            m = (own == -1) & (own64 == -1)
            pr = sims[p].profile_z()
            d = np.sqrt(np.sum((X - X64) ** 2, axis=1))
            res[p][f"step{t}"] = dict(
                rel_l2_u=float(np.linalg.norm(u[m] - u64[m]) / np.linalg.norm(u64[m])),
                rel_l2_profile=float(np.linalg.norm(pr - pr64) / np.linalg.norm(pr64)),
                pos_rms=float(np.sqrt(np.mean(d ** 2))),
                owner_flips=int((own != own64).sum()))
    first = horizons[-1] // 2
    mu = {p: sims[p].mu_rel(first=first) for p in precs}
    for p in precs[1:]:
        res[p]["mu_rel"] = mu[p]
        res[p]["mu_rel_rel_err"] = abs(mu[p] - mu["p64"]) / abs(mu["p64"])
    res["p64_mu_rel"] = mu["p64"]
    res["mu_rel_window"] = [first, horizons[-1] - 1]
    for s in sims.values():
        s.close()
    return res


def batch_leg(steps=2000, seed=4, prec="pmx16"):
    """64 uneven wall-bounded channels advanced together by one replayed HIP
    graph with autotuned LB tiles; apparent viscosity per channel from the
    mean mixture velocity over steps steps/2 + 1 .. steps."""
    from paper_1005_2594_amd import Batch
    chans = synth.config4(seed=seed)
    t0 = time.perf_counter()
    b = Batch([c["params"] for c in chans], precision=prec)
    for s, c in zip(b.channels, chans):
        s.set_particles(c["X"], c["q"])
        s.init_fluid()
    tiles = b.autotune(reps=5)
    b.track(steps)
    b.capture(2)
    b.sync()
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    b.run(steps)
    b.sync()
    dt = time.perf_counter() - t0
    mu = b.mu_rel(first=steps // 2)
    sites = sum(c["params"]["nx"] * c["params"]["ny"] * c["params"]["nz"] for c in chans)
    shapes = {}
    for t in tiles:
        k = "x".join(str(int(v)) for v in t)
        shapes[k] = shapes.get(k, 0) + 1
    b.close()
    return {
        "workload": f"{len(chans)} channels (W, W, Lz), W~U{{32..96}}, Lz~U{{64..192}}, Ht~U[0.1,0.5], "
                    f"g~logU[1e-7,1e-5], walls y=0,W-1; populations {prec}; one graph of 2 steps replayed",
        "channels": len(chans), "sites": sites, "cells": int(sum(len(c["X"]) for c in chans)),
        "steps": steps, "seconds": round(dt, 3), "ms_per_step": round(dt / steps * 1e3, 4),
        "mlups": round(sites * steps / dt / 1e6, 1), "setup_seconds": round(t_setup, 2),
        "tiles": shapes,
        "mu_rel": {"window": [steps // 2, steps - 1], "mean": float(np.mean(mu)), "min": float(np.min(mu)),
                   "max": float(np.max(mu)), "per_channel": [round(float(m), 5) for m in mu]},
    }


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
    return {"value": round(ns * steps / dt / 1e6, 3), "unit": "MLUPS", "cores": O.num_threads(), "kind": "oracle",
            "sample": f"{steps} steps of the 256^3 Ht=0.4 workload in FP64 (all sites), set-up excluded",
            "seconds": round(dt, 2)}


def copy_calibration(nbytes=1 << 31, reps=4):
    """A plain device-to-device copy of known size, for scaling rocprofv3's
    FETCH_SIZE / WRITE_SIZE counters to bytes."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(f"# copy calibration: {reps} copies of {nbytes} bytes", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=256, help="box edge")
    ap.add_argument("--cpu-steps", type=int, default=2)
    ap.add_argument("--batch-steps", type=int, default=2000)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-error", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--only", default=None, help="run only this precision (profiling)")
    ap.add_argument("--kernel-steps", type=int, default=50, help="steps of the per-kernel timing pass")
    ap.add_argument("--serial", action="store_true", help="every kernel in sequence in the timed region too")
    ap.add_argument("--copy-calibrate", action="store_true", help="also run a copy of known size (counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; multi-GPU runs are not part of it",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)
    if args.copy_calibrate:
        copy_calibration()

    cfg = synth.config3(n=args.n)
    ns = args.n ** 3
    results = {}
    for prec in ([args.only] if args.only else [HEAD, "pmx16", "p32"]):
        r = run_gpu(cfg, prec, args.steps, args.warmup, args.kernel_steps, args.serial)
        results[prec] = r
        print(f"# {prec}: {r['seconds'] * 1e3 / args.steps:.3f} ms/step, "
              f"{ns * args.steps / r['seconds'] / 1e6:.0f} MLUPS, kernels "
              f"{ {k: round(v[0] / max(v[1], 1), 4) for k, v in r['kernel_times'].items()} }", flush=True)
        r["sim"].close()

    head = args.only or HEAD
    r = results[head]
    mlups = ns * args.steps / r["seconds"] / 1e6
    lb_ms, lb_cnt = r["kernel_times"].get("lb", (float("nan"), 1))
    lb_avg_s = lb_ms / max(lb_cnt, 1) / 1e3
    algo = lb_algorithmic_bytes(r["n_fluid"], ns, head)
    achieved = algo / lb_avg_s / 1e9
    traffic = measured_traffic(head) if args.n == 256 else None
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
                        f"f0=1e-6; populations stored as {STORE_DESC.get(head, head)}",
            "sites": ns, "cells": len(cfg["X"]), "precision": head,
            "fluid_sites": round(r["n_fluid"]),
            "fluid_mlups": round(r["n_fluid"] * args.steps / r["seconds"] / 1e6, 1),
            "kernel_ms_per_step": {k: round(v[0] / max(v[1], 1), 4) for k, v in r["kernel_times"].items()},
            "kernel_pass": f"{args.kernel_steps} steps after the timed region, every kernel in sequence on the "
                           "handle's stream, HIP events around each launch",
            "paper_context": "the paper reports no absolute throughput; its only performance figures are parallel "
                             "efficiencies of its CPU code on IBM BlueGene/P (combined LB + particles 95.7 % at "
                             "16,384 and 85.2 % at 32,768 cores relative to 2,048; pure LB 98.1 % at 32,768) on a "
                             "1024^2 x 2048 lattice with 4.1e6 cells (Sec. IV)",
            "concurrency": "serial" if args.serial else "cell list + potentials and momentum exchange on two side "
                                                        "streams beside the lattice kernels, joined before the integrator",
        },
        "roofline": {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None if traffic is None else round(traffic / lb_avg_s / 1e9, 1),
            "kernel": "lb_kernel_tau1", "algorithmic_bytes_per_launch": algo,
            "hbm_bytes_per_launch": traffic,
            "avg_launch_ms": round(lb_avg_s * 1e3, 5),
        },
    }
    # the other storage precisions of the same workload: FP32, and FP16
    # deviations stored per direction alone
    for other in ("p32", "pmx16"):
        if other not in results or other == head:
            continue
        ro = results[other]
        line["config"][f"{other}_mlups"] = round(ns * args.steps / ro["seconds"] / 1e6, 1)
        line["config"][f"{other}_ms_per_step"] = round(ro["seconds"] * 1e3 / args.steps, 4)
        lo, co = ro["kernel_times"].get("lb", (float("nan"), 1))
        line["config"][f"{other}_lb_ms"] = round(lo / max(co, 1), 5)
        line["config"][f"{other}_lb_frac"] = round(lb_algorithmic_bytes(ro["n_fluid"], ns, other) /
                                                   (lo / max(co, 1) / 1e3) / 1e9 / HBM_PEAK_GBS, 4)
    if not args.no_error:
        line["config"]["error_vs_p64_64cube"] = error_report_64()
    if not args.no_batch:
        line["config"]["batch"] = batch_leg(steps=args.batch_steps)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(cfg, args.cpu_steps)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
