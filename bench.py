"""Throughput of the coupled LB / rigid-ellipsoid time step on one MI355X.

Workload: 256^3 periodic box, Kolmogorov body force f_z = 1e-6 sin(2 pi y/256),
hematocrit 0.4 (256,337 cells with half axes (2.5, 1.0)), tau = 1.  The
headline number is the mixed-precision path: the deviations n*_r - w_r rho0
stored in FP16 as a per-node part (the density deviation) plus per-direction
residuals, FP32 collision, link momenta (Eq. 12) and per-cell sums in FP64
from the decoded populations, FP64 integration.  Beside it: FP16 deviations stored per
direction alone (the same storage size, ~8x the velocity error) and the
FP32-storage path.  One step = every kernel of the time
step (rasterisation, cover/uncover, fused LB, momentum-exchange reduction,
cell list, pair and wall forces, integration, the per-step mixture record of
the apparent viscosity).  Inputs are resident in HBM before the timed region.

Also reported (in "config"): the error of every path against the FP64
oracle on the 64^3 companion workload, stepped in lockstep on the host cores,
with the oracle's own response to perturbed inputs beside it; the
whole-step effective and counter bandwidths; the batched ensemble of 64
uneven channels (one launch per kernel for all channels, one replayed HIP
graph, LB tiles tuned on the fused launch, apparent viscosity per channel);
the vessel bifurcation with stenosis in the dense and the indexed layouts;
the paper's 1024^2 x 2048 system with 4.1e6 cells in the large-lattice
layout (when the device has the memory free); and the oracle on the host
cores ("cpu_baseline").

Prints one JSON line.  --gpus N > 1 exits: the benchmark runs on one GPU.
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
HEAD = "pmx16s"
STORE_DESC = {
    "pmx16s": "FP16 deviations n*_r - w_r rho0 split into a per-node FP16 density part and per-direction "
              "FP16 residuals (2 B per population), FP32 collision (pmx16s)",
    "pmx16": "FP16 deviations (n*_r - w_r rho0)/w_r per direction (2 B per population), FP32 collision (pmx16)",
    "p32": "FP32 deviations, FP32 collision (p32)",
}


def lb_algorithmic_bytes(n_fluid: float, n_sites: int, prec: str) -> float:
    """Bytes one LB launch must move: for every fluid node 19 populations read
    and written plus its density deviation written and read (the density in
    the moving-boundary term of Eq. 10), and one 4-byte flag word per site."""
    s = STORE_BYTES[prec]
    return n_fluid * (2 * 19 * s + 2 * s) + 4.0 * n_sites


CSRC = os.path.join(ROOT, "paper_1005_2594_amd", "csrc")


def csrc_sha256() -> str:
    """Hash of every HIP source of the library (the step's kernels)."""
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".h")):
            h.update(name.encode())
            h.update(open(os.path.join(CSRC, name), "rb").read())
    return h.hexdigest()


def step_algorithmic_bytes(n_fluid: float, n_sites: int, n_cells: int, prec: str) -> float:
    """Bytes one whole step must move: the LB's (populations of every fluid
    node read and written, density, flags) and about 200 bytes per cell (its
    state read and written, forces); link-level data stays on chip."""
    return lb_algorithmic_bytes(n_fluid, n_sites, prec) + 200.0 * n_cells


def counter_summary(prec: str):
    """The committed rocprofv3 counter summary of the 256^3 workload
    (profiles/step_traffic_<prec>_256.txt) as a dict, or None when it was
    taken on other kernel sources than these."""
    path = os.path.join(ROOT, "profiles", f"step_traffic_{prec}_256.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    return kv if kv.get("csrc_sha256") == csrc_sha256() else None


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
    # the per-step mixture record (the apparent-viscosity observable) is part
    # of the timed step: every step below records it
    # (steps eager + 2 warm replays + steps timed; the kernel pass after them
    # is not stored)
    cap = 2 * steps + 2
    sim.track(cap)
    # eager: one launch per kernel
    t0 = time.perf_counter()
    sim.step(steps)
    sim.sync()
    eager_s = time.perf_counter() - t0
    # graph replay of a two-step capture (cgb_capture / cgb_replay): the
    # same kernels, launched as one sequence
    sim.capture(2)
    sim.replay(2)
    sim.sync()
    t0 = time.perf_counter()
    sim.replay(steps - steps % 2)
    if steps % 2:
        sim.step(1)
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
    # apparent viscosity over the timed steps (the last `steps` rows of the record)
    mu = None
    if len(sim.get_track()) == cap:
        try:
            mu = sim.mu_rel(first=steps + 2)
        except Exception:  # a driving with no estimator
            mu = None
    return dict(seconds=t1 - t0, eager_seconds=eager_s, n_fluid=nf, kernel_times=kt, obs=ob, sim=sim, mu_rel=mu)


def error_report_64(seed=3, horizons=(100, 250, 500)):
    """The GPU paths (FP64, FP32, FP16 per direction, split FP16) against the
    FP64 oracle on the 64^3 companion workload (same cell density, 4,005
    cells), all stepped in lockstep: the oracle on the host cores, so this
    is also the oracle's full 64^3 run of the CPU baseline.  At each horizon:
    relative L2 error of the fluid velocity (nodes fluid in both), RMS error
    of the cell positions, relative L2 error of the cell velocities; every
    step: the number of nodes whose owner differs from the oracle's (a node
    covered or freed one step apart), accumulated.  Beside them, from
    tests/golden/conditioning_64cube.json (written by the oracle alone): the
    oracle's own response to relative perturbations of the cell positions,
    which puts the errors in proportion.  Apparent viscosity: Kolmogorov
    estimator over the last half of the run."""
    from oracle import oracle as O
    from paper_1005_2594_amd import Sim
    cfg = synth.config3_companion(seed=seed)
    p = cfg["params"]
    precs = ("p64", "p32", "pmx16", "pmx16s")
    sims = {q: Sim(p, precision=q) for q in precs}
    for s in sims.values():
        s.set_particles(cfg["X"], cfg["q"])
        s.init_fluid()
        s.track(horizons[-1])
    o = O.Oracle(p)
    o.set_particles(cfg["X"], cfg["q"])
    o.init_fluid()
    n_box = p["nx"]
    res = {q: {} for q in precs}
    mism = {q: 0 for q in precs}
    first = {q: None for q in precs}
    A_orc = np.empty(horizons[-1])
    t_orc = 0.0
    for t in range(1, horizons[-1] + 1):
        t0 = time.perf_counter()
        o.step(1)
        t_orc += time.perf_counter() - t0
        A_orc[t - 1] = o.mixture()[0]
        own_o = o.owner()
        for q, s in sims.items():
            s.step(1)
            d = int((s.owner() != own_o).sum())
            if d and first[q] is None:
                first[q] = t
            mism[q] += d
        if t not in horizons:
            continue
        _, u_o = o.fields()
        X_o, _, V_o, _ = o.particles()
        for q, s in sims.items():
            own = s.owner()
            _, u = s.fields()
            X, _, V, _ = s.particles()
            m = (own == -1) & (own_o == -1)
            dX = X - X_o
            dX -= n_box * np.round(dX / n_box)
            res[q][f"step{t}"] = dict(
                rel_l2_u=float(np.linalg.norm(u[m] - u_o[m]) / np.linalg.norm(u_o[m])),
                pos_rms=float(np.sqrt(np.mean(np.sum(dX * dX, axis=1)))),
                rel_l2_V=float(np.linalg.norm(V - V_o) / np.linalg.norm(V_o)),
                owner_mismatch_node_steps=mism[q])
    first_step = horizons[-1] // 2
    mu_o = O.mu_rel_kolmogorov(A_orc, p["f0"], p["rho0"], p["ny"], first_step)
    for q, s in sims.items():
        mu = s.mu_rel(first=first_step)
        res[q]["mu_rel"] = mu
        res[q]["mu_rel_rel_err"] = abs(mu - mu_o) / abs(mu_o)
        res[q]["first_owner_mismatch_step"] = first[q]
        s.close()
    res["oracle_mu_rel"] = mu_o
    res["mu_rel_window"] = [first_step, horizons[-1] - 1]
    ns = p["nx"] * p["ny"] * p["nz"]
    res["oracle_run"] = {"steps": horizons[-1], "seconds": round(t_orc, 1), "cores": O.num_threads(),
                         "mlups": round(ns * horizons[-1] / t_orc / 1e6, 3)}
    cond = os.path.join(ROOT, "tests", "golden", "conditioning_64cube.json")
    if os.path.exists(cond):
        c = json.load(open(cond))
        res["oracle_conditioning"] = {
            "source": "tests/golden/conditioning_64cube.json (the oracle against itself with the cell x "
                      "coordinates scaled by 1 + eps)",
            **{f"step{h}": [{k: r[k] for k in ("eps", "rel_l2_u", "pos_rms", "owner_mismatch_node_steps")}
                            for r in c["steps"][str(h)]] for h in horizons if str(h) in c["steps"]}}
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
    tiles = b.autotune(reps=20)
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


def paper_scale_leg(steps=20, warmup=3, kernel_steps=5, prec="pmx16s"):
    """The paper's largest system (Sec. IV: 1024^2 x 2048 sites, 4.1e6 cells)
    on this one GPU, in the large-lattice layout (64-bit lane addresses, cell
    nodes' momenta in their own unused population slots)."""
    import torch
    free, total = torch.cuda.mem_get_info()
    if free < 250e9:
        return {"skipped": f"needs about 250 GB of free device memory, {free / 1e9:.0f} GB free"}
    cfg = synth.paper_scale_suspension()
    t0 = time.perf_counter()
    r = run_gpu(cfg, prec, steps, warmup, kernel_steps=kernel_steps)
    sim = r["sim"]
    nx, ny, nz = synth.PAPER_SCALE
    ns = nx * ny * nz
    out = {
        "workload": cfg["name"] + f", Ht 0.05, tau=1, f0=1e-6; {prec}, large-lattice layout",
        "sites": ns, "cells": len(cfg["X"]), "steps": steps,
        "ms_per_step": round(r["seconds"] / steps * 1e3, 3),
        "mlups": round(ns * steps / r["seconds"] / 1e6, 1),
        "fluid_mlups": round(r["n_fluid"] * steps / r["seconds"] / 1e6, 1),
        "device_bytes": int(sim.device_bytes),
        "device_total_bytes": int(total),
        "kernel_ms_per_step": {k: round(t / max(c, 1), 4) for k, (t, c) in r["kernel_times"].items()},
        "wall_seconds_with_setup": round(time.perf_counter() - t0, 1),
    }
    sim.close()
    print(f"# paper scale: {out['ms_per_step']:.2f} ms/step, {out['mlups']:.0f} MLUPS, "
          f"{out['device_bytes'] / 1e9:.1f} GB", flush=True)
    return out


def vessel_leg(steps=200, warmup=10, prec="pmx16s"):
    """The bifurcation workload of Sec. IV at a size that fills the GPU, in
    the dense and the indexed layout (results identical, checked by the GPU
    tests): time per step, rate per site and per vessel node, device memory,
    and the flow fraction of the constricted branch at the end."""
    from paper_1005_2594_amd import Sim
    cfg = synth.vessel_network()
    m, p = cfg["mask"], cfg["params"]
    L_, ny, nx = m.shape
    ns, nc = m.size, int((1 - m).sum())
    out = {"workload": cfg["name"] + f", entrance force, {prec}", "sites": ns, "vessel_nodes": nc,
           "cells": len(cfg["X"]), "steps": steps}
    xs = np.arange(nx)
    cx = (nx - 1) / 2.0
    for idx in (0, 1):
        g = Sim(dict(p, indexed=idx), m, precision=prec)
        g.set_particles(cfg["X"], cfg["q"])
        g.init_fluid()
        g.step(warmup)
        g.sync()
        t0 = time.perf_counter()
        g.step(steps)
        g.sync()
        dt = time.perf_counter() - t0
        u = g.mixture_box((0, 0, L_ // 2), (nx, ny, 1))[0]
        q_hat = float(u[:, xs > cx, 2].sum() / u[:, xs != cx, 2].sum())
        key = "indexed" if idx else "dense"
        out[key] = {"ms_per_step": round(dt / steps * 1e3, 4), "mlups_sites": round(ns * steps / dt / 1e6, 1),
                    "mlups_vessel_nodes": round(nc * steps / dt / 1e6, 1), "device_bytes": int(g.device_bytes),
                    "flow_fraction_constricted": round(q_hat, 6)}
        g.close()
    print(f"# vessels: dense {out['dense']['ms_per_step']} ms, indexed {out['indexed']['ms_per_step']} ms per step",
          flush=True)
    return out


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
    cores = O.num_threads()
    out = {"value": round(ns * steps / dt / 1e6, 3), "unit": "MLUPS", "cores": cores, "kind": "oracle",
           "sample": f"{steps} steps of the 256^3 Ht=0.4 workload in FP64 (all sites), set-up excluded",
           "seconds": round(dt, 2)}
    # the 64^3 companion on one core and on all of them, and the host CPU
    c64 = synth.config3_companion()
    rates = {}
    for nt in (1, cores):
        O.set_num_threads(nt)
        o = O.Oracle(c64["params"])
        o.set_particles(c64["X"], c64["q"])
        o.init_fluid()
        k = 5 if nt == 1 else 20
        t0 = time.perf_counter()
        o.step(k)
        rates[nt] = 64 ** 3 * k / (time.perf_counter() - t0) / 1e6
    O.set_num_threads(cores)
    # the 24 x 24 x 48 channel with 20 cells (P64 parity workload), 100 steps
    c1 = synth.config1()
    o = O.Oracle(c1["params"], c1.get("walls"))
    o.set_particles(c1["X"], c1["q"])
    o.init_fluid()
    t0 = time.perf_counter()
    o.step(100)
    out["channel_24x24x48_100_steps_seconds"] = round(time.perf_counter() - t0, 3)
    out["mlups_64cube_1core"] = round(rates[1], 3)
    out[f"mlups_64cube_{cores}cores"] = round(rates[cores], 3)
    cpu = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    out["cpu_model"] = cpu
    return out


def copy_ceiling(nbytes=1 << 31, reps=10):
    """The bandwidth a plain device-to-device copy reaches on this GPU (bytes
    read plus bytes written per second), the practical ceiling beside the
    vendor peak: HIP events on torch's stream, around reps copies."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(2):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    s = e0.elapsed_time(e1) / 1e3
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * nbytes * reps / s / 1e9


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
    ap.add_argument("--no-paper-scale", action="store_true")
    ap.add_argument("--no-vessels", action="store_true")
    ap.add_argument("--only", default=None, help="run only this precision (profiling)")
    ap.add_argument("--kernel-steps", type=int, default=50, help="steps of the per-kernel timing pass")
    ap.add_argument("--serial", action="store_true", help="every kernel in sequence in the timed region too")
    ap.add_argument("--copy-calibrate", action="store_true", help="also run a copy of known size (counter scaling)")
    ap.add_argument("--batch-only", action="store_true",
                    help="run only the 64-channel ensemble and print its record (profiling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; runs on several GPUs are not supported",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)
    if args.copy_calibrate:
        copy_calibration()
    if args.batch_only:
        r = batch_leg(steps=args.batch_steps)
        print(json.dumps({k: v for k, v in r.items() if k != "mu_rel"}), flush=True)
        return

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
    cs = counter_summary(head) if args.n == 256 else None
    traffic = None if cs is None else float(cs["lb_fetch_bytes_per_launch"]) + float(cs["lb_write_bytes_per_launch"])
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
            "concurrency": "serial" if args.serial else "cell list + potentials on a side stream beside the lattice "
                                                        "kernels, joined before the integrator",
            "launch": "timed steps replayed from a HIP graph of a two-step capture (cgb_capture / cgb_replay)",
            "observables": "the per-step mixture record (Kolmogorov apparent viscosity) is taken in every timed "
                           "step; mu_rel over the timed steps: " + (f"{r['mu_rel']:.4f}" if r["mu_rel"] else "n/a") +
                           " (a spin-up transient: at 256^3 the shear flow takes ~1e4 steps to develop)",
            "eager_ms_per_step": round(r["eager_seconds"] * 1e3 / args.steps, 4),
            "eager_mlups": round(ns * args.steps / r["eager_seconds"] / 1e6, 1),
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
    # the practical ceiling: a plain copy's bandwidth on this GPU
    ceil_gbs = copy_ceiling()
    line["roofline"]["copy_ceiling_gbs"] = round(ceil_gbs, 1)
    line["roofline"]["frac_of_copy_ceiling"] = round(achieved / ceil_gbs, 4)
    # the other storage precisions of the same workload: FP32, and FP16
    # deviations stored per direction alone
    # the whole step: algorithmic bytes per step over the step time, and the
    # counter bytes of every kernel of a step over the step time
    sa = step_algorithmic_bytes(r["n_fluid"], ns, len(cfg["X"]), head)
    step_s = r["seconds"] / args.steps
    line["config"]["step_algorithmic_bytes"] = round(sa)
    line["config"]["step_effective_gbs"] = round(sa / step_s / 1e9, 1)
    line["config"]["step_effective_frac"] = round(sa / step_s / 1e9 / HBM_PEAK_GBS, 4)
    if cs is not None:
        sb = float(cs["step_fetch_bytes"]) + float(cs["step_write_bytes"])
        line["config"]["step_counter_bytes"] = round(sb)
        line["config"]["step_counter_gbs"] = round(sb / step_s / 1e9, 1)
        line["config"]["step_counter_frac"] = round(sb / step_s / 1e9 / HBM_PEAK_GBS, 4)
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
        line["config"]["error_vs_oracle_64cube"] = error_report_64()
    if not args.no_batch:
        line["config"]["batch"] = batch_leg(steps=args.batch_steps)
    if not args.no_vessels:
        line["config"]["vessels"] = vessel_leg()
    if not args.no_paper_scale:
        line["config"]["paper_scale"] = paper_scale_leg()
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(cfg, args.cpu_steps)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
