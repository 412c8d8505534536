"""Learned closure for the apparent viscosity of the batched channels.

The plain method (the batched ensemble of wall-bounded channels, apparent
viscosity from the mean mixture velocity) produces samples
(hematocrit, log shear rate, width / R_perp) -> mu_rel; an ensemble of small
networks (``Mlp``, trained on the device) maps new inputs to mu_rel, and any
input on which the members disagree by more than a threshold (relative
spread) is answered by the plain method instead.

Shear rate: the wall shear rate of the plasma's plane Poiseuille flow under
the same body force, g N_f / (2 nu), N_f = W - 2 fluid planes, nu = (2 tau - 1)/6.

Command line (writes .npz / .json files):
    python -m paper_1005_2594_amd.closure gen --seeds 100-163 --out train.npz
    python -m paper_1005_2594_amd.closure fit --train train.npz --test test.npz --out report.json
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

from .cgb import MLP_BATCH, MLP_PARAMS, Batch, CgbError, Mlp

FEATURES = ("hematocrit", "log wall shear rate", "width / R_perp")


def features(ch) -> np.ndarray:
    p = ch["params"]
    nu = (2.0 * p["tau"] - 1.0) / 6.0
    nf = p["ny"] - 2
    g = p["g"][2]
    return np.array([ch["hematocrit"], math.log(g * nf / (2.0 * nu)), p["ny"] / p["R_perp"]])


def simulate(chans, steps=2000, precision="pmx16", autotune=True):
    """Plain method on a list of channels: mu_rel over steps steps/2 .. steps-1
    (NaN for a channel that became unstable) and the seconds it took."""
    t0 = time.perf_counter()
    b = Batch([c["params"] for c in chans], precision=precision)
    try:
        for s, c in zip(b.channels, chans):
            s.set_particles(c["X"], c["q"])
            s.init_fluid()
        if autotune:
            b.autotune(reps=3)
        b.track(steps)
        b.capture(2)
        b.run(steps)
        try:
            b.sync()
            mu = b.mu_rel(first=steps // 2)
        except CgbError:
            mu = np.full(len(chans), np.nan)
            for k, s in enumerate(b.channels):
                try:
                    s.sync()
                    mu[k] = s.mu_rel(first=steps // 2)
                except CgbError:
                    pass
    finally:
        b.close()
    return mu, time.perf_counter() - t0


def dataset(seeds, steps=2000, make=None, log=print):
    """(X, mu, seconds) from one batch of channels per seed (make(seed) gives
    the channels; the uneven-channel recipe by default)."""
    if make is None:
        import synth
        make = lambda s: synth.config4(seed=s)  # noqa: E731
    X, M, secs = [], [], 0.0
    for s in seeds:
        chans = make(s)
        mu, dt = simulate(chans, steps)
        secs += dt
        X.append(np.stack([features(c) for c in chans]))
        M.append(mu)
        log(f"# seed {s}: {len(chans)} channels, {dt:.1f} s, unstable {int(np.isnan(mu).sum())}")
    return np.concatenate(X), np.concatenate(M), secs


def he_init(rng, members):
    """He-uniform weights, zero biases, in the parameter order of the network."""
    out = np.zeros((members, MLP_PARAMS))
    for m in range(members):
        k = 0
        for shape, fan_in, is_w in (((64, 3), 3, True), ((64,), 0, False), ((64, 64), 64, True), ((64,), 0, False),
                                    ((64,), 64, True), ((1,), 0, False)):
            n = int(np.prod(shape))
            if is_w:
                lim = math.sqrt(6.0 / fan_in)
                out[m, k:k + n] = rng.uniform(-lim, lim, n)
            k += n
    return out


def train_ensemble(X, mu, members=5, epochs=400, lr=2e-3, seed=0):
    """Members differ in their initial weights and in the order of their
    mini-batches (the random numbers are drawn here and passed in)."""
    ok = np.isfinite(mu) & (mu > 0)
    X, mu = X[ok], mu[ok]
    rng = np.random.default_rng(seed)
    net = Mlp(members)
    net.set_params(he_init(rng, members))
    lm = np.log(mu)
    net.set_norm(X.mean(0), np.maximum(X.std(0), 1e-6), float(lm.mean()), float(max(lm.std(), 1e-6)))
    steps = max(1, epochs * len(X) // MLP_BATCH)
    idx = np.stack([np.concatenate([rng.permutation(len(X)) for _ in range(steps * MLP_BATCH // len(X) + 1)])
                    [:steps * MLP_BATCH].reshape(steps, MLP_BATCH) for _ in range(members)]).astype(np.int32)
    t0 = time.perf_counter()
    loss = net.train(X, mu, idx, lr)
    return net, dict(steps=steps, seconds=time.perf_counter() - t0, final_loss=float(loss[:, -50:].mean()),
                     first_loss=float(loss[:, :10].mean()), samples=int(len(X)))


def evaluate(net, X, mu, threshold=0.05):
    """Surrogate against the plain method on held-out samples: error of the
    accepted predictions (spread <= threshold) and the fallback fraction."""
    ok = np.isfinite(mu)
    mean, spread = net.predict(X[ok])
    err = np.abs(mean - mu[ok]) / mu[ok]
    acc = spread <= threshold
    return dict(samples=int(ok.sum()), accepted=int(acc.sum()), fallback_fraction=float(1 - acc.mean()),
                median_rel_err_all=float(np.median(err)), median_rel_err_accepted=float(np.median(err[acc])) if acc.any() else None,
                p90_rel_err_accepted=float(np.quantile(err[acc], 0.9)) if acc.any() else None,
                max_rel_err_accepted=float(err[acc].max()) if acc.any() else None,
                median_spread=float(np.median(spread)))


def local_noise(Xtr, mutr, X, k=8):
    """Scatter of the plain method's own answers near each query: the sample
    standard deviation of ln mu over the k training samples nearest to it in
    standardised inputs.  Where the plain method's answers scatter, no
    surrogate can be trusted, whatever its members agree on."""
    ok = np.isfinite(mutr) & (mutr > 0)
    Xtr, lm = Xtr[ok], np.log(mutr[ok])
    m, sd = Xtr.mean(0), np.maximum(Xtr.std(0), 1e-12)
    A, B = (Xtr - m) / sd, (np.asarray(X, dtype=np.float64) - m) / sd
    d2 = (B * B).sum(1)[:, None] + (A * A).sum(1)[None, :] - 2.0 * B @ A.T
    nn = np.argpartition(d2, k, axis=1)[:, :k]
    return lm[nn].std(axis=1, ddof=1)


def fallback_analysis(net, X, mu, Xtr=None, mutr=None, thresholds=(0.05, 0.03, 0.02, 0.01, 0.005),
                      noise_thresholds=(0.3, 0.2, 0.15, 0.1)):
    """How well the members' spread predicts the error on held-out samples:
    the rank correlation of spread and error, and for each spread threshold
    the fraction sent to the plain method and the error of the rest; the
    inputs of the worst answers."""
    ok = np.isfinite(mu)
    X, mu = X[ok], mu[ok]
    mean, spread = net.predict(X)
    err = np.abs(mean - mu) / mu
    rank = lambda v: np.argsort(np.argsort(v)).astype(np.float64)  # noqa: E731
    rs, re = rank(spread), rank(err)
    rho = float(np.corrcoef(rs, re)[0, 1])
    sweep = []
    for t in thresholds:
        acc = spread <= t
        sweep.append(dict(threshold=t, fallback_fraction=float(1 - acc.mean()),
                          p90_rel_err_accepted=float(np.quantile(err[acc], 0.9)) if acc.any() else None,
                          max_rel_err_accepted=float(err[acc].max()) if acc.any() else None))
    worst = np.argsort(err)[::-1][:5]
    out = dict(spearman_spread_error=rho, sweep=sweep,
               worst=[dict(inputs=[float(v) for v in X[k]], mu=float(mu[k]), predicted=float(mean[k]),
                           rel_err=float(err[k]), spread=float(spread[k])) for k in worst])
    if Xtr is not None:
        # the alternative criterion: the local scatter of the plain method
        nz = local_noise(Xtr, mutr, X)
        out["spearman_local_noise_error"] = float(np.corrcoef(rank(nz), re)[0, 1])
        out["local_noise_sweep"] = []
        for t in noise_thresholds:
            acc = (nz <= t) & (spread <= 0.05)
            out["local_noise_sweep"].append(dict(
                threshold=t, fallback_fraction=float(1 - acc.mean()),
                median_rel_err_accepted=float(np.median(err[acc])) if acc.any() else None,
                p90_rel_err_accepted=float(np.quantile(err[acc], 0.9)) if acc.any() else None,
                max_rel_err_accepted=float(err[acc].max()) if acc.any() else None))
        for w, k in zip(out["worst"], worst):
            w["local_noise"] = float(nz[k])
    return out


def predict_or_simulate(net, chans, threshold=0.05, steps=2000, train=None, noise_threshold=None):
    """mu_rel for channels: the ensemble mean where the members agree within
    threshold (and, given the training samples train = (X, mu) and
    noise_threshold, where the plain method's own answers near the query
    scatter by at most noise_threshold in ln mu), the plain method
    elsewhere.  Returns (mu, used_plain mask)."""
    X = np.stack([features(c) for c in chans]).astype(np.float32)
    mean, spread = net.predict(X)
    mu = mean.astype(np.float64)
    plain = spread > threshold
    if train is not None and noise_threshold is not None:
        plain |= local_noise(train[0], train[1], X) > noise_threshold
    if plain.any():
        sub = [c for c, f in zip(chans, plain) if f]
        mu_p, _ = simulate(sub, steps)
        mu[plain] = mu_p
    return mu, plain


def time_inference(net, X, n=1 << 20, seed=0, reps=5):
    """Ensemble inference on n points uniform over the box of X, inputs and
    outputs resident on the device; milliseconds per call (HIP events)."""
    import torch
    rng = np.random.default_rng(seed)
    lo, hi = X.min(0), X.max(0)
    q = torch.from_numpy(rng.uniform(lo, hi, (n, 3)).astype(np.float32)).cuda()
    mean = torch.empty(n, device="cuda")
    spread = torch.empty(n, device="cuda")
    # a stream of its own: handle 0 (torch's default stream) would mean the
    # network's own stream to the library, not the stream the events are on
    st = torch.cuda.Stream()
    torch.cuda.synchronize()
    net.predict_device(n, q.data_ptr(), mean.data_ptr(), spread.data_ptr(), st.cuda_stream)
    st.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        net.predict_device(n, q.data_ptr(), mean.data_ptr(), spread.data_ptr(), st.cuda_stream)
    e1.record(st)
    st.synchronize()
    ms = e0.elapsed_time(e1) / reps
    flop = 5 * n * 2 * (3 * 64 + 64 * 64 + 64)
    return dict(points=n, ms=ms, tflops=flop / (ms * 1e-3) / 1e12,
                fallback_fraction=float((spread > 0.05).float().mean().item()))


def _seeds(s):
    a, b = s.split("-") if "-" in s else (s, s)
    return list(range(int(a), int(b) + 1))


def main(argv=None):
    ap = argparse.ArgumentParser(prog="python -m paper_1005_2594_amd.closure")
    sub = ap.add_subparsers(dest="cmd", required=True)
    g = sub.add_parser("gen")
    g.add_argument("--seeds", required=True)
    g.add_argument("--steps", type=int, default=2000)
    g.add_argument("--out", required=True)
    f = sub.add_parser("fit")
    f.add_argument("--train", nargs="+", required=True)
    f.add_argument("--test", nargs="+", required=True)
    f.add_argument("--members", type=int, default=5)
    f.add_argument("--epochs", type=int, default=400)
    f.add_argument("--lr", type=float, default=2e-3)
    f.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    if a.cmd == "gen":
        X, mu, secs = dataset(_seeds(a.seeds), a.steps)
        np.savez(a.out, X=X, mu=mu, seconds=secs, steps=a.steps)
        print(json.dumps({"samples": len(mu), "unstable": int(np.isnan(mu).sum()), "seconds": secs}), flush=True)
        return 0
    load = lambda paths: [np.load(p) for p in paths]  # noqa: E731
    tr, te = load(a.train), load(a.test)
    Xtr = np.concatenate([d["X"] for d in tr]); mtr = np.concatenate([d["mu"] for d in tr])
    Xte = np.concatenate([d["X"] for d in te]); mte = np.concatenate([d["mu"] for d in te])
    plain_s = sum(float(d["seconds"]) for d in tr + te) / (len(mtr) + len(mte))
    net, info = train_ensemble(Xtr, mtr, a.members, a.epochs, a.lr)
    rep = dict(features=FEATURES, train=info, test=evaluate(net, Xte, mte), inference=time_inference(net, Xtr),
               fallback=fallback_analysis(net, Xte, mte, Xtr, mtr), plain_seconds_per_sample=plain_s)
    rep["gain"] = dict(plain_seconds_per_sample=plain_s,
                       surrogate_seconds_per_sample=rep["inference"]["ms"] * 1e-3 / rep["inference"]["points"])
    with open(a.out, "w") as fh:
        json.dump(rep, fh, indent=1)
    print(json.dumps(rep), flush=True)
    net.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
