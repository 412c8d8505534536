"""What the learned closure gains over the plain method without it: on
held-out channels the ensemble answers orders of magnitude faster, its
accepted answers stay close to the plain method's, and the inputs it is
unsure of fall back to the plain method (so those answers are the plain
method's exactly).  Small channels and short runs keep it quick; the full
recipe (64 batches of 64 channels, 2000 steps) is the closure's command line."""
import time

import numpy as np
import pytest

import synth
from parity_util import say

pytestmark = pytest.mark.gpu

STEPS = 800


def small(seed):
    return synth.config4(seed=seed, n_channels=32, w_range=(14, 32), lz_range=(16, 40))


def test_closure_gain_and_fallback():
    from paper_1005_2594_amd import closure
    X, mu, secs = closure.dataset(range(300, 308), STEPS, make=small, log=say)
    Xt, mut, secs_t = closure.dataset([310], STEPS, make=small, log=say)
    assert np.isfinite(mu).mean() > 0.9
    net, info = closure.train_ensemble(X, mu, members=5, epochs=2000, lr=2e-3)
    say("train", info)
    ev = closure.evaluate(net, Xt, mut, threshold=0.05)
    say("held-out", ev)
    assert info["final_loss"] < 0.5 * info["first_loss"]
    # the ensemble has learned the trend: on held-out channels it beats the
    # best constant answer (the training median) by a clear margin; the rest
    # of the scatter is the random cell arrangement, which the three inputs
    # do not see
    ok = np.isfinite(mut)
    const = np.median(mu[np.isfinite(mu)])
    e_const = np.median(np.abs(const - mut[ok]) / mut[ok])
    say(f"median error: ensemble {ev['median_rel_err_all']:.3f}, constant {e_const:.3f}")
    assert ev["median_rel_err_all"] < 0.7 * e_const
    # ensemble answers for the held-out channels, falling back where unsure
    chans = small(310)
    t0 = time.perf_counter()
    mu_c, plain = closure.predict_or_simulate(net, chans, threshold=0.05, steps=STEPS)
    t_closure = time.perf_counter() - t0
    ok = np.isfinite(mut)
    acc = ok & ~plain
    err = np.abs(mu_c[acc] - mut[acc]) / mut[acc]
    say(f"accepted {acc.sum()} of {ok.sum()}, median err {np.median(err) if acc.any() else None}, "
        f"closure {t_closure:.2f} s vs plain {secs_t:.2f} s")
    # fallback answers are the plain method's own numbers (same seeds, same kernels)
    fb = ok & plain
    if fb.any():
        assert np.allclose(mu_c[fb], mut[fb], rtol=1e-6)
    if acc.any():
        assert np.median(err) < 0.25
    # per answered input the surrogate costs a tiny fraction of a plain run
    Q = np.repeat(Xt, 1000, axis=0).astype(np.float32)
    t0 = time.perf_counter()
    net.predict(Q)
    per_q = (time.perf_counter() - t0) / len(Q)
    per_plain = secs_t / len(chans)
    say(f"seconds per answer: surrogate {per_q:.2e}, plain {per_plain:.2e}")
    assert per_q < 1e-3 * per_plain
    net.close()
