"""The closure network on the device against the FP64 reference: forward
outputs, batch gradients and the Adam step, then training and the ensemble
spread."""
import numpy as np
import pytest

from oracle import mlp_oracle as M
from parity_util import say

pytestmark = pytest.mark.gpu


def _params(rng, members):
    p = M.init_params(rng, members)
    for m in range(members):
        d = M.unpack(p[m])
        d["b1"][:] = 0.1 * rng.standard_normal(64)
        d["b2"][:] = 0.1 * rng.standard_normal(64)
        d["b3"][:] = 0.2
        p[m] = M.pack(d)
    return p.astype(np.float32).astype(np.float64)


def test_forward_matches_oracle():
    from paper_1005_2594_amd import Mlp
    rng = np.random.default_rng(10)
    p = _params(rng, 5)
    x = rng.standard_normal((1003, 3)).astype(np.float32)  # ragged: not a multiple of 16
    net = Mlp(5)
    net.set_params(p)
    y = net.forward(x)
    for m in range(5):
        yo = M.forward(p[m], x.astype(np.float64), bf16_ops=True)
        e = np.max(np.abs(y[m] - yo)) / np.max(np.abs(yo))
        ex = np.max(np.abs(y[m] - M.forward(p[m], x.astype(np.float64)))) / np.max(np.abs(yo))
        say(f"member {m}: vs bf16 reference {e:.2e}, vs exact FP64 {ex:.2e}")
        assert e < 2e-5
        assert ex < 3e-2
    net.close()


def test_forward_full_batch_matches_oracle_on_samples():
    # the inference workload: 2^20 query points through all five members in
    # one call; 4096 sampled outputs per member against the reference
    from paper_1005_2594_amd import Mlp
    rng = np.random.default_rng(12)
    p = _params(rng, 5)
    n = 1 << 20
    x = rng.standard_normal((n, 3)).astype(np.float32)
    net = Mlp(5)
    net.set_params(p)
    y = net.forward(x)
    assert y.shape == (5, n) and np.all(np.isfinite(y))
    idx = np.sort(rng.choice(n, 4096, replace=False))
    idx[0], idx[-1] = 0, n - 1  # first and last rows included
    for m in range(5):
        xs = x[idx].astype(np.float64)
        yo, it = M.forward(p[m], xs, bf16_ops=True, keep=True)
        scale = np.max(np.abs(yo))
        err = np.abs(y[m, idx] - yo)
        # the device sums in FP32 in another order, so where a first-layer
        # activation lies at a BF16 rounding boundary the two sides may round
        # it to neighbouring BF16 values, one unit in the last place apart;
        # to first order that moves the output by dy/dh1_k times that unit.
        # Bound: every activation of the point flipped, plus FP32 rounding
        dydh = (it["W3"] * M.dsilu(it["z2"])) @ it["W2"]
        ulp = np.ldexp(1.0, np.frexp(it["h1"])[1] - 8)
        bound = np.sum(np.abs(dydh) * ulp, axis=1) + 2e-5 * scale
        ex = np.max(np.abs(y[m, idx] - M.forward(p[m], xs))) / scale
        ok = float(np.mean(err < 2e-5 * scale))
        say(f"member {m}, 2^20 points, 4096 sampled: vs bf16 reference max {err.max() / scale:.2e} "
            f"(of the flip bound {np.max(err / bound):.2f}), share within 2e-5 {ok:.4f}; vs exact FP64 {ex:.2e}")
        assert np.all(err <= bound)
        assert ok >= 0.99  # flips are rare: all other outputs agree to FP32 rounding
        assert ex < 3e-2
    net.close()


def test_gradient_matches_oracle():
    from paper_1005_2594_amd import Mlp
    rng = np.random.default_rng(11)
    members = 3
    p = _params(rng, members)
    x = rng.standard_normal((500, 3)).astype(np.float32)
    t = rng.standard_normal(500).astype(np.float32)
    idx = np.stack([rng.choice(500, 128, replace=False) for _ in range(members)]).astype(np.int32)
    net = Mlp(members)
    net.set_params(p)
    g, loss = net.grad(x, t, idx)
    for m in range(members):
        xb, tb = x[idx[m]].astype(np.float64), t[idx[m]].astype(np.float64)
        Lo, go = M.loss_and_grad(p[m], xb, tb, bf16_ops=True)
        _, gx = M.loss_and_grad(p[m], xb, tb)
        assert loss[m] == pytest.approx(Lo, rel=1e-4)
        for name, sl in (("W1", slice(0, 192)), ("b1", slice(192, 256)), ("W2", slice(256, 4352)),
                         ("b2", slice(4352, 4416)), ("W3", slice(4416, 4480)), ("b3", slice(4480, 4481))):
            e = np.max(np.abs(g[m, sl] - go[sl])) / max(np.max(np.abs(go[sl])), 1e-12)
            ex = np.max(np.abs(g[m, sl] - gx[sl])) / max(np.max(np.abs(gx[sl])), 1e-12)
            say(f"member {m} {name}: vs bf16 reference {e:.2e}, vs exact FP64 {ex:.2e}")
            assert e < 1e-3, (m, name, e)
            assert ex < 5e-2, (m, name, ex)
    net.close()


def test_adam_step_matches_oracle():
    from paper_1005_2594_amd import Mlp
    rng = np.random.default_rng(12)
    p = _params(rng, 2)
    x = rng.standard_normal((300, 3)).astype(np.float32)
    mu = np.exp(0.3 * rng.standard_normal(300)).astype(np.float32)
    idx = np.stack([rng.choice(300, (2, 128)) for _ in range(2)]).astype(np.int32)  # [members][steps][batch]
    net = Mlp(2)
    net.set_params(p)  # identity standardisation: t = log mu
    net.train(x, mu, idx, lr=1e-3)
    pg = net.params()
    for m in range(2):
        opt = M.Adam(p[m], lr=1e-3)
        for s in range(2):
            xb = x[idx[m, s]].astype(np.float64)
            tb = np.log(mu[idx[m, s]]).astype(np.float32).astype(np.float64)
            _, go = M.loss_and_grad(opt.p, xb, tb, bf16_ops=True)
            opt.step(go)
        # each step moves a parameter by at most lr; agreement to a small
        # fraction of that (gradients differ by rounding)
        assert np.max(np.abs(pg[m] - opt.p)) < 2e-4, np.max(np.abs(pg[m] - opt.p))
    net.close()


def test_training_fits_and_spread_reflects_uncertainty():
    from paper_1005_2594_amd import Mlp
    rng = np.random.default_rng(13)
    members, n = 5, 2048
    x = rng.uniform([0.1, -3.0, 10.0], [0.5, 1.0, 40.0], (n, 3)).astype(np.float32)
    mu = np.exp(2.0 * x[:, 0] + 0.2 * np.sin(x[:, 1]) + 0.01 * x[:, 2]).astype(np.float32)
    net = Mlp(members)
    net.set_params(M.init_params(rng, members))
    net.set_norm(x.mean(0), x.std(0), float(np.log(mu).mean()), float(np.log(mu).std()))
    steps = 600
    idx = rng.integers(0, n, (members, steps, 128)).astype(np.int32)
    loss = net.train(x, mu, idx, lr=3e-3)
    say("loss first/last", loss[:, :5].mean(), loss[:, -20:].mean())
    assert loss[:, -20:].mean() < 0.02 * loss[:, :5].mean()
    xt = rng.uniform([0.1, -3.0, 10.0], [0.5, 1.0, 40.0], (1000, 3)).astype(np.float32)
    mut = np.exp(2.0 * xt[:, 0] + 0.2 * np.sin(xt[:, 1]) + 0.01 * xt[:, 2])
    mean, spread = net.predict(xt)
    err = np.abs(mean - mut) / mut
    say("in-range median rel err", np.median(err), "max", err.max(), "median spread", np.median(spread))
    assert np.median(err) < 0.02 and np.median(spread) < 0.05
    # far outside the training box the members disagree
    xo = np.array([[0.9, 4.0, 150.0]] * 16, dtype=np.float32)
    _, so = net.predict(xo)
    say("out-of-range spread", so[0])
    assert so[0] > 5 * np.median(spread)
    # device entry point gives the host one's values
    import torch
    xd = torch.from_numpy(xt).cuda()
    md = torch.empty(1000, device="cuda"); sd = torch.empty(1000, device="cuda")
    net.predict_device(1000, xd.data_ptr(), md.data_ptr(), sd.data_ptr(), torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert np.array_equal(md.cpu().numpy(), mean)
    net.close()


def test_training_is_bit_reproducible():
    # every sum over a training batch runs in a fixed order: two handles
    # trained from the same parameters on the same batches agree bit for bit
    from paper_1005_2594_amd import Mlp
    rng = np.random.default_rng(14)
    members, n, steps = 3, 700, 40
    p = _params(rng, members)
    x = rng.standard_normal((n, 3)).astype(np.float32)
    mu = np.exp(0.3 * rng.standard_normal(n)).astype(np.float32)
    idx = rng.integers(0, n, (members, steps, 128)).astype(np.int32)
    out = []
    for _ in range(2):
        net = Mlp(members)
        net.set_params(p)
        loss = net.train(x, mu, idx, lr=2e-3)
        g, gl = net.grad(x, np.log(mu), idx[:, 0])
        out.append((net.params(), loss, g, gl))
        net.close()
    for a, b in zip(*out):
        assert np.array_equal(a, b)
