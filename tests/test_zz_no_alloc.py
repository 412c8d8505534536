"""The training entry point that allocates no device memory
(cgb_mlp_train_noalloc) against cgb_mlp_train: same inputs, bit-identical
parameters and losses, on two calls in a row, the second smaller."""
import numpy as np
import pytest

from oracle import mlp_oracle as M
from parity_util import say

pytestmark = pytest.mark.gpu


def test_noalloc_training_matches_train():
    from paper_1005_2594_amd import Mlp
    from paper_1005_2594_amd.cgb import CgbError
    rng = np.random.default_rng(31)
    members = 5
    p = M.init_params(rng, members).astype(np.float32)
    nets = [Mlp(members), Mlp(members)]
    for net in nets:
        net.set_params(p)
        net.set_norm([0.3, -1.0, 20.0], [0.1, 1.2, 8.0], 1.0, 0.7)
    for n, steps in ((3000, 60), (700, 25)):
        say(f"case: noalloc training, {members} members, {n} samples, {steps} steps")
        x = rng.uniform([0.1, -3.0, 10.0], [0.5, 1.0, 40.0], (n, 3)).astype(np.float32)
        mu = np.exp(2.0 * x[:, 0] + 0.2 * np.sin(x[:, 1])).astype(np.float32)
        idx = rng.integers(0, n, (members, steps, 128)).astype(np.int32)
        la = nets[0].train(x, mu, idx, lr=2e-3)
        lb = nets[1].train_noalloc(x, mu, idx, lr=2e-3)
        assert np.array_equal(la, lb)
        assert np.array_equal(nets[0].params(), nets[1].params())
        assert np.all(np.isfinite(lb)) and lb[:, -5:].mean() < lb[:, :5].mean()
    # beyond the staging limits: refused, nothing changed
    before = nets[1].params()
    big = np.ones((65537, 3), np.float32)
    with pytest.raises(CgbError):
        nets[1].train_noalloc(big, np.ones(65537, np.float32), np.zeros((members, 1, 128), np.int32), 1e-3)
    assert np.array_equal(before, nets[1].params())
    for net in nets:
        net.close()
