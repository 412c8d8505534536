"""Pins of the closure network's reference: gradients against finite
differences, the bfloat16 rounding against its definition, Adam against its
first-step closed form, and a fit of a smooth function."""
import numpy as np
import pytest

from oracle import mlp_oracle as M


def test_parameter_count():
    assert M.NPARAM == 64 * 3 + 64 + 64 * 64 + 64 + 64 + 1 == 4481


def test_bf16_rounding():
    # exactly representable values stay; halfway cases go to even; the
    # result always has 8 significant bits
    assert M.bf16(1.0) == 1.0 and M.bf16(-2.5) == -2.5
    assert M.bf16(1.0 + 2 ** -8) == 1.0             # halfway, 1.0 is even
    assert M.bf16(1.0 + 3 * 2 ** -8) == 1.0 + 2 ** -6  # halfway, rounds up to even
    assert M.bf16(1.0 + 2 ** -7 + 2 ** -9) == 1.0 + 2 ** -7
    rng = np.random.default_rng(0)
    a = rng.standard_normal(1000)
    r = M.bf16(a)
    assert np.all(np.abs(r - a) <= 2 ** -8 * np.abs(a) + 1e-300)
    m, e = np.frexp(r)
    assert np.all(np.abs(m * 2 ** 8 - np.round(m * 2 ** 8)) == 0)


@pytest.mark.parametrize("bf", [False, True])
def test_gradient_matches_finite_differences(bf):
    rng = np.random.default_rng(1)
    p = M.init_params(rng, 1)[0]
    p[M.NPARAM - 1] = 0.3
    x = rng.standard_normal((20, 3))
    t = rng.standard_normal(20)
    L, g = M.loss_and_grad(p, x, t, bf16_ops=False)
    idx = rng.choice(M.NPARAM, 60, replace=False)
    idx = np.concatenate([idx, [0, 191, 192, 255, 256, 4351, 4352, 4415, 4416, 4480]])
    h = 1e-6
    for i in idx:
        e = np.zeros(M.NPARAM); e[i] = h
        fd = (M.loss_and_grad(p + e, x, t)[0] - M.loss_and_grad(p - e, x, t)[0]) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-5, abs=1e-9), i
    if bf:
        # the bfloat16 variant is the same gradient up to the rounding of its operands
        _, gb = M.loss_and_grad(p, x, t, bf16_ops=True)
        assert np.max(np.abs(gb - g)) < 0.05 * np.max(np.abs(g))


def test_adam_first_step():
    # first step: m_hat = g, v_hat = g^2, so every parameter moves by lr * sign(g)
    # (up to eps)
    g = np.array([0.5, -2.0, 1e-3])
    a = M.Adam(np.zeros(3), lr=0.01)
    p = a.step(g)
    assert np.allclose(p, -0.01 * np.sign(g), rtol=1e-4)


def test_fits_a_smooth_function():
    # full-batch Adam on y = sin(x0) + 0.5 x1 x2 reaches a small error
    rng = np.random.default_rng(2)
    x = rng.uniform(-1, 1, (256, 3))
    t = np.sin(x[:, 0]) + 0.5 * x[:, 1] * x[:, 2]
    p = M.init_params(rng, 1)[0]
    opt = M.Adam(p, lr=3e-3)
    L0 = M.loss_and_grad(opt.p, x, t)[0]
    for _ in range(400):
        L, g = M.loss_and_grad(opt.p, x, t)
        opt.step(g)
    assert L < 0.02 * L0


def test_forward_by_hand():
    # A network whose output is worked out by hand, using sigma(ln 3) = 3/4:
    # W1 rows (1, 0, 0) and (0, -1, 0); input (ln 3, ln 3, 5) gives
    # z1 = (ln 3, -ln 3, 0, ...), h1 = (3/4 ln 3, -1/4 ln 3, 0, ...);
    # W2[0] = (2, 2, 0, ...) gives z2_0 = ln 3 and h2_0 = 3/4 ln 3;
    # W2[1] = (-4, 0, ...) gives z2_1 = -3 ln 3 and h2_1 = -3 ln 3 / 28
    # (sigma(-3 ln 3) = 1/28); W3 = (1, 14, 0, ...), b3 = 1/2:
    # y = 3/4 ln 3 - 3/2 ln 3 + 1/2 = 1/2 - 3/4 ln 3.  A zero input gives b3
    # plus the second layer's biases through SiLU: b2 = (0, 0, 2, ...) and
    # W3[2] = 1 add silu(2) = 2 / (1 + e^-2) to every output.
    d = {name: np.zeros(shape) for name, shape in M.SIZES}
    d["W1"][0] = (1, 0, 0)
    d["W1"][1] = (0, -1, 0)
    d["W2"][0, :2] = (2, 2)
    d["W2"][1, 0] = -4
    d["b2"][2] = 2.0
    d["W3"][:3] = (1, 14, 1)
    d["b3"][0] = 0.5
    p = M.pack(d)
    l3 = np.log(3.0)
    x = np.array([[l3, l3, 5.0], [0.0, 0.0, 0.0]])
    extra = 2.0 / (1.0 + np.exp(-2.0))
    want = np.array([0.5 - 0.75 * l3 + extra, 0.5 + extra])
    y = M.forward(p, x)
    assert np.max(np.abs(y - want)) < 1e-15
    # the device's operand rounding: W entries here are exact in bfloat16, so
    # only h1 = (3/4 ln 3, -1/4 ln 3) changes, to its nearest bfloat16 value
    h0, h1 = M.bf16(0.75 * l3), M.bf16(-0.25 * l3)
    z2 = 2 * (h0 + h1)
    z21 = -4 * h0
    want_bf = 0.5 + z2 / (1 + np.exp(-z2)) + 14 * z21 / (1 + np.exp(-z21)) + extra
    assert abs(M.forward(p, x, bf16_ops=True)[0] - want_bf) < 1e-15
