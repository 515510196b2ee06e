"""Pins of the FP64 MLP oracle (not GPU): backward against central finite
differences, forward against hand-computable closed forms, the bfloat16
rounding against IEEE bit patterns, and the first Adam step in closed form."""
import numpy as np
import pytest

from oracle import mlp


def rand_params(seed, scale=0.3):
    return np.random.default_rng(seed).normal(0, scale, size=mlp.NPARAM)


def test_layout_size():
    assert mlp.NPARAM == 8 * 64 + 64 + 64 * 64 + 64 + 64 * 2 + 2 == 4866


def test_forward_closed_forms():
    p = np.zeros(mlp.NPARAM)
    u = mlp.unpack(p)
    # zero weights: output is the last bias
    p[-2:] = [0.25, -1.5]
    y, _ = mlp.forward(p, np.ones((3, 8)))
    assert np.allclose(y, [[0.25, -1.5]] * 3)
    # one path: x0 -> h1[5] -> h2[7] -> y1
    p = np.zeros(mlp.NPARAM)
    off = {}
    at = 0
    for name, shape in mlp.SIZES:
        off[name] = at
        at += int(np.prod(shape))
    p[off["W1"] + 0 * 64 + 5] = 0.7
    p[off["W2"] + 5 * 64 + 7] = -1.3
    p[off["W3"] + 7 * 2 + 1] = 2.0
    x = np.zeros((1, 8))
    x[0, 0] = 0.9
    y, _ = mlp.forward(p, x)
    assert y[0, 0] == 0.0
    assert y[0, 1] == pytest.approx(2.0 * np.tanh(-1.3 * np.tanh(0.7 * 0.9)), rel=1e-15)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_backward_matches_central_differences(seed):
    rng = np.random.default_rng(100 + seed)
    p = rand_params(seed)
    x = rng.normal(size=(5, 8))
    dy = rng.normal(size=(5, 2))
    y, cache = mlp.forward(p, x)
    g = mlp.backward(p, x, cache, dy)
    idx = rng.choice(mlp.NPARAM, size=120, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros(mlp.NPARAM)
        e[i] = h
        fp = (mlp.forward(p + e, x)[0] * dy).sum()
        fm = (mlp.forward(p - e, x)[0] * dy).sum()
        fd = (fp - fm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_loss_gradient_matches_differences():
    rng = np.random.default_rng(7)
    y = rng.normal(size=(6, 2))
    t = rng.normal(size=(6, 2))
    w = rng.uniform(1, 5, size=6)
    loss, dy = mlp.loss_and_dy(y, t, w)
    for k in range(6):
        for o in range(2):
            e = np.zeros_like(y)
            e[k, o] = 1e-7
            fd = (mlp.loss_and_dy(y + e, t, w)[0] - mlp.loss_and_dy(y - e, t, w)[0]) / 2e-7
            assert fd == pytest.approx(dy[k, o], rel=1e-6, abs=1e-9)


def test_bf16_rounding_bit_patterns():
    vals = np.array([1.0, -2.0, 1.0 + 2**-8, 1.0 + 3 * 2**-8, 1.0 + 2**-9, 0.0, -0.0, np.inf], dtype=np.float32)
    # 1+2^-8 is a tie between 0x3F80 and 0x3F81: even wins; 1+3*2^-8 ties to 0x3F82
    assert mlp.bf16_round(vals).tolist() == [0x3F80, 0xC000, 0x3F80, 0x3F82, 0x3F80, 0x0000, 0x8000, 0x7F80]
    x = np.random.default_rng(1).normal(size=1000).astype(np.float32)
    back = mlp.bf16_to_f64(mlp.bf16_round(x))
    assert np.all(np.abs(back - x) <= np.abs(x) * 2**-8)


def test_first_adam_step_closed_form():
    w = np.array([0.5, -0.25, 1.0])
    g = np.array([0.1, -3.0, 0.0])
    w1, m1, v1 = mlp.adam_step(w, np.zeros(3), np.zeros(3), g, lr=0.01, b1=0.9, b2=0.999, eps=1e-8, wd=0.0, step=1)
    # bias-corrected first step: w - lr * g / (|g| + eps)
    assert np.allclose(w1, w - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m1, 0.1 * g) and np.allclose(v1, 0.001 * g * g)
