"""Pins of the oracle's surrogate network (learned form).

* gradients against central finite differences of the loss (a dropped
  term, wrong sign or transposed operand in ``backward`` fails it);
* GELU against tabulated normal-CDF values and its own finite differences;
* a network with zero weights reduces to its biases (closed form);
* the first Adam step moves every parameter by lr * sign(g);
* bfloat16 rounding on values whose nearest-even result is known exactly;
* the bfloat16 mode stays within bfloat16 accuracy of the float64 mode;
* Adam training of a small network fits a smooth function;
* the fallback rule on a constructed grid.
"""
import numpy as np
import pytest

from oracle import mlp

SMALL = (6, 8, 8, 8, 1)


def _data(n=24, seed=0, widths=SMALL):
    rng = np.random.default_rng(seed)
    p = rng.standard_normal(mlp.num_params(widths)) * 0.4
    X = rng.standard_normal((n, widths[0]))
    t = rng.standard_normal(n)
    return p, X, t


def test_gradient_matches_finite_differences():
    p, X, t = _data()
    y, c = mlp.forward(p, X, SMALL)
    g = mlp.backward(p, c, y, t, SMALL)
    eps = 1e-6
    num = np.empty_like(p)
    for k in range(len(p)):
        q = p.copy()
        q[k] += eps
        a = mlp.loss(mlp.forward(q, X, SMALL)[0], t)
        q[k] -= 2 * eps
        b = mlp.loss(mlp.forward(q, X, SMALL)[0], t)
        num[k] = (a - b) / (2 * eps)
    assert np.max(np.abs(num - g)) <= 1e-7 * np.max(np.abs(g))


def test_gelu_values_and_derivative():
    # Phi(1) = 0.8413447460685429, Phi(-1) = 0.15865525393145707 (normal-CDF table)
    assert mlp.gelu(np.array([1.0]))[0] == pytest.approx(0.8413447460685429, rel=1e-15)
    assert mlp.gelu(np.array([-1.0]))[0] == pytest.approx(-0.15865525393145707, rel=1e-14)
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    assert mlp.gelu(np.array([40.0]))[0] == 40.0 and mlp.gelu(np.array([-40.0]))[0] == 0.0
    x = np.linspace(-5, 5, 41)
    h = 1e-6
    fd = (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h)
    assert np.max(np.abs(fd - mlp.gelu_grad(x))) <= 1e-8
    assert mlp.gelu_grad(np.array([0.0]))[0] == 0.5


def test_zero_weights_reduce_to_biases():
    p = np.zeros(mlp.num_params(SMALL))
    P = mlp.unflatten(p, SMALL)
    P["b3"][:] = np.arange(8) * 0.25 - 1.0
    P["W4"][:, 0] = 1.0
    P["b4"][0] = 0.5
    y, _ = mlp.forward(p, np.ones((3, 6)), SMALL)
    b3 = np.arange(8) * 0.25 - 1.0
    # gelu(b3) by the tabulated Phi values is not needed: the sum is checked
    # against an independent closed form of x Phi(x) via the complementary erf
    from math import erfc, sqrt
    expect = 0.5 + sum(b * 0.5 * erfc(-b / sqrt(2.0)) for b in b3)
    assert np.allclose(y, expect, rtol=1e-14, atol=1e-14)


def test_first_adam_step_is_signed_lr():
    rng = np.random.default_rng(3)
    p = rng.standard_normal(50)
    g = rng.standard_normal(50)
    p1, m, v = mlp.adam_step(p, g, np.zeros(50), np.zeros(50), 1, lr=1e-3, eps=0.0)
    assert np.allclose(p1, p - 1e-3 * np.sign(g), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_bf16_rounding_known_values():
    # 1 + 2^-8 lies halfway between 1 and 1 + 2^-7: ties go to the even mantissa (1.0)
    vals = np.array([1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -9, -3.0, 0.0, 65504.0])
    exp = np.array([1.0, 1.0 + 2.0 ** -6, 1.0, -3.0, 0.0, 65536.0])
    assert np.array_equal(mlp.bf16(vals), exp)


def test_bf16_mode_close_to_float64():
    rng = np.random.default_rng(5)
    w = (6, 64, 64, 64, 1)
    p = rng.standard_normal(mlp.num_params(w)) * 0.2
    X = rng.uniform(-1, 1, (128, 6))
    t = rng.standard_normal(128)
    y, c = mlp.forward(p, X, w)
    yq, cq = mlp.forward(p, X, w, bf16_ops=True)
    assert np.max(np.abs(yq - y)) <= 3e-2 * np.max(np.abs(y))
    g = mlp.backward(p, c, y, t, w)
    gq = mlp.backward(p, cq, yq, t, w, bf16_ops=True)
    assert np.linalg.norm(gq - g) <= 3e-2 * np.linalg.norm(g)


def test_adam_fits_smooth_function():
    rng = np.random.default_rng(11)
    w = (6, 32, 32, 32, 1)
    p = rng.standard_normal(mlp.num_params(w))
    P = mlp.unflatten(p, w)
    for i in range(1, 5):
        P[f"W{i}"][:] *= np.sqrt(2.0 / w[i - 1])
        P[f"b{i}"][:] = 0.0
    X = rng.uniform(-1, 1, (256, 6))
    t = np.sin(2 * X[:, 4]) * np.exp(-X[:, 5] ** 2) + 0.3 * X[:, 0]
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    l0 = mlp.loss(mlp.forward(p, X, w)[0], t)
    for k in range(1, 401):
        y, c = mlp.forward(p, X, w)
        p, m, v = mlp.adam_step(p, mlp.backward(p, c, y, t, w), m, v, k, lr=3e-3)
    assert mlp.loss(mlp.forward(p, X, w)[0], t) <= 0.05 * l0


def test_fallback_rows():
    mean = np.zeros((4, 5))
    mean[1, 2] = 10.0
    std = np.full((4, 5), 0.1)
    std[3, 4] = 0.6              # 6% of the peak 10
    std[2, 0] = 0.5              # exactly 5%: not above
    assert list(mlp.fallback_rows(mean, std, 0.05)) == [False, False, False, True]
