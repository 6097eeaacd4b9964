"""Pins of the closure network's FP64 reference (CPU only): gradients against
central finite differences, bfloat16 rounding against torch's conversion, and
that Adam on the reference gradients lowers the loss."""
import numpy as np
import pytest
import torch

from oracle import mlp


def _batch(n, seed=0):
    rng = np.random.default_rng(seed)
    X = rng.normal(0, 1, (n, mlp.NIN))
    Y = np.stack([rng.uniform(0.2, 0.6, n), rng.normal(0, 0.1, n)], axis=1)
    return X, Y


def test_gradient_matches_finite_differences():
    theta = mlp.init_params(1)
    X, Y = _batch(16)
    loss, g = mlp.loss_and_grad(theta, X, Y, bf16=False)
    rng = np.random.default_rng(3)
    # every bias entry plus a random sample of weight entries (W1 padded rows excluded)
    o = 0
    idx = []
    for name, shp in mlp.SHAPES:
        n = int(np.prod(shp))
        if name.startswith("b"):
            idx += list(range(o, o + n))
        else:
            lo = o if name != "W1" else o
            hi = o + (n if name != "W1" else mlp.NIN * mlp.NH)
            idx += list(rng.choice(np.arange(lo, hi), 40, replace=False))
        o += n
    h = 1e-6
    for k in idx:
        tp = theta.copy()
        tm = theta.copy()
        tp[k] += h
        tm[k] -= h
        fd = (mlp.loss_and_grad(tp, X, Y, bf16=False)[0] - mlp.loss_and_grad(tm, X, Y, bf16=False)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])) + 1e-9, (k, fd, g[k])


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(5)
    x = np.concatenate([rng.normal(0, 1, 1000) * 10.0 ** rng.integers(-20, 20, 1000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.0078125, 3.0e38]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(mlp.bf16_round(x), ref)


def test_adam_reduces_loss():
    theta = mlp.init_params(2)
    X, Y = _batch(256, seed=7)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    l0 = mlp.loss_and_grad(theta, X, Y)[0]
    for t in range(1, 51):
        loss, g = mlp.loss_and_grad(theta, X, Y)
        theta, m, v = mlp.adam_step(theta, m, v, g, t, lr=3e-3)
    assert mlp.loss_and_grad(theta, X, Y)[0] < 0.5 * l0


def test_sigmoid_output_in_unit_interval():
    theta = mlp.init_params(0)
    X, _ = _batch(64)
    out, _ = mlp.forward(theta, X)
    assert np.all((out[:, 0] > 0) & (out[:, 0] < 1))
