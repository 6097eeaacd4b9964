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


def test_residual_targets_and_seed_round_trip():
    """The factor-change target and the seeding rule invert each other inside
    the representable range, and an unchanged factor maps to s = 1/2."""
    rng = np.random.default_rng(9)
    G, nx = 6, 5
    fp = rng.uniform(0.2, 0.8, (G, nx))
    f = fp + rng.uniform(-0.9, 0.9, (G, nx)) * mlp.DF
    E = 10 ** rng.uniform(-3, 0, (G, nx))
    Y = mlp.targets(f, fp, E, E, 3)
    got, ok = mlp.seed(fp.ravel(), Y[:, 0])
    assert ok.all()
    np.testing.assert_allclose(got, f.ravel(), rtol=0, atol=1e-14)
    Y0 = mlp.targets(fp, fp, E, E, 3)
    assert np.all(Y0[:, 0] == 0.5) and np.all(Y0[:, 1] == 0.0)
    # a change beyond the range saturates; a seed outside (0, 1) keeps the old factor
    Yc = mlp.targets(fp + 3 * mlp.DF, fp, E, E, 3)
    assert np.all(Yc[:, 0] == 0.99)
    s, ok = mlp.seed(np.array([0.01, 0.5]), np.array([0.0, 1.0]))
    assert not ok[0] and ok[1] and s[0] == 0.01 and abs(s[1] - 0.55) < 1e-15


def test_features_temperature_change_column():
    rng = np.random.default_rng(4)
    G, nx = 3, 4
    T = 10 ** rng.uniform(-2, 0, nx)
    Tp = T * rng.uniform(0.5, 1.5, nx)
    kap = 10 ** rng.uniform(-1, 2, (G, nx))
    fp = rng.uniform(0.3, 0.6, (G, nx))
    F = mlp.features(T, np.array([0.1, 1.0, 10.0]), kap, np.full(nx, 0.5), 1.0, fp, Tp).reshape(G, nx, mlp.NIN)
    np.testing.assert_allclose(F[:, :, 6], np.log(T / Tp)[None, :].repeat(G, 0), rtol=1e-15)
    np.testing.assert_array_equal(F[:, :, 5], fp)
    F0 = mlp.features(T, np.array([0.1, 1.0, 10.0]), kap, np.full(nx, 0.5), 1.0, fp).reshape(G, nx, mlp.NIN)
    assert np.all(F0[:, :, 6] == 0.0)


def test_adam_bias_correction_gives_scaled_sign_steps():
    """With the bias-corrected moments, a constant gradient g moves every
    parameter by -lr g / (|g| + eps) at every step, the first one included
    (m_hat = g, v_hat = g^2 exactly); without the correction the first step
    would be sqrt(1 - beta2) / (1 - beta1) = 0.316 times that."""
    rng = np.random.default_rng(12)
    n = 64
    theta0 = rng.normal(0, 1, n)
    g = rng.normal(0, 1, n) * 10.0 ** rng.integers(-6, 3, n)
    lr, eps = 1e-3, 1e-8
    theta, m, v = theta0.copy(), np.zeros(n), np.zeros(n)
    for t in range(1, 4):
        prev = theta
        theta, m, v = mlp.adam_step(theta, m, v, g, t, lr=lr, eps=eps)
        np.testing.assert_allclose(theta - prev, -lr * g / (np.abs(g) + eps), rtol=1e-9, atol=1e-18)
