"""FP64 reference of the learned closure network (oracle; test infrastructure only).

The closure is a multilayer perceptron 7 -> 128 -> 128 -> 128 -> 2 with ReLU
hidden layers.  Output 0 passes through a logistic sigmoid s and predicts the
change of the group Eddington factor over a time step as a residual on the
previous factor: f_seed = f^{j-1} + DF (2 s - 1), DF = 0.05; output 1 is a
linear prolongation correction r_g,i (the log change of the within-block
spectral shape).  The loss of a batch of n samples is
(1/n) sum [(shat - s)^2 + (rhat - r)^2].

The GPU runs the products in bfloat16 with float32 accumulation: the weights
and each layer's input activations are rounded to bfloat16 (round to nearest,
ties to even) before the product.  ``forward(..., bf16=True)`` applies the same
rounding points and evaluates everything else in float64, so GPU and oracle
differ only by the float32 accumulation.  The pure float64 path
(``bf16=False``) is pinned by central finite differences.

Parameter vector layout (float32 on the GPU, float64 here), row-major:
  W1 [8][128]  (input features padded from 7 to 8 with a zero row)
  b1 [128]
  W2 [128][128], b2 [128], W3 [128][128], b3 [128]
  W4 [128][2], b4 [2]
"""
from __future__ import annotations

import numpy as np

NIN, NIN_PAD, NH, NOUT = 7, 8, 128, 2
DF = 0.05  # scale of the predicted factor change
SHAPES = [("W1", (NIN_PAD, NH)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)),
          ("W3", (NH, NH)), ("b3", (NH,)), ("W4", (NH, NOUT)), ("b4", (NOUT,))]
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta):
    out, o = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = np.asarray(theta[o:o + n], dtype=np.float64).reshape(shp)
        o += n
    return out


def pack(p):
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def init_params(seed=0):
    """He-normal weights (the padded input rows of W1 are zero), zero biases."""
    rng = np.random.default_rng(seed)
    p = {}
    p["W1"] = np.zeros((NIN_PAD, NH))
    p["W1"][:NIN] = rng.normal(0.0, np.sqrt(2.0 / NIN), (NIN, NH))
    p["b1"] = np.zeros(NH)
    p["W2"] = rng.normal(0.0, np.sqrt(2.0 / NH), (NH, NH))
    p["b2"] = np.zeros(NH)
    p["W3"] = rng.normal(0.0, np.sqrt(2.0 / NH), (NH, NH))
    p["b3"] = np.zeros(NH)
    p["W4"] = rng.normal(0.0, np.sqrt(1.0 / NH), (NH, NOUT))
    p["b4"] = np.zeros(NOUT)
    return pack(p).astype(np.float32).astype(np.float64)


def bf16_round(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def _q(x, bf16):
    return bf16_round(x) if bf16 else np.asarray(x, dtype=np.float64)


def forward(theta, X, bf16=True):
    """X [n, 5] (or [n, 8]) standardised features -> (out [n, 2], cache)."""
    p = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    if X.shape[1] == NIN:
        X = np.concatenate([X, np.zeros((X.shape[0], NIN_PAD - NIN))], axis=1)
    a0 = _q(X, bf16)
    z1 = a0 @ _q(p["W1"], bf16) + p["b1"]
    h1 = np.maximum(z1, 0.0)
    a1 = _q(h1, bf16)
    z2 = a1 @ _q(p["W2"], bf16) + p["b2"]
    h2 = np.maximum(z2, 0.0)
    a2 = _q(h2, bf16)
    z3 = a2 @ _q(p["W3"], bf16) + p["b3"]
    h3 = np.maximum(z3, 0.0)
    a3 = _q(h3, bf16)
    o = a3 @ _q(p["W4"], bf16) + p["b4"]
    fhat = 1.0 / (1.0 + np.exp(-o[:, 0]))
    out = np.stack([fhat, o[:, 1]], axis=1)
    cache = dict(p=p, a=[a0, a1, a2, a3], z=[z1, z2, z3], o=o, fhat=fhat, bf16=bf16)
    return out, cache


def loss_and_grad(theta, X, Y, bf16=True):
    """Mean-squared loss of (fhat, rhat) vs Y [n, 2] and its gradient with
    respect to the parameter vector (back-propagation in float64 through the
    same rounded forward values)."""
    out, c = forward(theta, X, bf16)
    Y = np.asarray(Y, dtype=np.float64)
    n = X.shape[0]
    d = out - Y
    loss = float(np.sum(d * d) / n)
    fh = c["fhat"]
    do = np.stack([2.0 * d[:, 0] * fh * (1.0 - fh), 2.0 * d[:, 1]], axis=1) / n
    p, a, z = c["p"], c["a"], c["z"]
    W = {k: _q(p[k], bf16) for k in ("W1", "W2", "W3", "W4")}
    g = {}
    g["W4"] = a[3].T @ do
    g["b4"] = do.sum(axis=0)
    dz3 = (do @ W["W4"].T) * (z[2] > 0)
    g["W3"] = a[2].T @ dz3
    g["b3"] = dz3.sum(axis=0)
    dz2 = (dz3 @ W["W3"].T) * (z[1] > 0)
    g["W2"] = a[1].T @ dz2
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2 @ W["W2"].T) * (z[0] > 0)
    g["W1"] = a[0].T @ dz1
    g["b1"] = dz1.sum(axis=0)
    return loss, pack(g)


def adam_step(theta, m, v, grad, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (t counts from 1); returns new (theta, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def features(T, nu_center, kappa, dx, T_left, f_prev, T_prev=None):
    """Closure inputs per (group g, cell i), sample index g * nx + i:
    log T_i, log nu_g, log(kappa_g,i dx_i), log T_{i-1}, log T_{i+1}, the
    current factor f_g,i, and log(T_i / T_i^prev), the temperature change of
    the last time step (0 without a previous step).  The left neighbour of
    cell 0 is the incoming Planck temperature when positive (else T_0), the
    right neighbour of the last cell is the cell itself."""
    T = np.asarray(T, dtype=np.float64)
    G, nx = kappa.shape
    Tl = np.concatenate([[T_left if T_left > 0 else T[0]], T[:-1]])
    Tr = np.concatenate([T[1:], [T[-1]]])
    f = np.empty((G, nx, NIN))
    f[:, :, 0] = np.log(T)[None, :]
    f[:, :, 1] = np.log(np.asarray(nu_center))[:, None]
    f[:, :, 2] = np.log(kappa * np.asarray(dx)[None, :])
    f[:, :, 3] = np.log(Tl)[None, :]
    f[:, :, 4] = np.log(Tr)[None, :]
    f[:, :, 5] = np.asarray(f_prev, dtype=np.float64).reshape(G, nx)
    f[:, :, 6] = 0.0 if T_prev is None else np.log(T / np.asarray(T_prev, dtype=np.float64))[None, :]
    return f.reshape(G * nx, NIN)


def standardise(F, mean, std):
    return (np.asarray(F) - np.asarray(mean)[None, :]) / np.asarray(std)[None, :]


def targets(f, f_prev, E_new, E_prev, block, tiny=1e-290):
    """Training targets per (g, i): (s, r) with s = 1/2 + (f - f_prev) / (2 DF)
    clipped to [0.01, 0.99] (the sigmoid value that reproduces the factor
    change) and r the log change of the within-block spectral shape,
    r = log((E_g/E_p) / (E'_g/E'_p)), E_p the sum over the `block` consecutive
    groups containing g; 0 where a share is not above tiny; clipped to [-2, 2]
    (groups near underflow change their share by orders of magnitude and would
    otherwise dominate the loss).  Arrays [G, nx] -> [G * nx, 2]."""
    E_new = np.asarray(E_new, dtype=np.float64)
    E_prev = np.asarray(E_prev, dtype=np.float64)
    G, nx = E_new.shape
    r = np.zeros((G, nx))
    for g0 in range(0, G, block):
        sl = slice(g0, min(G, g0 + block))
        sn = E_new[sl].sum(axis=0)
        sp = E_prev[sl].sum(axis=0)
        for g in range(sl.start, sl.stop):
            ok = (sn > tiny) & (sp > tiny) & (E_new[g] > tiny) & (E_prev[g] > tiny)
            r[g] = np.where(ok, np.log(np.where(ok, (E_new[g] / np.where(ok, sn, 1)) /
                                                 (E_prev[g] / np.where(ok, sp, 1)), 1.0)), 0.0)
    r = np.clip(r, -2.0, 2.0)
    df = np.asarray(f, dtype=np.float64).ravel() - np.asarray(f_prev, dtype=np.float64).ravel()
    s = np.clip(0.5 + df / (2.0 * DF), 0.01, 0.99)
    return np.stack([s, r.ravel()], axis=1)


def seed(f_prev, s_hat):
    """Seeded factor f_prev + DF (2 s_hat - 1), kept only inside (0, 1)
    (else f_prev); returns (factors, accepted mask)."""
    f_prev = np.asarray(f_prev, dtype=np.float64)
    cand = f_prev + DF * (2.0 * np.asarray(s_hat, dtype=np.float64) - 1.0)
    ok = (cand > 0.0) & (cand < 1.0)
    return np.where(ok, cand, f_prev), ok
