"""Learned closure: training data from the solver's own time steps and training
on the GPU with the library's MFMA kernels.

Samples are (group, cell) pairs.  Inputs: the closure features at the start
of a time step (temperature profile T^{j-1} and its neighbours, group centre,
optical depth of the cell at T^{j-1}, the current factor f^{j-1} and the
temperature change of the previous step).  Targets: the change of the cell
Eddington factor over the step, f^j - f^{j-1}, as the sigmoid value
1/2 + (f^j - f^{j-1}) / (2 DF), and the change of the within-block spectral
shape (blocks of the first coarse frequency grid).  The solver adds the
predicted change to f^{j-1} only to seed transport iteration s = 0; the plain
sweeps decide convergence.
"""
from __future__ import annotations

import dataclasses
from typing import List, Sequence

import numpy as np

from . import binding

NIN, NIN_PAD, NH, NOUT = 7, 8, 128, 2


def init_params(seed: int = 0) -> np.ndarray:
    """He-normal weights (zero padded input rows), zero biases, float32."""
    rng = np.random.default_rng(seed)
    W1 = np.zeros((NIN_PAD, NH))
    W1[:NIN] = rng.normal(0.0, np.sqrt(2.0 / NIN), (NIN, NH))
    W2 = rng.normal(0.0, np.sqrt(2.0 / NH), (NH, NH))
    W3 = rng.normal(0.0, np.sqrt(2.0 / NH), (NH, NH))
    W4 = rng.normal(0.0, np.sqrt(1.0 / NH), (NH, NOUT))
    parts = [W1, np.zeros(NH), W2, np.zeros(NH), W3, np.zeros(NH), W4, np.zeros(NOUT)]
    return np.concatenate([p.ravel() for p in parts]).astype(np.float32)


@dataclasses.dataclass
class Dataset:
    X: object  # torch cuda float32 [n, 8], standardised
    Y: object  # torch cuda float32 [n, 2]
    mean: np.ndarray
    std: np.ndarray
    n_steps: int
    n_sweeps: int


def generate(slab, cfg, levels: Sequence[int], nsteps: int, n_samples: int, seed: int = 0) -> Dataset:
    """Runs the plain solver for nsteps steps and samples (features, targets)."""
    import torch

    sv = binding.Solver([slab], [levels], cfg)
    st = sv.new_state()
    sv.state_init(st, slab.T0)
    n = slab.ng * slab.nx
    kappa, B = sv.empty(binding.TR_K_GI), sv.empty(binding.TR_K_GI)
    zero, one = np.zeros(NIN), np.ones(NIN)
    block = max(1, slab.ng // levels[1]) if len(levels) > 2 else slab.ng
    xs, ys = [], []
    stats = (binding.TrStats * 1)()
    T_hist = None
    for _ in range(nsteps):
        T0 = st["T"].clone()
        E0 = st["E"].clone()
        f0 = st["f"].clone()
        sv.opacity(T0, kappa, B)
        X = torch.empty((n, NIN_PAD), dtype=torch.float32, device="cuda")
        sv.mlp_features(T0, T_hist, kappa, f0, zero, one, X)
        sv.step(st, stats=stats)
        Y = torch.empty((n, NOUT), dtype=torch.float32, device="cuda")
        sv.closure_targets(st["f"], f0, st["E"], E0, block, Y)
        xs.append(X)
        ys.append(Y)
        T_hist = T0
    torch.cuda.synchronize()
    sv.close()
    Xa = torch.cat(xs).cpu().numpy()
    Ya = torch.cat(ys).cpu().numpy()
    rng = np.random.default_rng(seed)
    take = rng.permutation(Xa.shape[0])[:min(n_samples, Xa.shape[0])]
    Xs, Ys = Xa[take], Ya[take]
    mean = Xs[:, :NIN].astype(np.float64).mean(axis=0)
    std = Xs[:, :NIN].astype(np.float64).std(axis=0)
    std = np.where(std > 0, std, 1.0)
    Xs[:, :NIN] = ((Xs[:, :NIN] - mean) / std).astype(np.float32)
    Xs[:, NIN:] = 0.0
    return Dataset(X=torch.as_tensor(Xs).to("cuda"), Y=torch.as_tensor(Ys).to("cuda"), mean=mean, std=std,
                   n_steps=nsteps, n_sweeps=int(stats[0].n_ti))


def train(ds: Dataset, epochs: int = 20, batch: int = 4096, lr: float = 1e-3, seed: int = 0):
    """Minibatch Adam on the GPU; returns (network, per-epoch mean losses)."""
    import torch

    net = binding.Mlp(init_params(seed))
    rng = np.random.default_rng(seed + 1)
    n = ds.X.shape[0]
    losses: List[float] = []
    for _ in range(epochs):
        perm = torch.as_tensor(rng.permutation(n).astype(np.int32)).to("cuda")
        losses.append(net.train_epoch(ds.X, ds.Y, perm, batch, lr))
    torch.cuda.synchronize()
    return net, losses
