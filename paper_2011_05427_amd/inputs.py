"""Seeded, synthetic problem definitions for the 1-D slab multigroup TRT workloads.

This module is the single source of problem *inputs* shared by the GPU library's
tests/benchmark and by the CPU oracle.  It holds none of the method's arithmetic:
it lays out meshes, frequency-group edges, angular quadrature (taken from
``numpy.polynomial.legendre.leggauss``), per-cell opacity constants, boundary
temperatures and solver settings.  Everything the method computes from these
(Planck group integrals, opacities, sweeps, moments, low-order solves, ...) is
implemented separately on each side.

Problem statement followed (paper Sec. 2, Eqs. rt-nu, eb-nu and the multigroup
form Eqs. rt, rt-bc, rt-ic; test set-up of Sec. 6):
  * slab [0, X], ``nx`` cells, cell edges ``x_edges``;
  * ``ng`` frequency groups; group g spans [nu_edges[g], nu_edges[g+1]] for the
    Planck integrals, with the first edge 0 and the last edge +inf so that the
    group Planck functions sum to a_R c T^4 / 2;
  * opacity law kappa_g(T) = C_cell / nu_c^3 * (1 - exp(-nu_c / T)) evaluated at
    the geometric centre nu_c of each log-spaced group (sigma_E = sigma_B =
    sigma_R = kappa_g);
  * Gauss-Legendre S_N quadrature on [-1, 1];
  * isotropic incoming Planck radiation at temperature ``T_left`` / ``T_right``
    (a non-positive value means vacuum);
  * material energy eps = c_v T, initial temperature T0 and I^0 = B_g(T0).

Units: cm, ns, keV, GJ (c = 29.9792458 cm/ns, a_R = 0.01372 GJ cm^-3 keV^-4).
"""
from __future__ import annotations

import dataclasses
import json
from typing import List, Optional, Sequence

import numpy as np

C_LIGHT = 29.9792458  # cm / ns
A_RAD = 0.01372  # GJ / (cm^3 keV^4)

CYCLE_V, CYCLE_W, CYCLE_F = 0, 1, 2
# Opacity model of a slab: the point law kappa_g(T) = C / nu_c^3 (1 - exp(-nu_c / T))
# at the group centre for sigma_E = sigma_B = sigma_R, or the paper's group
# averages (Planck-weighted sigma_B,g at T, sigma_E,g at T and the radiation
# temperature, Rosseland sigma_R,g) of the spectral law C / nu^3 (1 - exp(-nu / T)).
OPAC_POINT, OPAC_SPECTRAL = 0, 1
_CYCLE_NAMES = {"V": CYCLE_V, "W": CYCLE_W, "F": CYCLE_F}


@dataclasses.dataclass
class Slab:
    """One slab problem (arrays are float64 numpy arrays)."""

    x_edges: np.ndarray  # [nx+1]
    nu_edges: np.ndarray  # [ng+1]; nu_edges[0] may be 0, nu_edges[ng] may be inf
    nu_center: np.ndarray  # [ng]
    mu: np.ndarray  # [nmu], ascending
    w: np.ndarray  # [nmu]
    C_cell: np.ndarray  # [nx] opacity constant per cell
    T_left: float  # incoming Planck temperature at x=0 (<=0: vacuum)
    T_right: float  # incoming Planck temperature at x=X (<=0: vacuum)
    cv: float
    dt: float
    T0: float
    c: float = C_LIGHT
    aR: float = A_RAD
    opacity: int = 0  # OPAC_POINT / OPAC_SPECTRAL

    @property
    def nx(self) -> int:
        return len(self.x_edges) - 1

    @property
    def ng(self) -> int:
        return len(self.nu_center)

    @property
    def nmu(self) -> int:
        return len(self.mu)

    def cell_updates_per_sweep(self) -> int:
        return self.nx * self.ng * self.nmu


@dataclasses.dataclass
class SolverCfg:
    """Iteration settings of the multigrid-in-frequency MLQD step (paper Alg. 3)."""

    levels: List[int]  # groups per frequency grid, fine first, grey (1) last
    cycle: int = CYCLE_V  # CYCLE_V / CYCLE_W / CYCLE_F
    lmax: int = 4  # maximum number of cycles per transport iteration
    eps: float = 1e-10  # outer (transport) tolerance
    eps_inner: float = 1e-11  # inner (low-order) tolerance
    max_outer: int = 50
    secant: bool = True  # diagonal secant Frechet derivative of grey sigma_E
    precision: int = 0  # 0: binary64 intensities; 1: binary32 storage of the corner intensities


def gauss_legendre(n: int):
    mu, w = np.polynomial.legendre.leggauss(n)
    return np.asarray(mu, dtype=np.float64), np.asarray(w, dtype=np.float64)


def log_groups(ng: int, lo: float, hi: float):
    """ng log-spaced groups on [lo, hi]; end groups extend to 0 and +inf for the
    Planck integrals, group centres are the geometric means of the log edges."""
    e = np.logspace(np.log10(lo), np.log10(hi), ng + 1)
    centre = np.sqrt(e[:-1] * e[1:])
    edges = e.copy()
    edges[0] = 0.0
    edges[-1] = np.inf
    return edges, centre


def make_slab(nx: int, ng: int, nmu: int, *, C1: float = 27.0, C2: float = 2.7,
              X: float = 4.0, nu_lo: float = 0.01, nu_hi: float = 100.0,
              T_left: float = 1.0, T_right: float = 0.0, cv: float = 0.5,
              dt: float = 0.002, T0: float = 0.001, opacity: int = OPAC_POINT) -> Slab:
    """Two-zone slab: cells [0, nx//2) use C1, the rest C2."""
    x = np.linspace(0.0, X, nx + 1)
    edges, centre = log_groups(ng, nu_lo, nu_hi)
    mu, w = gauss_legendre(nmu)
    C = np.where(np.arange(nx) < nx // 2, C1, C2).astype(np.float64)
    return Slab(x_edges=x, nu_edges=edges, nu_center=centre, mu=mu, w=w, C_cell=C,
                T_left=T_left, T_right=T_right, cv=cv, dt=dt, T0=T0, opacity=opacity)


def double_gauss_legendre(n: int):
    """Double S_n: the n-point Gauss-Legendre rule mapped to each half range
    [-1, 0] and [0, 1] (2 n directions, ascending, weights summing to 2)."""
    x, w = gauss_legendre(n)
    mp, wp = 0.5 * (x + 1.0), 0.5 * w
    return np.concatenate([-mp[::-1], mp]), np.concatenate([wp[::-1], wp])


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

FC_DT = (0.02, 0.04)  # ns: the two time steps of the Fleck-Cummings runs (150 and 75 steps to 3 ns)


def fc_slab(dt: float = 0.02, opacity: int = OPAC_SPECTRAL) -> Slab:
    """The paper's Fleck-Cummings set-up (Sec. 6): [0, 4] cm in 10 uniform
    cells, one material with the spectral opacity 27 / nu^3 (1 - exp(-nu / T)),
    black-body incoming at 1 keV on the left, vacuum on the right, T0 = 1e-3
    keV, c_v = 0.5917 a_R T_b^3 with T_b = 1 keV, 256 groups: 254 log-spaced
    between 1e-4 and 10 keV and the two end groups [0, 1e-4] and [10, inf)
    (the paper's 1e7 keV bound carries no Planck energy in binary64), double
    S8.  The group opacities are the paper's spectral averages (default) or,
    with opacity=OPAC_POINT, the point law at a group centre; the end groups'
    centres (point law only) extend the log spacing by one ratio."""
    r = (10.0 / 1e-4) ** (1.0 / 254)
    x = np.linspace(0.0, 4.0, 11)
    edges, centre = log_groups(256, 1e-4 / r, 10.0 * r)
    mu, w = double_gauss_legendre(8)
    return Slab(x_edges=x, nu_edges=edges, nu_center=centre, mu=mu, w=w, C_cell=np.full(10, 27.0),
                T_left=1.0, T_right=0.0, cv=0.5917 * A_RAD, dt=dt, T0=0.001, opacity=opacity)


def config_fc(dt: float = 0.02, levels=(256, 1), cycle: int = CYCLE_V, lmax: int = 4,
              opacity: int = OPAC_SPECTRAL):
    """Fleck-Cummings runs of Tables 1 (dt = 0.02 ns) and 2 (0.04 ns): eps =
    1e-6, inner eps = 1e-7, to t = 3 ns."""
    cfg = SolverCfg(levels=list(levels), cycle=cycle, lmax=lmax, eps=1e-6, eps_inner=1e-7)
    return [fc_slab(dt, opacity)], cfg, int(round(3.0 / dt))


def config_small():
    """50 cells, S8, 16 groups, two-grid V (16 -> 1), one step dt=0.002."""
    slab = make_slab(50, 16, 8)
    cfg = SolverCfg(levels=[16, 1], cycle=CYCLE_V, lmax=4)
    return [slab], cfg, 1


def config_paper_scale():
    """200 cells, S16, 512 groups, hierarchy 512,128,32,8,1 with V cycle, 20 steps."""
    slab = make_slab(200, 512, 16)
    cfg = SolverCfg(levels=[512, 128, 32, 8, 1], cycle=CYCLE_V, lmax=4)
    return [slab], cfg, 20


def config_large():
    """2000 cells, S32, 4096 groups, F cycle on 4096,1024,256,64,16,1, 50 steps."""
    slab = make_slab(2000, 4096, 32)
    cfg = SolverCfg(levels=[4096, 1024, 256, 64, 16, 1], cycle=CYCLE_F, lmax=2)
    return [slab], cfg, 50


BATCH_SEED = 201105427


def batch_instances(n_slabs: int = 256, seed: int = BATCH_SEED):
    """Uneven slab batch: nx ~ U{50..400}, G in {64..1024}, S8/S16, C per zone
    log-uniform in [1, 100], left boundary temperature U[0.5, 1.5]."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_slabs):
        nx = int(rng.integers(50, 401))
        ng = int(rng.choice([64, 128, 256, 512, 1024]))
        nmu = int(rng.choice([8, 16]))
        c1, c2 = (10.0 ** rng.uniform(0.0, 2.0, size=2)).tolist()
        tb = float(rng.uniform(0.5, 1.5))
        out.append(dict(nx=nx, ng=ng, nmu=nmu, C1=c1, C2=c2, T_left=tb))
    return out


def config_batch(n_slabs: int = 256, seed: int = BATCH_SEED, scale: float = 1.0):
    """W cycle G -> G/8 -> 1 for every slab.  ``scale`` < 1 shrinks nx and ng
    (for CPU-size test cases) while keeping the distribution's shape."""
    slabs = []
    for d in batch_instances(n_slabs, seed):
        nx = max(4, int(round(d["nx"] * scale)))
        ng = max(8, int(d["ng"] * scale) // 8 * 8)
        slabs.append(make_slab(nx, ng, d["nmu"], C1=d["C1"], C2=d["C2"], T_left=d["T_left"]))
    # every slab shares the cycle shape; level sizes are per slab (G, G/8, 1)
    cfg = SolverCfg(levels=[0, 0, 1], cycle=CYCLE_W, lmax=2)
    return slabs, cfg, 1


def levels_for(slab: Slab, cfg: SolverCfg) -> List[int]:
    """Resolve per-slab level sizes (batch configs give G, G/8, 1)."""
    if cfg.levels[0] == 0:
        return [slab.ng, max(1, slab.ng // 8), 1]
    return list(cfg.levels)


def slab_to_json(s: Slab) -> dict:
    d = dataclasses.asdict(s)
    for k, v in d.items():
        if isinstance(v, np.ndarray):
            d[k] = [float(t) for t in v]
    return d


def dump_instances(path: str, slabs: Sequence[Slab]) -> None:
    with open(path, "w") as fh:
        json.dump([slab_to_json(s) for s in slabs], fh)
