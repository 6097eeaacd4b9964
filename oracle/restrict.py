"""Restriction of LOQD coefficients onto a coarser frequency grid (oracle).

TEST INFRASTRUCTURE ONLY.

Paper Sec. 4 and Sec. 5: the coarse-group equations are the sums of the finer
equations over the groups of each coarse group, closed exactly by weighted
averages of the finer coefficients (Eqs. coeff-gamma, g-notation, eta-gamma for
Omega^1 -> Omega^gamma; Eqs. coeff-Gamma, eta-Gamma, g2G-notation for
Omega^gamma -> Omega^Gamma; the discrete forms mloqd1-d-gamma, mloqd2-d-gamma
with the upwind split of the compensation term into eta_hat and eta_check).

For a block Lambda_p of finer groups and the finer solution (E, F, boundary E):
  sigma_E,p  = <sigma_E>_E            (weights E of the cell)
  e_p        = sum e                  (emission; equals 2 <sigma_B>_B B_p)
  abar_p,e   = <a_e>_{E_R(e)}         bbar_p,e = <b_e>_{E_L(e)}
               (on the fine grid a_e, b_e are the cell QD factors, so these are
                the E-weighted factors <f>_E of the right / left neighbour)
  sigma_R,p  = <sigma_R>_{|F|}        at every edge
  xi_p,e     = h_e sum (sigma_R - sigma_R,p) F_e
  eta_hat    = xi / (c sum E_R)  if xi > 0,   eta_check = -xi / (c sum E_L)  if xi < 0
  a_p,e      = abar + eta_hat,   b_p,e = bbar + eta_check
  C_p        = <C>_{E_boundary},  Phi_p = sum Phi
  E^old_p    = sum E^old,         F^old_p = sum F^old
Readings: xi includes the edge length h_e that multiplies sigma_R F in the
discrete first moment (the printed xi omits it, which would break the exact
sum-over-groups property the paper states); the right/left coefficients are
weighted separately by the energy density they multiply; the inhomogeneous part
of the boundary condition is restricted additively.  With these choices the
coarse equations are satisfied exactly by the block sums of a finer solution at
the same temperature.  A weighted average whose weights sum to TINY = 1e-290
or less falls back to the plain block mean, and a compensation term is dropped
when the energy density it would divide by is that small.
"""
from __future__ import annotations

import numpy as np

from .lo import Level, LOSolution, edge_lengths
from .moments import TINY


def _blocks(x, P):
    """[G, ...] -> [P, r, ...] contiguous uniform blocks."""
    G = x.shape[0]
    if G % P:
        raise ValueError(f"{G} groups do not split into {P} uniform blocks")
    return x.reshape((P, G // P) + x.shape[1:])


def _wavg(psi, H, P):
    """<psi>_H over each block, falling back to the plain mean when sum H <= 0."""
    pb = _blocks(psi, P)
    hb = _blocks(H, P)
    num = np.sum(pb * hb, axis=1)
    den = np.sum(hb, axis=1)
    mean = np.mean(pb, axis=1)
    ok = den > TINY
    return np.where(ok, num / np.where(ok, den, 1.0), mean)


def restrict(lv: Level, sol: LOSolution, P: int, dx, c) -> Level:
    """Coefficients of the P-group level obtained from level ``lv`` and its
    solution ``sol`` (block sums of contiguous groups)."""
    h = edge_lengths(dx)
    u = sol.E_ext()  # [G, nx+2]
    ER = u[:, 1:]  # energy density right of each edge [G, nx+1]
    EL = u[:, :-1]
    absF = np.abs(sol.F)

    sigE = _wavg(lv.sigE, sol.E, P)
    emis = np.sum(_blocks(lv.emis, P), axis=1)
    abar = _wavg(lv.a, ER, P)
    bbar = _wavg(lv.b, EL, P)
    sigR = _wavg(lv.sigR, absF, P)
    xi = h[None, :] * np.sum((_blocks(lv.sigR, P) - sigR[:, None, :]) * _blocks(sol.F, P), axis=1)
    ERp = np.sum(_blocks(ER, P), axis=1)
    ELp = np.sum(_blocks(EL, P), axis=1)
    eta_hat = np.where((xi > 0) & (ERp > TINY), xi / (c * np.where(ERp > TINY, ERp, 1.0)), 0.0)
    eta_chk = np.where((xi < 0) & (ELp > TINY), -xi / (c * np.where(ELp > TINY, ELp, 1.0)), 0.0)
    C = np.stack([_wavg(lv.C[:, 0], sol.Ebnd[:, 0], P), _wavg(lv.C[:, 1], sol.Ebnd[:, 1], P)], axis=1)
    return Level(
        sigE=sigE,
        emis=emis,
        a=abar + eta_hat,
        b=bbar + eta_chk,
        sigR=sigR,
        C=C,
        Phi=np.sum(_blocks(lv.Phi, P), axis=1),
        Eold=np.sum(_blocks(lv.Eold, P), axis=1),
        Fold=np.sum(_blocks(lv.Fold, P), axis=1),
    )
