"""Prolongation of a coarse-group spectrum to the fine groups (oracle).

TEST INFRASTRUCTURE ONLY.

The paper's multigrid moves coarse-grid information back to the fine grid only
through the temperature (the fine spectrum is re-solved at the new T, Alg. 3);
it names prolongation between frequency grids as a general multigrid operator
(Sec. 1, Sec. 7).  The learned closure adds an explicit one: the energy
density of coarse group p is distributed over its fine groups g by the
previous within-block spectral shape, corrected by the network's prediction
r_g of the log change of that shape:

  w_g = E'_g exp(r_g),   E_g = E_p w_g / sum_{g' in p} w_g'

with E' the previous fine spectrum.  When the block's weights sum to TINY or
less the coarse value is split evenly.  By construction the prolonged groups
of a block sum to E_p, and with r = 0 and E_p the block sum of E' the previous
spectrum is reproduced.
"""
from __future__ import annotations

import numpy as np

from .moments import TINY


def prolong(E_coarse, E_prev, r=None):
    """E_coarse [n_p][nx], E_prev [G][nx], r [G][nx] or None -> E_fine [G][nx]
    (G a multiple of n_p; block p holds groups p G/n_p .. (p+1) G/n_p - 1)."""
    E_coarse = np.asarray(E_coarse, dtype=np.float64)
    E_prev = np.asarray(E_prev, dtype=np.float64)
    n_p, nx = E_coarse.shape
    G = E_prev.shape[0]
    blk = G // n_p
    corr = np.zeros_like(E_prev) if r is None else np.asarray(r, dtype=np.float64)
    out = np.empty_like(E_prev)
    for p in range(n_p):
        sl = slice(p * blk, (p + 1) * blk)
        w = E_prev[sl] * np.exp(corr[sl])
        W = w.sum(axis=0)
        ok = W > TINY
        out[sl] = np.where(ok[None, :], E_coarse[p][None, :] * w / np.where(ok, W, 1.0)[None, :],
                           E_coarse[p][None, :] / blk)
    return out
