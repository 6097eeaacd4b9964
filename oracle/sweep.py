"""High-order transport sweep (oracle; test infrastructure only).

Paper Sec. 5: the multigroup RT equation (Eq. rt) is integrated in time by the
implicit (backward) Euler scheme with opacities and emission at the new time
level, and in space by the simple corner balance (SCB) method.  For one group g
and direction mu on a slab cell i = [x_{i-1/2}, x_{i+1/2}] the time-discrete
equation is

    mu dI/dx + sigma* I = q*,   sigma* = kappa_g(T_i) + 1/(c dt),
                                q*_corner = kappa_g(T_i) B_g(T_i) + I^{j-1}_corner / (c dt).

SCB in one dimension keeps one unknown per corner (left corner L at x_{i-1/2},
right corner R at x_{i+1/2}) and balances each half cell.  For mu > 0, with
upwind inflow I_in at x_{i-1/2}, the flux at the cell centre taken as the
average (I_L + I_R)/2 and the outflow at x_{i+1/2} equal to I_R:

    left half:   mu (I_L + I_R)/2 - mu I_in + sigma* dx/2 I_L = dx/2 q*_L
    right half:  mu I_R - mu (I_L + I_R)/2 + sigma* dx/2 I_R = dx/2 q*_R

For mu < 0 the roles of the corners are mirrored (the sweep runs from x = X to
x = 0, inflow enters at x_{i+1/2}).  The 2x2 system is solved by Cramer's rule.
"""
from __future__ import annotations

import numpy as np


def sweep(mu, x_edges, kappa, B, I_prev, inc_left, inc_right, c, dt, source=None):
    """One transport sweep over every group and direction.

    mu        [M] direction cosines
    x_edges   [nx+1]
    kappa, B  [G, nx] opacity and group Planck function at the sweep temperature
    I_prev    [G, M, nx, 2] corner intensities at the previous time level
              (corner 0 = left corner, corner 1 = right corner)
    inc_left  [G] isotropic incoming intensity at x = 0 (used for mu > 0)
    inc_right [G] isotropic incoming intensity at x = X (used for mu < 0)
    source    [G, nx] emission sigma_B,g B_g of the group (default kappa B,
              the point law where sigma_B = sigma_E = kappa); kappa is then
              the absorption opacity sigma_E,g and B is not used
    returns I [G, M, nx, 2]
    """
    mu = np.asarray(mu, dtype=np.float64)
    dx = np.diff(np.asarray(x_edges, dtype=np.float64))
    G, nx = kappa.shape
    M = len(mu)
    inv_cdt = 1.0 / (c * dt)
    sig = kappa + inv_cdt
    src = kappa * B if source is None else np.asarray(source, dtype=np.float64)
    I = np.empty((G, M, nx, 2))
    for m in range(M):
        amu = abs(mu[m])
        if mu[m] > 0:
            order = range(nx)
            up, dn = 0, 1  # upwind corner, downwind corner
            I_in = np.array(inc_left, dtype=np.float64)
        else:
            order = range(nx - 1, -1, -1)
            up, dn = 1, 0
            I_in = np.array(inc_right, dtype=np.float64)
        for i in order:
            # half-cell balances in upwind/downwind form:
            #   (a + b) I_up + a I_dn = s_up + |mu| I_in
            #   -a I_up + (a + b) I_dn = s_dn
            a = amu / 2.0
            b = sig[:, i] * dx[i] / 2.0
            s_up = dx[i] / 2.0 * (src[:, i] + inv_cdt * I_prev[:, m, i, up])
            s_dn = dx[i] / 2.0 * (src[:, i] + inv_cdt * I_prev[:, m, i, dn])
            r1 = s_up + amu * I_in
            r2 = s_dn
            det = (a + b) * (a + b) + a * a
            I_up = (r1 * (a + b) - a * r2) / det
            I_dn = ((a + b) * r2 + a * r1) / det
            I[:, m, i, up] = I_up
            I[:, m, i, dn] = I_dn
            I_in = I_dn
    return I
