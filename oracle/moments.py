"""Angular moments of the high-order solution (oracle; test infrastructure only).

Paper Sec. 3.1:
  * group QD (Eddington) factor f_g = int mu^2 I_g dmu / int I_g dmu   (Eq. f_g),
    taken here from the cell-average corner intensity (I_L + I_R)/2;
  * boundary QD factors C_g^- (x = 0, outgoing half-range mu < 0) and C_g^+
    (x = X, outgoing half-range mu > 0) (Eq. c_g);
  * incoming half-range moments E_g^{in}, F_g^{in} and the boundary condition
    F_g = c C_g (E_g - E_g^{in}) + F_g^{in} (Eq. mloqd-bcs), written here as
    F_g = c C_g E_g + Phi_g with Phi_g = F_g^{in} - c C_g E_g^{in}.
Edge intensities: at x = 0 the mu > 0 values are the incoming data and the mu < 0
values are the left corners of cell 1; at x = X the mu > 0 values are the right
corners of cell nx and the mu < 0 values the incoming data.

A ratio whose denominator is below TINY = 1e-290 (zero, negative, or so close
to the subnormal range that the intensity has lost its precision) falls back to
the isotropic value of the quadrature: f_iso = sum w mu^2 / sum w and
C = -/+ sum_{mu>0} w mu / sum_{mu>0} w.  Without the margin a boundary factor
built from subnormal outgoing intensities jitters between sweeps, and because C
multiplies E - E_in with a large incoming E_in the jitter keeps the transport
iterations from converging below ~1e-9.
"""
from __future__ import annotations

import dataclasses

import numpy as np

TINY = 1e-290


@dataclasses.dataclass
class Factors:
    f: np.ndarray  # [G, nx]
    f_bnd: np.ndarray  # [G, 2] edge factors at x=0 and x=X
    C: np.ndarray  # [G, 2] C^- at x=0 (<=0), C^+ at x=X (>=0)
    Phi: np.ndarray  # [G, 2] inhomogeneous part of the boundary condition
    n_guard: int = 0  # number of isotropic fall-backs used


def iso_factors(mu, w):
    mu = np.asarray(mu, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    f_iso = np.sum(w * mu * mu) / np.sum(w)
    pos = mu > 0
    c_iso = np.sum(w[pos] * mu[pos]) / np.sum(w[pos])
    return f_iso, c_iso


def _ratio(num, den, default):
    ok = (den > TINY) & (num > 0)
    out = np.where(ok, num / np.where(ok, den, 1.0), default)
    return out, int(np.count_nonzero(~ok))


def _ratio_signed(num, den, default):
    ok = den > TINY
    out = np.where(ok, num / np.where(ok, den, 1.0), default)
    return out, int(np.count_nonzero(~ok))


def factors(mu, w, I, inc_left, inc_right, c):
    """QD factors and boundary data from corner intensities I [G, M, nx, 2]."""
    mu = np.asarray(mu, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    f_iso, c_iso = iso_factors(mu, w)
    pos = mu > 0
    neg = mu < 0
    G = I.shape[0]
    Ibar = 0.5 * (I[..., 0] + I[..., 1])  # [G, M, nx]
    phi = np.einsum("m,gmi->gi", w, Ibar)
    chi = np.einsum("m,gmi->gi", w * mu * mu, Ibar)
    f, n1 = _ratio(chi, phi, f_iso)

    inc_l = np.asarray(inc_left, dtype=np.float64)
    inc_r = np.asarray(inc_right, dtype=np.float64)
    # edge intensities psi [G, M]
    psi_l = np.where(pos[None, :], inc_l[:, None], I[:, :, 0, 0])
    psi_r = np.where(pos[None, :], I[:, :, -1, 1], inc_r[:, None])
    f_bnd = np.empty((G, 2))
    f_bnd[:, 0], n2 = _ratio(psi_l @ (w * mu * mu), psi_l @ w, f_iso)
    f_bnd[:, 1], n3 = _ratio(psi_r @ (w * mu * mu), psi_r @ w, f_iso)

    C = np.empty((G, 2))
    # x = 0: outgoing half range mu < 0 (C^- <= 0)
    C[:, 0], n4 = _ratio_signed(psi_l[:, neg] @ (w[neg] * mu[neg]), psi_l[:, neg] @ w[neg], -c_iso)
    # x = X: outgoing half range mu > 0
    C[:, 1], n5 = _ratio_signed(psi_r[:, pos] @ (w[pos] * mu[pos]), psi_r[:, pos] @ w[pos], c_iso)

    # incoming half-range moments
    Ein_l = np.sum(w[pos]) * inc_l / c
    Fin_l = np.sum(w[pos] * mu[pos]) * inc_l
    Ein_r = np.sum(w[neg]) * inc_r / c
    Fin_r = np.sum(w[neg] * mu[neg]) * inc_r
    Phi = np.empty((G, 2))
    Phi[:, 0] = Fin_l - c * C[:, 0] * Ein_l
    Phi[:, 1] = Fin_r - c * C[:, 1] * Ein_r
    return Factors(f=f, f_bnd=f_bnd, C=C, Phi=Phi, n_guard=n1 + n2 + n3 + n4 + n5)


def energy_flux(mu, w, I, c):
    """Cell-average group energy density E_g = (1/c) sum w Ibar and flux
    sum w mu Ibar (Eqs. E_g, F_g) -> ([G, nx], [G, nx])."""
    Ibar = 0.5 * (I[..., 0] + I[..., 1])
    E = np.einsum("m,gmi->gi", w, Ibar) / c
    F = np.einsum("m,gmi->gi", w * mu, Ibar)
    return E, F
