"""Group opacities by their defining spectral integrals (oracle; test
infrastructure only).

Paper Sec. 2 (the multigroup RT equation, Eq. rt, and the definitions that
follow it) and Sec. 3.1 (the Rosseland group opacity of the first moment
equation, Eq. mloqd-2).  For a group omega_g = [nu_g, nu_{g+1}] and a spectral
opacity sigma(nu, T):

    sigma_B,g(T)      = int sigma(nu, T) B(nu, T)  dnu / int B(nu, T)  dnu
    sigma_E,g(T, T_r) = int sigma(nu, T) B(nu, T_r) dnu / int B(nu, T_r) dnu
    sigma_R,g(T, T_r) = int dB/dT'(nu, T_r) dnu / int dB/dT'(nu, T_r) / sigma(nu, T) dnu

with B the Planck function times 2 pi (any constant factor of B cancels in
each ratio).  sigma_B,g enters the method only through the group emission
sigma_B,g B_g (source of the RT equation and 2 sigma_B,g B_g of the LO
balance).  The effective radiation temperature T_r is not defined in the paper;
reading: T_r = (E / a_R)^(1/4) with E the grey (total) radiation energy density
of the latest grey solve in the cell.

Spectral opacity of the Fleck-Cummings test (Sec. 6), with hnu and kT in keV:
    sigma(nu, T) = C / nu^3 (1 - exp(-nu / T)),  C = 27.

Every integral here is the definition evaluated by adaptive Gauss-Kronrod
quadrature (scipy.integrate.quad, relative tolerance 1e-13; an open last
group is cut where its weights have decayed by e^(-190)).  To keep the
integrands finite in the Wien tail (nu >> T_r), the weights of both integrals
of a ratio are multiplied by exp(nu_g / T_r) (the common factor cancels):
    b(nu)  = nu^3 exp(-(nu - nu_g)/T_r) / (1 - exp(-nu/T_r))          ~ B(nu, T_r)
    db(nu) = nu^4 exp(-(nu - nu_g)/T_r) / (1 - exp(-nu/T_r))^2        ~ dB/dT'(nu, T_r)
The last group may extend to infinity.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.integrate import quad

EPSREL = 1e-13


def fc_sigma(C):
    """Spectral opacity of the Fleck-Cummings test, sigma(nu, T) = C / nu^3 (1 - e^(-nu/T))."""
    def sigma(nu, T):
        return C / nu ** 3 * (-math.expm1(-nu / T))
    return sigma


def _b(nu, a, Tr):
    return nu ** 3 * math.exp(-(nu - a) / Tr) / (-math.expm1(-nu / Tr))


def _db(nu, a, Tr):
    d = -math.expm1(-nu / Tr)
    return nu ** 4 * math.exp(-(nu - a) / Tr) / (d * d)


def _q(f, a, b, Tr):
    """int_a^b f; an open group ends at max(a, 8 T_r) + 200 T_r, beyond which
    every integrand here is below e^(-190) of its largest value."""
    if not np.isfinite(b):
        b = max(a, 8.0 * Tr) + 200.0 * Tr
    v, _ = quad(f, a, b, epsabs=0.0, epsrel=EPSREL, limit=400)
    return v


def _safe(f):
    """The integrands are smooth with finite limits at nu = 0 (0 there)."""
    def g(nu):
        return 0.0 if nu <= 0.0 else f(nu)
    return g


def group_sigma_E(a, b, T, Tr, sigma):
    """sigma_E,g(T, T_r) of the group [a, b] (b may be inf)."""
    num = _q(_safe(lambda nu: sigma(nu, T) * _b(nu, a, Tr)), a, b, Tr)
    den = _q(_safe(lambda nu: _b(nu, a, Tr)), a, b, Tr)
    return num / den


def group_sigma_B(a, b, T, sigma):
    """sigma_B,g(T): sigma_E,g with the weights at the material temperature."""
    return group_sigma_E(a, b, T, T, sigma)


def group_sigma_R(a, b, T, Tr, sigma):
    """sigma_R,g(T, T_r): the dB/dT-weighted harmonic mean of sigma."""
    num = _q(_safe(lambda nu: _db(nu, a, Tr)), a, b, Tr)
    den = _q(_safe(lambda nu: _db(nu, a, Tr) / sigma(nu, T)), a, b, Tr)
    return num / den


def radiation_temperature(Egrey, aR):
    """Reading: T_r = (E / a_R)^(1/4) from the grey energy density."""
    return (np.maximum(np.asarray(Egrey, dtype=np.float64), 1e-300) / aR) ** 0.25


def spectral_tables(nu_edges, C_cell, T, Tr, aR, c):
    """Group coefficients of the FC opacity law per (group g, cell i):
    (sigma_E [G, nx], emission source sigma_B,g B_g [G, nx], sigma_R [G, nx]).

    sigma_E and sigma_R are the quadratures of their definitions; the source
    is sigma_B,g(T) times the group Planck integral B_g(T), evaluated as
    sigma_B,g B_g = int sigma(nu, T) B(nu, T) dnu, which for this opacity law
    has the closed form (the stimulated-emission factor cancels the Planck
    denominator):  C (a_R c / 2)(15 / pi^4) T (e^(-nu_g/T) - e^(-nu_{g+1}/T))."""
    nu_edges = np.asarray(nu_edges, dtype=np.float64)
    T = np.atleast_1d(np.asarray(T, dtype=np.float64))
    Tr = np.atleast_1d(np.asarray(Tr, dtype=np.float64))
    C_cell = np.asarray(C_cell, dtype=np.float64)
    G, nx = len(nu_edges) - 1, len(T)
    sE = np.empty((G, nx))
    sR = np.empty((G, nx))
    for i in range(nx):
        sig = fc_sigma(C_cell[i])
        for g in range(G):
            a, b = nu_edges[g], nu_edges[g + 1]
            sE[g, i] = group_sigma_E(a, b, T[i], Tr[i], sig)
            sR[g, i] = group_sigma_R(a, b, T[i], Tr[i], sig)
    return sE, emission(nu_edges, C_cell, T, aR, c), sR


def emission(nu_edges, C_cell, T, aR, c):
    """sigma_B,g B_g(T) of the FC law in closed form -> [G, nx], written as
    e^(-x_g) (1 - e^(-(x_{g+1} - x_g))) so that narrow groups keep their
    relative precision (x = nu / T)."""
    nu_edges = np.asarray(nu_edges, dtype=np.float64)
    T = np.atleast_1d(np.asarray(T, dtype=np.float64))
    K = aR * c / 2.0 * 15.0 / math.pi ** 4
    with np.errstate(over="ignore", invalid="ignore", divide="ignore"):
        x = nu_edges[:, None] / T[None, :]
        d = x[1:] - x[:-1]
        val = np.exp(-x[:-1]) * (-np.expm1(-d))
    return np.asarray(C_cell)[None, :] * K * T[None, :] * val


def emission_dT(nu_edges, C_cell, T, aR, c):
    """d/dT of sigma_B,g B_g(T) (closed form) -> [G, nx]:
    C K [(1 + x_g) e^(-x_g) - (1 + x_{g+1}) e^(-x_{g+1})],  x = nu / T,
    written as C K e^(-x_g) [-(1 + x_g) expm1(-d) - d e^(-d)], d = x_{g+1} - x_g."""
    nu_edges = np.asarray(nu_edges, dtype=np.float64)
    T = np.atleast_1d(np.asarray(T, dtype=np.float64))
    K = aR * c / 2.0 * 15.0 / math.pi ** 4
    with np.errstate(over="ignore", invalid="ignore", divide="ignore"):
        x = nu_edges[:, None] / T[None, :]
        xa = x[:-1]
        d = x[1:] - xa
        tail = np.where(np.isfinite(d), d * np.exp(-d), 0.0)
        val = np.exp(-xa) * (-(1.0 + xa) * np.expm1(-d) - tail)
    return np.asarray(C_cell)[None, :] * K * val
