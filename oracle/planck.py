"""Group Planck integrals and the opacity law (oracle; test infrastructure only).

Paper Sec. 2: B(nu, T) = 4 pi h nu^3 / c^2 / (exp(h nu / kT) - 1) is the Planck
function times 2 pi, so the slab (azimuth-integrated) intensity of black-body
radiation integrates over all frequencies to a_R c T^4 / 2.  With h nu and kT in
keV and x = nu / T the group integral is

    B_g(T) = (a_R c T^4 / 2) * (15 / pi^4) * int_{x_g}^{x_{g+1}} t^3 / (e^t - 1) dt.

The dimensionless integral is evaluated with the two textbook series:
  * x < 2:  int_0^x t^3/(e^t-1) dt = sum_k B_k x^(k+3) / (k! (k+3))   (Bernoulli B_k)
  * x >= 2: int_x^inf t^3/(e^t-1) dt = sum_n e^(-n x) (x^3/n + 3x^2/n^2 + 6x/n^3 + 6/n^4)
and a group whose two ends both lie in the tail range is differenced from the
tails (no cancellation of two numbers close to pi^4/15).

Opacity (the workloads' point law at the group centre nu_c, standing in for the
Planck-weighted group averages of Sec. 2):
    kappa_g(T) = C / nu_c^3 * (1 - exp(-nu_c / T)),  sigma_E = sigma_B = sigma_R = kappa_g.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import bernoulli

TOTAL = math.pi ** 4 / 15.0  # int_0^inf t^3/(e^t-1) dt
X_SWITCH = 2.0

_NB = 48
_BK = bernoulli(_NB)  # B_0..B_NB with B_1 = -1/2
_HEAD_COEF = np.array([_BK[k] / (math.factorial(k) * (k + 3)) for k in range(_NB + 1)])


def head_integral(x):
    """int_0^x t^3/(e^t-1) dt for 0 <= x < 2 (Bernoulli series)."""
    x = np.asarray(x, dtype=np.float64)
    acc = np.zeros_like(x)
    for k in range(_NB, -1, -1):
        acc = acc * x + _HEAD_COEF[k]
    return acc * x ** 3


def tail_integral(x):
    """int_x^inf t^3/(e^t-1) dt for x >= 2 (sum over the geometric expansion);
    +inf gives 0."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    fin = np.isfinite(x)
    xf = x[fin]
    acc = np.zeros_like(xf)
    for n in range(1, 64):
        en = np.exp(-n * xf)
        term = en * (xf ** 3 / n + 3 * xf ** 2 / n ** 2 + 6 * xf / n ** 3 + 6.0 / n ** 4)
        acc = acc + term
        if np.all(term <= 1e-18 * np.maximum(acc, 1e-300)):
            break
    out[fin] = acc
    return out


def _interval_integral(lo, hi):
    """int_lo^hi t^3/(e^t-1) dt elementwise, lo <= hi, hi may be inf."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    out = np.empty(np.broadcast(lo, hi).shape)
    lo, hi = np.broadcast_arrays(lo, hi)
    both_tail = lo >= X_SWITCH
    both_head = hi < X_SWITCH
    mixed = ~(both_tail | both_head)
    out[both_tail] = tail_integral(lo[both_tail]) - tail_integral(hi[both_tail])
    out[both_head] = head_integral(hi[both_head]) - head_integral(lo[both_head])
    out[mixed] = (TOTAL - tail_integral(hi[mixed])) - head_integral(lo[mixed])
    return out


def _x4_over_expm1(x):
    """x^4 / (e^x - 1), with the limits 0 at x = 0 and x = inf."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    ok = np.isfinite(x) & (x > 0)
    xo = x[ok]
    out[ok] = xo ** 4 * np.exp(-xo) / (-np.expm1(-xo))
    return out


def planck_groups(nu_edges, T, aR, c):
    """B_g(T_i) for every group g and cell i -> array [ng, nx]."""
    nu_edges = np.asarray(nu_edges, dtype=np.float64)
    T = np.atleast_1d(np.asarray(T, dtype=np.float64))
    with np.errstate(over="ignore", invalid="ignore", divide="ignore"):
        x = nu_edges[:, None] / T[None, :]  # [ng+1, nx]
    val = _interval_integral(x[:-1], x[1:])
    scale = aR * c * T ** 4 / 2.0 / TOTAL
    return val * scale[None, :]


def planck_groups_dT(nu_edges, T, aR, c):
    """dB_g/dT at T_i -> [ng, nx].

    d/dT of (a_R c T^4 / 2)(15/pi^4) int_{nu_g/T}^{nu_{g+1}/T} ... gives
    4 B_g / T - (a_R c T^4 / 2)(15/pi^4)(1/T) [x^4/(e^x-1)]_{x_g}^{x_{g+1}}.
    """
    nu_edges = np.asarray(nu_edges, dtype=np.float64)
    T = np.atleast_1d(np.asarray(T, dtype=np.float64))
    B = planck_groups(nu_edges, T, aR, c)
    with np.errstate(over="ignore", invalid="ignore", divide="ignore"):
        x = nu_edges[:, None] / T[None, :]
    g = _x4_over_expm1(x)
    scale = aR * c * T ** 4 / 2.0 / TOTAL
    return 4.0 * B / T[None, :] - scale[None, :] / T[None, :] * (g[1:] - g[:-1])


def opacity(nu_center, C_cell, T):
    """kappa_g(T_i) = C_i / nu_g^3 * (1 - exp(-nu_g / T_i)) -> [ng, nx]."""
    nu = np.asarray(nu_center, dtype=np.float64)[:, None]
    T = np.atleast_1d(np.asarray(T, dtype=np.float64))[None, :]
    C = np.asarray(C_cell, dtype=np.float64)[None, :]
    return C / nu ** 3 * (-np.expm1(-nu / T))


def opacity_dT(nu_center, C_cell, T):
    """d kappa_g / dT = -C_i / nu_g^2 * exp(-nu_g / T_i) / T_i^2 -> [ng, nx]."""
    nu = np.asarray(nu_center, dtype=np.float64)[:, None]
    T = np.atleast_1d(np.asarray(T, dtype=np.float64))[None, :]
    C = np.asarray(C_cell, dtype=np.float64)[None, :]
    return -C / nu ** 2 * np.exp(-nu / T) / T ** 2


def boundary_intensity(nu_edges, T_b, aR, c):
    """Isotropic incoming Planck intensity per group, I_g = B_g(T_b); vacuum
    (T_b <= 0) gives zeros.  -> [ng]"""
    ng = len(nu_edges) - 1
    if T_b <= 0.0:
        return np.zeros(ng)
    return planck_groups(nu_edges, np.array([T_b]), aR, c)[:, 0]
