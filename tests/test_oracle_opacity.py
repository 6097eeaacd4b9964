"""Pins of the oracle's group opacities (CPU only): the spectral averages of
Sec. 2 (sigma_B,g, sigma_E,g) and Sec. 3.1 (Rosseland sigma_R,g) against what
the mathematics fixes independently of the quadrature:

* a constant spectral opacity gives every group average equal to it;
* a narrow group gives the point value at its centre (second order);
* over the whole spectrum the FC law has closed forms: the Planck mean
  15 C / (pi^4 T^3), sigma_E = 15 C (psi(1 + T_r/T) + gamma) / (pi^4 T_r^3)
  (digamma function psi, Euler's gamma), and for T << T_r the Rosseland mean
  C 4! zeta(4) / (7! zeta(7) T_r^3);
* the group emission sigma_B,g B_g equals its closed form, and sigma_E at
  T_r = T times B_g(T) equals it as well;
* averages are consistent under splitting a group (weighted means add up);
* the closed-form emission derivative agrees with finite differences and the
  emission of all groups sums to C (a_R c / 2)(15 / pi^4) T.
"""
import math

import numpy as np
import pytest
from scipy.special import digamma, zeta

from oracle import opacity, planck
from paper_2011_05427_amd import inputs

AR, C = inputs.A_RAD, inputs.C_LIGHT
K = AR * C / 2 * 15 / math.pi ** 4


@pytest.mark.parametrize("a,b", [(0.0, 0.05), (0.3, 0.35), (2.0, 9.0), (10.0, np.inf)])
def test_constant_opacity_gives_itself(a, b):
    sig = lambda nu, T: 3.7
    for T, Tr in ((0.1, 0.1), (0.05, 0.8), (1.0, 0.02)):
        assert abs(opacity.group_sigma_E(a, b, T, Tr, sig) - 3.7) < 1e-13 * 3.7
        assert abs(opacity.group_sigma_B(a, b, T, sig) - 3.7) < 1e-13 * 3.7
        assert abs(opacity.group_sigma_R(a, b, T, Tr, sig) - 3.7) < 1e-13 * 3.7


def test_narrow_group_tends_to_point_value_at_second_order():
    sig = opacity.fc_sigma(27.0)
    T, Tr, nu = 0.3, 0.7, 1.1
    errs = []
    for d in (0.02, 0.01):
        a, b = nu * (1 - d), nu * (1 + d)
        pt = sig(nu, T)
        errs.append([abs(f - pt) / pt for f in (opacity.group_sigma_E(a, b, T, Tr, sig),
                                               opacity.group_sigma_B(a, b, T, sig),
                                               opacity.group_sigma_R(a, b, T, Tr, sig))])
    for e1, e2 in zip(*errs):
        assert e2 < 1e-3 and 3.6 < e1 / e2 < 4.4, errs


@pytest.mark.parametrize("T,Tr", [(0.1, 0.1), (0.01, 0.5), (0.8, 0.2)])
def test_whole_spectrum_closed_forms(T, Tr):
    Cz = 27.0
    sig = opacity.fc_sigma(Cz)
    planck_mean = 15 * Cz / (math.pi ** 4 * T ** 3)
    assert abs(opacity.group_sigma_B(0.0, np.inf, T, sig) / planck_mean - 1) < 1e-12
    rho = Tr / T
    sE = 15 * Cz * (digamma(1 + rho) + np.euler_gamma) / (math.pi ** 4 * Tr ** 3)
    assert abs(opacity.group_sigma_E(0.0, np.inf, T, Tr, sig) / sE - 1) < 1e-12
    # Rosseland mean with the stimulated-emission factor at 1 (T << T_r)
    sR = Cz * math.factorial(4) * zeta(4) / (math.factorial(7) * zeta(7) * Tr ** 3)
    assert abs(opacity.group_sigma_R(0.0, np.inf, Tr * 1e-6, Tr, sig) / sR - 1) < 1e-11


def test_group_emission_closed_form_and_equal_temperatures():
    slab = inputs.fc_slab()
    edges = slab.nu_edges[::16].copy()  # 17 edges: 0, ..., inf
    edges[-1] = np.inf
    T = np.array([0.001, 0.05, 0.3, 1.0])
    em = opacity.emission(edges, np.full(4, 27.0), T, AR, C)
    B = planck.planck_groups(edges, T, AR, C)
    sig = opacity.fc_sigma(27.0)
    for i, t in enumerate(T):
        for g in range(len(edges) - 1):
            if B[g, i] < 1e-250:
                continue
            sb = opacity.group_sigma_B(edges[g], edges[g + 1], t, sig)
            se = opacity.group_sigma_E(edges[g], edges[g + 1], t, t, sig)
            assert abs(sb * B[g, i] / em[g, i] - 1) < 1e-11, (g, t)
            assert abs(se * B[g, i] / em[g, i] - 1) < 1e-11, (g, t)
    np.testing.assert_allclose(em.sum(axis=0), 27.0 * K * T, rtol=1e-14)


def test_averages_are_consistent_when_a_group_is_split():
    sig = opacity.fc_sigma(10.0)
    T, Tr = 0.2, 0.45
    a, m, b = 0.1, 0.37, 1.3
    # sigma_E weighted by the Planck integral at T_r adds up
    Bw = lambda lo, hi: planck.planck_groups(np.array([lo, hi]), np.array([Tr]), AR, C)[0, 0]
    lhs = opacity.group_sigma_E(a, b, T, Tr, sig) * Bw(a, b)
    rhs = opacity.group_sigma_E(a, m, T, Tr, sig) * Bw(a, m) + opacity.group_sigma_E(m, b, T, Tr, sig) * Bw(m, b)
    assert abs(lhs / rhs - 1) < 1e-12
    # the Rosseland average is harmonic: integral of dB/dT / sigma_R adds up
    dB = lambda lo, hi: planck.planck_groups_dT(np.array([lo, hi]), np.array([Tr]), AR, C)[0, 0]
    lhs = dB(a, b) / opacity.group_sigma_R(a, b, T, Tr, sig)
    rhs = dB(a, m) / opacity.group_sigma_R(a, m, T, Tr, sig) + dB(m, b) / opacity.group_sigma_R(m, b, T, Tr, sig)
    assert abs(lhs / rhs - 1) < 1e-12


def test_emission_derivative():
    edges = np.concatenate([[0.0], np.logspace(-3, 1, 20), [np.inf]])
    Cc = np.array([27.0, 2.7])
    T = np.array([0.02, 0.6])
    d = opacity.emission_dT(edges, Cc, T, AR, C)
    h = 1e-6 * T
    fd = (opacity.emission(edges, Cc, T + h, AR, C) - opacity.emission(edges, Cc, T - h, AR, C)) / (2 * h)
    np.testing.assert_allclose(d, fd, rtol=1e-7, atol=1e-9 * np.abs(d).max())
    np.testing.assert_allclose(d.sum(axis=0), Cc * K, rtol=1e-14)


def test_spectral_tables_shapes_and_temperature_reading():
    edges = np.array([0.0, 0.01, 0.1, 1.0, np.inf])
    T = np.array([0.05, 0.3])
    Tr = opacity.radiation_temperature(AR * np.array([0.2, 0.3]) ** 4, AR)
    np.testing.assert_allclose(Tr, [0.2, 0.3], rtol=1e-15)
    sE, src, sR = opacity.spectral_tables(edges, np.array([27.0, 27.0]), T, Tr, AR, C)
    assert sE.shape == src.shape == sR.shape == (4, 2)
    assert np.all(sE > 0) and np.all(sR > 0) and np.all(src > 0)
