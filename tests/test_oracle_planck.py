"""Pins of the oracle's Planck group integrals and opacity law (CPU only).

The group integral is checked against its definition by adaptive quadrature of
the Planck function, against the normalisation implied by the paper's
definition of B as 2 pi times the Planck function (sum over groups covering
[0, inf) equals a_R c T^4 / 2), and the derivatives against finite differences.
"""
import math

import numpy as np
import pytest
from scipy.integrate import quad

from oracle import planck
from paper_2011_05427_amd import inputs

AR, C = inputs.A_RAD, inputs.C_LIGHT


def _planck_density(nu, T):
    # (a_R c / 2) (15/pi^4) nu^3 / (exp(nu/T) - 1): 2 pi x Planck in keV units
    if nu == 0.0:
        return 0.0
    return AR * C / 2.0 * 15.0 / math.pi ** 4 * nu ** 3 / math.expm1(nu / T)


@pytest.mark.parametrize("T", [1e-3, 0.02, 0.3, 1.0, 1.5])
def test_group_sum_is_total_emission(T):
    edges, _ = inputs.log_groups(64, 0.01, 100.0)
    B = planck.planck_groups(edges, np.array([T]), AR, C)[:, 0]
    assert np.all(B >= 0)
    np.testing.assert_allclose(B.sum(), AR * C * T ** 4 / 2.0, rtol=2e-14)


@pytest.mark.parametrize("T", [0.05, 0.4, 1.0])
def test_group_integral_matches_quadrature(T):
    edges = np.array([0.0, 0.013, 0.05, 0.2, 0.7, 1.1, 3.0, 7.5, 20.0])
    B = planck.planck_groups(edges, np.array([T]), AR, C)[:, 0]
    for g in range(len(edges) - 1):
        ref, err = quad(_planck_density, edges[g], edges[g + 1], args=(T,), epsabs=0, epsrel=1e-13, limit=200)
        assert B[g] == pytest.approx(ref, rel=1e-12, abs=1e-300)


def test_head_and_tail_meet_at_switch():
    for x in (1.5, 2.0, 2.5):
        assert planck.head_integral(np.array([x]))[0] + planck.tail_integral(np.array([x]))[0] == \
            pytest.approx(math.pi ** 4 / 15, rel=2e-15)


def test_tail_of_cold_groups_underflows_to_zero():
    edges, _ = inputs.log_groups(16, 0.01, 100.0)
    B = planck.planck_groups(edges, np.array([1e-3]), AR, C)[:, 0]
    assert B[-1] == 0.0 and np.isfinite(B).all()


@pytest.mark.parametrize("T", [0.01, 0.3, 1.2])
def test_planck_derivative_matches_finite_difference(T):
    edges, _ = inputs.log_groups(24, 0.01, 100.0)
    h = 1e-6 * T
    fd = (planck.planck_groups(edges, np.array([T + h]), AR, C) - planck.planck_groups(edges, np.array([T - h]), AR, C)) / (2 * h)
    an = planck.planck_groups_dT(edges, np.array([T]), AR, C)
    scale = np.max(np.abs(an))
    np.testing.assert_allclose(an, fd, rtol=1e-6, atol=1e-9 * scale)
    # total: d/dT (a_R c T^4 / 2) = 2 a_R c T^3
    assert an.sum() == pytest.approx(2 * AR * C * T ** 3, rel=1e-12)


def test_opacity_law_and_derivative():
    nu = np.array([0.01, 0.3, 5.0, 80.0])
    Cc = np.array([27.0, 2.7])
    T = np.array([0.001, 0.7])
    k = planck.opacity(nu, Cc, T)
    ref = Cc[None, :] / nu[:, None] ** 3 * (1 - np.exp(-nu[:, None] / T[None, :]))
    np.testing.assert_allclose(k, ref, rtol=1e-14)
    h = 1e-6 * T
    fd = (planck.opacity(nu, Cc, T + h) - planck.opacity(nu, Cc, T - h)) / (2 * h)
    np.testing.assert_allclose(planck.opacity_dT(nu, Cc, T), fd, rtol=1e-6, atol=1e-30)
