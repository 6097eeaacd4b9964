"""Pins of the oracle's SCB sweep and angular moments (CPU only).

Sweep: per-cell transmission of a pure absorber has the closed form
2 / ((1 + tau)^2 + 1) with tau = sigma dx / |mu| (the SCB 2x2 corner system with
no source); a constant solution is reproduced exactly; refining the mesh
converges to exp(-sigma X / |mu|) at second order; the mirror image of a problem
gives the mirror image of its solution.
Moments: quadrature exactness, isotropic factors (1/3, +/- C_iso) and the exact
boundary identity F = c C (E - E_in) + F_in of the paper's boundary condition.
"""
import numpy as np
import pytest

from oracle import moments
from oracle.sweep import sweep
from paper_2011_05427_amd import inputs

C = inputs.C_LIGHT


def _uniform(n, X=1.0):
    return np.linspace(0.0, X, n + 1)


@pytest.mark.parametrize("sig", [0.3, 2.0, 40.0])
def test_pure_absorber_cell_transmission(sig):
    mu, w = inputs.gauss_legendre(8)
    nx = 5
    x = _uniform(nx, 0.5)
    kappa = np.full((1, nx), sig)
    Bz = np.zeros((1, nx))
    Ip = np.zeros((1, 8, nx, 2))
    I = sweep(mu, x, kappa, Bz, Ip, np.ones(1), np.ones(1), C, np.inf)
    dx = x[1] - x[0]
    for m in range(8):
        tau = sig * dx / abs(mu[m])
        t = 2.0 / ((1 + tau) ** 2 + 1)
        if mu[m] > 0:
            out = I[0, m, :, 1]
            np.testing.assert_allclose(out, t ** np.arange(1, nx + 1), rtol=1e-14)
        else:
            out = I[0, m, ::-1, 0]
            np.testing.assert_allclose(out, t ** np.arange(1, nx + 1), rtol=1e-14)


def test_constant_solution_is_reproduced():
    mu, w = inputs.gauss_legendre(16)
    nx, G = 9, 3
    rng = np.random.default_rng(1)
    x = np.sort(np.concatenate([[0.0, 2.0], rng.uniform(0, 2.0, nx - 1)]))
    kappa = rng.uniform(0.1, 50.0, (G, nx))
    dt = 0.01
    Ic = np.array([0.7, 3.0, 1e-3])
    # q* = kappa B + I_prev/(c dt) must equal (kappa + 1/(c dt)) Ic in every corner
    Ip = np.broadcast_to(Ic[:, None, None, None], (G, 16, nx, 2)).copy()
    B = np.broadcast_to(Ic[:, None], (G, nx)).copy()
    I = sweep(mu, x, kappa, B, Ip, Ic, Ic, C, dt)
    np.testing.assert_allclose(I, np.broadcast_to(Ic[:, None, None, None], I.shape), rtol=2e-14)


def test_mesh_refinement_second_order():
    sig, X = 1.7, 1.0
    m_mu = np.array([0.6])
    errs = []
    for nx in (8, 16, 32, 64, 128):
        I = sweep(m_mu, _uniform(nx, X), np.full((1, nx), sig), np.zeros((1, nx)),
                  np.zeros((1, 1, nx, 2)), np.ones(1), np.ones(1), C, np.inf)
        errs.append(abs(I[0, 0, -1, 1] - np.exp(-sig * X / 0.6)))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(orders > 1.8) and orders[-1] > 1.95


def test_mirror_symmetry():
    mu, w = inputs.gauss_legendre(8)
    nx, G = 7, 2
    rng = np.random.default_rng(7)
    x = np.sort(np.concatenate([[0.0, 1.0], rng.uniform(0, 1.0, nx - 1)]))
    kappa = rng.uniform(0.5, 20, (G, nx))
    B = rng.uniform(0, 2, (G, nx))
    Ip = rng.uniform(0, 1, (G, 8, nx, 2))
    inl, inr = rng.uniform(0, 1, G), rng.uniform(0, 1, G)
    I = sweep(mu, x, kappa, B, Ip, inl, inr, C, 0.02)
    xm = (1.0 - x)[::-1]
    # mirror: cells reversed, corners swapped, directions reversed (mu ascending)
    Ipm = Ip[:, ::-1, ::-1, ::-1]
    Im = sweep(mu, xm, kappa[:, ::-1], B[:, ::-1], Ipm, inr, inl, C, 0.02)
    np.testing.assert_allclose(Im, I[:, ::-1, ::-1, ::-1], rtol=1e-13)


@pytest.mark.parametrize("n,ciso", [(8, 0.50576), (16, 0.50152), (32, 0.50039)])
def test_quadrature(n, ciso):
    mu, w = inputs.gauss_legendre(n)
    assert w.sum() == pytest.approx(2.0, rel=1e-15)
    for k in range(2 * n):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert np.sum(w * mu ** k) == pytest.approx(exact, abs=2e-15)
    f_iso, c_iso = moments.iso_factors(mu, w)
    assert f_iso == pytest.approx(1.0 / 3.0, abs=1e-15)
    assert c_iso == pytest.approx(ciso, abs=5e-6)


def test_isotropic_factors():
    mu, w = inputs.gauss_legendre(16)
    G, nx = 4, 6
    val = np.array([1.0, 0.2, 3.0, 0.0])
    I = np.broadcast_to(val[:, None, None, None], (G, 16, nx, 2)).copy()
    fac = moments.factors(mu, w, I, val, val, C)
    f_iso, c_iso = moments.iso_factors(mu, w)
    np.testing.assert_allclose(fac.f, 1.0 / 3.0, atol=1e-15)
    np.testing.assert_allclose(fac.f_bnd, 1.0 / 3.0, atol=1e-15)
    np.testing.assert_allclose(fac.C[:, 0], -c_iso, rtol=1e-15)
    np.testing.assert_allclose(fac.C[:, 1], c_iso, rtol=1e-15)
    E, F = moments.energy_flux(mu, w, I, C)
    np.testing.assert_allclose(F, 0.0, atol=1e-15)
    np.testing.assert_allclose(E, 2.0 * val[:, None] / C * np.ones((1, nx)), rtol=1e-15)
    assert fac.n_guard > 0  # the zero group used the isotropic defaults


def test_boundary_condition_identity():
    """F_edge = c C (E_edge - E_in) + F_in holds exactly for any intensity."""
    mu, w = inputs.gauss_legendre(8)
    G, nx = 3, 4
    rng = np.random.default_rng(3)
    I = rng.uniform(0.1, 2.0, (G, 8, nx, 2))
    inl, inr = rng.uniform(0, 1, G), rng.uniform(0, 1, G)
    fac = moments.factors(mu, w, I, inl, inr, C)
    pos = mu > 0
    psi_l = np.where(pos[None, :], inl[:, None], I[:, :, 0, 0])
    psi_r = np.where(pos[None, :], I[:, :, -1, 1], inr[:, None])
    for psi, side in ((psi_l, 0), (psi_r, 1)):
        E_edge = psi @ w / C
        F_edge = psi @ (w * mu)
        np.testing.assert_allclose(F_edge, C * fac.C[:, side] * E_edge + fac.Phi[:, side], rtol=1e-13)
        np.testing.assert_allclose(fac.f_bnd[:, side], psi @ (w * mu * mu) / (psi @ w), rtol=1e-14)


def test_cell_factor_converges_at_second_order_to_exact_eddington_factor():
    """Pure absorber lit from the left by unit isotropic radiation: the exact
    intensity is exp(-sigma x / mu) for mu > 0 and 0 for mu < 0, so the exact
    Eddington factor at x is sum_{mu>0} w mu^2 e^(-sigma x/mu) / sum_{mu>0} w
    e^(-sigma x/mu), and the outgoing boundary factor at X is the same ratio
    with mu instead of mu^2.  The discrete factors (cell average of the two
    corner values) converge to them at second order under refinement; any
    other corner weighting of the cell value converges only at first order."""
    mu, w = inputs.gauss_legendre(8)
    pos = mu > 0
    sig, X = 2.0, 1.0

    def errors(nx):
        x = _uniform(nx, X)
        xc = 0.5 * (x[:-1] + x[1:])
        I = sweep(mu, x, np.full((1, nx), sig), np.zeros((1, nx)), np.zeros((1, 8, nx, 2)),
                  np.ones(1), np.zeros(1), C, np.inf)
        fac = moments.factors(mu, w, I, np.ones(1), np.zeros(1), C)
        att = np.exp(-sig * xc[None, :] / mu[pos][:, None])
        f_exact = (w[pos] * mu[pos] ** 2) @ att / (w[pos] @ att)
        attX = np.exp(-sig * X / mu[pos])
        C_exact = (w[pos] * mu[pos]) @ attX / (w[pos] @ attX)
        fX_exact = (w[pos] * mu[pos] ** 2) @ attX / (w[pos] @ attX)
        return (np.max(np.abs(fac.f[0] - f_exact)), abs(fac.C[0, 1] - C_exact),
                abs(fac.f_bnd[0, 1] - fX_exact))

    e80, e160 = errors(80), errors(160)
    orders = [np.log2(a / b) for a, b in zip(e80, e160)]
    assert e160[0] < 1e-4 and orders[0] > 1.8, (e160, orders)
    assert e160[1] < 5e-5 and orders[1] > 1.8, (e160, orders)
    assert e160[2] < 5e-5 and orders[2] > 1.8, (e160, orders)
