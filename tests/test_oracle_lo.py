"""Pins of the oracle's low-order solves, restriction and grey/MEB Newton (CPU).

* the tridiagonal elimination agrees with a dense solve of the un-eliminated
  system (balance per cell, first moment per edge, two boundary conditions);
* restriction is an exact projection: at a fixed temperature the coarse and
  grey solutions equal the block sums of the finer solution (the paper's
  spectrum-consistency property of multigrid in frequency);
* one grey Newton update conserves energy to roundoff: the change of radiation
  plus material energy equals the net boundary inflow.
"""
import dataclasses

import numpy as np
import pytest

from oracle import lo
from oracle.restrict import restrict
from paper_2011_05427_amd import inputs

C = inputs.C_LIGHT


def random_level(rng, P, nx, *, coarse=False):
    a = rng.uniform(0.2, 0.6, (P, nx + 1))
    b = rng.uniform(0.2, 0.6, (P, nx + 1))
    return lo.Level(
        sigE=10 ** rng.uniform(-2, 3, (P, nx)),
        emis=rng.uniform(0, 5, (P, nx)),
        a=a, b=b,
        sigR=10 ** rng.uniform(-2, 3, (P, nx + 1)),
        C=np.stack([-rng.uniform(0.3, 0.7, P), rng.uniform(0.3, 0.7, P)], axis=1),
        Phi=np.stack([rng.uniform(0, 3, P), -rng.uniform(0, 0.1, P)], axis=1),
        Eold=rng.uniform(0, 2, (P, nx)),
        Fold=rng.uniform(-1, 1, (P, nx + 1)),
    )


def dense_solve(lv, dx, c, dt):
    """Unknowns: u = (E_1/2, E_0..E_nx-1, E_nx+1/2) then F_0..F_nx."""
    P, nx = lv.sigE.shape
    h = lo.edge_lengths(dx)
    n = (nx + 2) + (nx + 1)
    out_u, out_F = [], []
    for p in range(P):
        M = np.zeros((n, n))
        r = np.zeros(n)
        row = 0
        iF = lambda e: nx + 2 + e
        for i in range(nx):  # balance of cell i
            M[row, 1 + i] = dx[i] / dt + c * lv.sigE[p, i] * dx[i]
            M[row, iF(i + 1)] += 1.0
            M[row, iF(i)] -= 1.0
            r[row] = dx[i] * lv.emis[p, i] + dx[i] / dt * lv.Eold[p, i]
            row += 1
        for e in range(nx + 1):  # first moment on edge e: E_L = u[e], E_R = u[e+1]
            M[row, iF(e)] = h[e] / (c * dt) + lv.sigR[p, e] * h[e]
            M[row, e + 1] += c * lv.a[p, e]
            M[row, e] -= c * lv.b[p, e]
            r[row] = h[e] / (c * dt) * lv.Fold[p, e]
            row += 1
        M[row, iF(0)] = 1.0
        M[row, 0] = -c * lv.C[p, 0]
        r[row] = lv.Phi[p, 0]
        row += 1
        M[row, iF(nx)] = 1.0
        M[row, nx + 1] = -c * lv.C[p, 1]
        r[row] = lv.Phi[p, 1]
        x = np.linalg.solve(M, r)
        out_u.append(x[:nx + 2])
        out_F.append(x[nx + 2:])
    return np.array(out_u), np.array(out_F)


@pytest.mark.parametrize("nx", [1, 2, 7, 20])
def test_tridiagonal_matches_dense(nx):
    rng = np.random.default_rng(nx)
    dx = rng.uniform(0.05, 0.3, nx)
    lv = random_level(rng, 3, nx)
    sol = lo.solve_level(lv, dx, C, 0.01)
    u, F = dense_solve(lv, dx, C, 0.01)
    np.testing.assert_allclose(sol.E_ext(), u, rtol=1e-11)
    np.testing.assert_allclose(sol.F, F, rtol=1e-10, atol=1e-12 * np.max(np.abs(F)))
    res = lo.residual(lv, sol, dx, C, 0.01)
    assert max(res) < 1e-12


def _fine_from_physics(rng, G, nx, dx, separate_sigR=False):
    """A fine level built like the solver builds it: cell factors, point
    opacities, emission 2 kappa B, dx-weighted edge opacity (or, with
    separate_sigR, a Rosseland opacity and an emission of their own, as the
    group averages of a spectral opacity give)."""
    from oracle.moments import Factors
    kappa = 10 ** rng.uniform(-2, 4, (G, nx))
    B = rng.uniform(0.0, 1.0, (G, nx))
    fac = Factors(f=rng.uniform(0.25, 0.5, (G, nx)), f_bnd=rng.uniform(0.25, 0.6, (G, 2)),
                  C=np.stack([-rng.uniform(0.4, 0.6, G), rng.uniform(0.4, 0.6, G)], axis=1),
                  Phi=np.stack([rng.uniform(0, 2, G), np.zeros(G)], axis=1))
    Eo, Fo = rng.uniform(0, 1, (G, nx)), rng.uniform(-0.5, 0.5, (G, nx + 1))
    if separate_sigR:
        return lo.fine_level(kappa, B, fac, Eo, Fo, dx, emis=rng.uniform(0, 2, (G, nx)) * kappa,
                             sigR=kappa * 10 ** rng.uniform(-1, 1, (G, nx)))
    return lo.fine_level(kappa, B, fac, Eo, Fo, dx)


@pytest.mark.parametrize("G,P,sepR", [(16, 4, False), (16, 1, False), (32, 8, False), (12, 3, False),
                                      (16, 4, True), (12, 1, True)])
def test_restriction_is_exact_projection(G, P, sepR):
    rng = np.random.default_rng(G * 100 + P)
    nx = 9
    dx = rng.uniform(0.05, 0.2, nx)
    fine = _fine_from_physics(rng, G, nx, dx, sepR)
    fs = lo.solve_level(fine, dx, C, 0.004)
    coarse = restrict(fine, fs, P, dx, C)
    cs = lo.solve_level(coarse, dx, C, 0.004)
    r = G // P
    sums = lambda x: x.reshape((P, r) + x.shape[1:]).sum(axis=1)
    np.testing.assert_allclose(cs.E, sums(fs.E), rtol=1e-12)
    np.testing.assert_allclose(cs.Ebnd, sums(fs.Ebnd), rtol=1e-12)
    np.testing.assert_allclose(cs.F, sums(fs.F), rtol=1e-10, atol=1e-12 * np.max(np.abs(fs.F)))
    # coarse -> grey and fine -> grey both reproduce the total
    for lv, sol in ((coarse, cs), (fine, fs)):
        grey = restrict(lv, sol, 1, dx, C)
        gs = lo.solve_level(grey, dx, C, 0.004)
        np.testing.assert_allclose(gs.E[0], fs.E.sum(axis=0), rtol=1e-12)
        np.testing.assert_allclose(gs.F[0], fs.F.sum(axis=0), rtol=1e-10, atol=1e-12 * np.max(np.abs(fs.F)))


def test_compensation_without_edge_length_breaks_projection(monkeypatch):
    """The printed xi (without the edge length h_e) is not an exact projection
    on a non-trivial mesh; the reading that includes h_e is (test above)."""
    import oracle.restrict as rmod
    rng = np.random.default_rng(5)
    G, P, nx = 16, 4, 8
    dx = rng.uniform(0.05, 0.2, nx)
    fine = _fine_from_physics(rng, G, nx, dx)
    fs = lo.solve_level(fine, dx, C, 0.004)
    monkeypatch.setattr(rmod, "edge_lengths", lambda d: np.ones(len(d) + 1))
    coarse = rmod.restrict(fine, fs, P, dx, C)
    cs = lo.solve_level(coarse, dx, C, 0.004)
    sums = fs.E.reshape(P, G // P, nx).sum(axis=1)
    assert np.max(np.abs(cs.E - sums) / sums) > 1e-6


def test_grey_newton_conserves_energy():
    rng = np.random.default_rng(11)
    nx = 12
    dx = rng.uniform(0.05, 0.2, nx)
    grey = random_level(rng, 1, nx)
    Told = rng.uniform(0.1, 0.5, nx)
    Tstar = Told * rng.uniform(1.0, 1.3, nx)
    S = rng.uniform(0.5, 2.0, nx)
    dS = rng.uniform(1.0, 10.0, nx)
    Estar = rng.uniform(0.1, 1.0, nx)
    D = rng.uniform(-1.0, 1.0, nx)
    cv, dt = 0.5, 0.002
    gr = lo.grey_newton(grey, Tstar, Told, S, dS, Estar, D, cv, dx, C, dt)
    assert gr.n_floor == 0
    E, F = gr.sol.E[0], gr.sol.F[0]
    lhs = np.sum(dx * ((E - grey.Eold[0]) / dt + cv * (gr.T - Told) / dt))
    rhs = -(F[-1] - F[0])
    scale = np.sum(dx * (np.abs(E) + np.abs(grey.Eold[0]) + cv * (gr.T + Told)) / dt)
    assert abs(lhs - rhs) < 1e-13 * scale
    # the linearised MEB holds cell by cell
    dT = gr.T - Tstar
    meb = cv * (gr.T - Told) / dt - (C * grey.sigE[0] * E + C * D * Estar * dT - S - dS * dT)
    assert np.max(np.abs(meb)) < 1e-12 * np.max(cv * np.abs(gr.T) / dt)


@pytest.mark.parametrize("seed", [3, 4])
def test_steady_source_free_slab_matches_closed_form(seed):
    """Steady state (1/dt = 0), no absorption or emission, QD factors that vary
    from cell to cell and opacities that vary from cell to cell on a
    non-uniform mesh.  The continuous equations then give a constant flux F and
    c d(f E)/dx = -sigma F, so f E at a cell centre x_i is f_{1/2} E_{1/2} -
    (F/c) tau(x_i) with tau the optical depth from x = 0, and the two boundary
    conditions fix E_{1/2} and F.  The discrete first moment integrated
    between neighbouring cell centres with the dx-weighted edge opacity, and
    over the boundary half cells, reproduces this solution exactly at every
    cell centre and boundary; an edge length of dx_i, the arithmetic mean of
    the two opacities, or the QD factors attached to the wrong side of an
    edge do not."""
    from oracle.moments import Factors

    rng = np.random.default_rng(seed)
    nx = 9
    dx = rng.uniform(0.05, 0.5, nx)
    sig = 10 ** rng.uniform(-1, 1, nx)
    f = rng.uniform(0.25, 0.6, nx)
    fb = rng.uniform(0.3, 0.6, 2)
    Cm, Cp, Phim, Phip = -0.45, 0.55, 2.0, -0.3
    fac = Factors(f=f[None], f_bnd=fb[None], C=np.array([[Cm, Cp]]), Phi=np.array([[Phim, Phip]]))
    lv = lo.fine_level(sig[None], np.zeros((1, nx)), fac, np.zeros((1, nx)), np.zeros((1, nx + 1)), dx)
    lv = dataclasses.replace(lv, sigE=np.zeros((1, nx)), emis=np.zeros((1, nx)))
    sol = lo.solve_level(lv, dx, C, np.inf)

    tau_edge = np.concatenate([[0.0], np.cumsum(sig * dx)])
    tau_centre = tau_edge[:-1] + sig * dx / 2
    tauX = tau_edge[-1]
    # unknowns (E_{1/2}, F): F - c C^- E_{1/2} = Phi^-,
    # F - c C^+ E_{nx+1/2} = Phi^+ with f_{nx+1/2} E_{nx+1/2} = f_{1/2} E_{1/2} - F tau_X / c
    A = np.array([[-C * Cm, 1.0], [-C * Cp * fb[0] / fb[1], 1.0 + Cp * tauX / fb[1]]])
    E0, F = np.linalg.solve(A, [Phim, Phip])
    E_centre = (fb[0] * E0 - F * tau_centre / C) / f
    EX = (fb[0] * E0 - F * tauX / C) / fb[1]
    np.testing.assert_allclose(sol.E[0], E_centre, rtol=1e-12)
    np.testing.assert_allclose(sol.Ebnd[0], [E0, EX], rtol=1e-12)
    np.testing.assert_allclose(sol.F[0], np.full(nx + 1, F), rtol=1e-11)
