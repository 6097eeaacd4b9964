"""Discrete low-order QD (LOQD) equations at one frequency level (oracle).

TEST INFRASTRUCTURE ONLY.

Paper Sec. 5, Eqs. mloqd1-d / mloqd2-d (fine grid) and mloqd1-d-gamma /
mloqd2-d-gamma (coarse grids).  Cells i = 0..nx-1 have widths dx_i; edges
e = 0..nx sit at x_edges[e].  Every edge e carries one first-moment equation
that links the energy density on its left, E_L(e), and on its right, E_R(e):

  (h_e / (c dt)) (F_e - F_e^old) + c (a_e E_R(e) - b_e E_L(e)) + sigma_R,e h_e F_e = 0

with h_e = (dx_{e-1} + dx_e) / 2 for interior edges (the first moment is
integrated between neighbouring cell centres) and the two boundary half cells
h_0 = dx_0 / 2, h_nx = dx_{nx-1} / 2, whose outer unknowns are the boundary
energy densities E_{1/2}, E_{nx+1/2}.  On the fine grid a_e and b_e are the QD
factors of the neighbouring cells (or the boundary edge factors); on coarse
grids they carry the upwind-split compensation terms (a = f + eta_hat on the
right, b = f + eta_check on the left).  The interior edge opacity is the
dx-weighted average of the cell values (paper, below Eq. mloqd2-d).

Every cell carries the photon balance (Eq. mloqd1-d, with the emission 2
sigma_B B of Eq. mloqd-1):

  (dx_i / dt) (E_i - E_i^old) + F_{i+1} - F_i + c sigma_E,i dx_i E_i = dx_i e_i

and the boundary conditions (Eq. mloqd-bcs) close the system:
  F_0 = c C^- E_{1/2} + Phi^-,   F_nx = c C^+ E_{nx+1/2} + Phi^+.

Eliminating each F_e through its own first-moment equation leaves a tridiagonal
system in u = (E_{1/2}, E_0, ..., E_{nx-1}, E_{nx+1/2}); it is solved here with
LAPACK's banded solver (partial pivoting), then F is recovered.
"""
from __future__ import annotations

import dataclasses

import numpy as np
from scipy.linalg import solve_banded


@dataclasses.dataclass
class Level:
    """Coefficients of the LOQD system of one frequency level with P groups."""

    sigE: np.ndarray  # [P, nx]
    emis: np.ndarray  # [P, nx] emission e_i (sum of 2 kappa B over the group's fine groups)
    a: np.ndarray  # [P, nx+1] coefficient of E_R(e)
    b: np.ndarray  # [P, nx+1] coefficient of E_L(e)
    sigR: np.ndarray  # [P, nx+1] edge opacity
    C: np.ndarray  # [P, 2]
    Phi: np.ndarray  # [P, 2]
    Eold: np.ndarray  # [P, nx]
    Fold: np.ndarray  # [P, nx+1]

    @property
    def P(self):
        return self.sigE.shape[0]


@dataclasses.dataclass
class LOSolution:
    E: np.ndarray  # [P, nx]
    F: np.ndarray  # [P, nx+1]
    Ebnd: np.ndarray  # [P, 2]

    def E_ext(self):
        """u = (E_{1/2}, E_0..E_{nx-1}, E_{nx+1/2}) -> [P, nx+2]; E_L(e) = u[e], E_R(e) = u[e+1]."""
        return np.concatenate([self.Ebnd[:, :1], self.E, self.Ebnd[:, 1:]], axis=1)


def edge_lengths(dx):
    dx = np.asarray(dx, dtype=np.float64)
    h = np.empty(len(dx) + 1)
    h[0] = dx[0] / 2.0
    h[-1] = dx[-1] / 2.0
    h[1:-1] = 0.5 * (dx[:-1] + dx[1:])
    return h


def edge_opacity(sig_cell, dx):
    """Edge opacity: dx-weighted average of the two neighbouring cells inside,
    the adjacent cell value on the two boundary edges.  [P, nx] -> [P, nx+1]"""
    dx = np.asarray(dx, dtype=np.float64)
    P, nx = sig_cell.shape
    out = np.empty((P, nx + 1))
    out[:, 0] = sig_cell[:, 0]
    out[:, -1] = sig_cell[:, -1]
    out[:, 1:-1] = (sig_cell[:, :-1] * dx[:-1] + sig_cell[:, 1:] * dx[1:]) / (dx[:-1] + dx[1:])
    return out


def fine_level(kappa, B, fac, Eold, Fold, dx, emis=None, sigR=None):
    """Fine-grid (Omega^1) coefficients from the opacity / Planck tables at the
    current temperature and the QD factors of the last sweep.  Point law
    (default): sigma_E = sigma_R = kappa and emission 2 kappa B.  With the
    group averages of the spectral opacity, kappa is sigma_E,g, `emis` the
    emission 2 sigma_B,g B_g and `sigR` the cell values of sigma_R,g."""
    G, nx = kappa.shape
    f_ext = np.concatenate([fac.f_bnd[:, :1], fac.f, fac.f_bnd[:, 1:]], axis=1)  # [G, nx+2]
    return Level(
        sigE=kappa.copy(),
        emis=2.0 * kappa * B if emis is None else np.array(emis, dtype=np.float64),
        a=f_ext[:, 1:].copy(),
        b=f_ext[:, :-1].copy(),
        sigR=edge_opacity(kappa if sigR is None else np.asarray(sigR, dtype=np.float64), dx),
        C=fac.C.copy(),
        Phi=fac.Phi.copy(),
        Eold=np.array(Eold, dtype=np.float64),
        Fold=np.array(Fold, dtype=np.float64),
    )


def assemble(lv: Level, dx, c, dt):
    """Tridiagonal system per group: returns (sub, diag, sup, rhs), each [P, nx+2],
    plus the per-edge (k, A) used to recover the fluxes."""
    dx = np.asarray(dx, dtype=np.float64)
    P, nx = lv.sigE.shape
    h = edge_lengths(dx)
    A = h / (c * dt)  # [nx+1]
    k = 1.0 / (A[None, :] + lv.sigR * h[None, :])  # [P, nx+1]
    n = nx + 2
    sub = np.zeros((P, n))
    diag = np.zeros((P, n))
    sup = np.zeros((P, n))
    rhs = np.zeros((P, n))
    # F_e = k_e (A_e Fold_e - c a_e u_{e+1} + c b_e u_e)
    # left boundary row: F_0 - c C^- u_0 = Phi^-
    diag[:, 0] = c * k[:, 0] * lv.b[:, 0] - c * lv.C[:, 0]
    sup[:, 0] = -c * k[:, 0] * lv.a[:, 0]
    rhs[:, 0] = lv.Phi[:, 0] - k[:, 0] * A[0] * lv.Fold[:, 0]
    # cell rows j = i + 1: balance with F_{e=j} on the right, F_{e=j-1} on the left
    j = np.arange(1, nx + 1)
    i = j - 1
    diag[:, j] = (dx[i] / dt + c * lv.sigE[:, i] * dx[i]
                  + c * k[:, j] * lv.b[:, j] + c * k[:, j - 1] * lv.a[:, j - 1])
    sub[:, j] = -c * k[:, j - 1] * lv.b[:, j - 1]
    sup[:, j] = -c * k[:, j] * lv.a[:, j]
    rhs[:, j] = (dx[i] * lv.emis[:, i] + dx[i] / dt * lv.Eold[:, i]
                 - k[:, j] * A[j] * lv.Fold[:, j] + k[:, j - 1] * A[j - 1] * lv.Fold[:, j - 1])
    # right boundary row: c C^+ u_{nx+1} - F_nx = -Phi^+
    diag[:, nx + 1] = c * k[:, nx] * lv.a[:, nx] + c * lv.C[:, 1]
    sub[:, nx + 1] = -c * k[:, nx] * lv.b[:, nx]
    rhs[:, nx + 1] = k[:, nx] * A[nx] * lv.Fold[:, nx] - lv.Phi[:, 1]
    return sub, diag, sup, rhs, k, A


def fluxes(lv: Level, u, k, A, c):
    """F_e from the edge first-moment equations, u = [P, nx+2]."""
    return k * (A[None, :] * lv.Fold - c * lv.a * u[:, 1:] + c * lv.b * u[:, :-1])


def solve_level(lv: Level, dx, c, dt) -> LOSolution:
    """Solve the LOQD equations of every group of one level."""
    sub, diag, sup, rhs, k, A = assemble(lv, dx, c, dt)
    P, n = diag.shape
    u = np.empty((P, n))
    ab = np.zeros((3, n))
    for p in range(P):
        ab[0, 1:] = sup[p, :-1]
        ab[1, :] = diag[p]
        ab[2, :-1] = sub[p, 1:]
        u[p] = solve_banded((1, 1), ab, rhs[p])
    F = fluxes(lv, u, k, A, c)
    return LOSolution(E=u[:, 1:-1].copy(), F=F, Ebnd=np.stack([u[:, 0], u[:, -1]], axis=1))


def residual(lv: Level, sol: LOSolution, dx, c, dt):
    """Residuals of the un-eliminated equations (balance per cell, first moment
    per edge, the two boundary conditions), each scaled by its largest term."""
    dx = np.asarray(dx, dtype=np.float64)
    h = edge_lengths(dx)
    u = sol.E_ext()
    E, F = sol.E, sol.F
    bal = (dx / dt) * (E - lv.Eold) + F[:, 1:] - F[:, :-1] + c * lv.sigE * dx * E - dx * lv.emis
    bal_s = np.maximum.reduce([np.abs((dx / dt) * E), np.abs((dx / dt) * lv.Eold), np.abs(F[:, 1:]),
                               np.abs(F[:, :-1]), np.abs(c * lv.sigE * dx * E), np.abs(dx * lv.emis)])
    fm = (h / (c * dt)) * (F - lv.Fold) + c * (lv.a * u[:, 1:] - lv.b * u[:, :-1]) + lv.sigR * h * F
    fm_s = np.maximum.reduce([np.abs((h / (c * dt)) * F), np.abs((h / (c * dt)) * lv.Fold),
                              np.abs(c * lv.a * u[:, 1:]), np.abs(c * lv.b * u[:, :-1]),
                              np.abs(lv.sigR * h * F)])
    bcl = F[:, 0] - (c * lv.C[:, 0] * u[:, 0] + lv.Phi[:, 0])
    bcr = F[:, -1] - (c * lv.C[:, 1] * u[:, -1] + lv.Phi[:, 1])
    bcl_s = np.maximum(np.abs(F[:, 0]), np.abs(c * lv.C[:, 0] * u[:, 0]) + np.abs(lv.Phi[:, 0]))
    bcr_s = np.maximum(np.abs(F[:, -1]), np.abs(c * lv.C[:, 1] * u[:, -1]) + np.abs(lv.Phi[:, 1]))
    tiny = 1e-300
    return (np.max(np.abs(bal) / np.maximum(bal_s, tiny)),
            np.max(np.abs(fm) / np.maximum(fm_s, tiny)),
            max(np.max(np.abs(bcl) / np.maximum(bcl_s, tiny)), np.max(np.abs(bcr) / np.maximum(bcr_s, tiny))))


# ---------------------------------------------------------------------------
# Grey level coupled to the material energy balance (Newton, one iteration)
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class GreyResult:
    T: np.ndarray  # [nx]
    sol: LOSolution  # grey E, F, boundary E
    sigE: np.ndarray  # grey sigma_E at the stage temperature (for the secant derivative)
    n_floor: int


def grey_newton(grey: Level, Tstar, Told, S, dS, Estar, D, cv, dx, c, dt) -> GreyResult:
    """One Newton iteration of the grey LOQD equations and the MEB (Eq. eb-Gamma-d).

    The MEB  c_v (T - T^old)/dt = c sigma_E(T) E - S(T),  with the emission
    S = sum_g 2 kappa_g B_g (= c sigma_B a_R T^4 for the exact grey sigma_B), is
    linearised at the stage temperature T*: S(T) ~ S* + S' dT and
    sigma_E(T) E ~ sigma_E* E + D E* dT (D: diagonal Frechet derivative of the
    grey opacity, Eq. f-derivative-d; E*: the stage spectrum's total energy).
    Solving the MEB for the local change gives dT = alpha + beta E with
        den   = c_v/dt + S' - c D E*
        alpha = (c_v (T^old - T*)/dt - S*) / den,   beta = c sigma_E* / den,
    which is substituted into the grey balance, so the grey system keeps the
    form of one LOQD level with effective absorption and emission.
    """
    Tstar = np.asarray(Tstar, dtype=np.float64)
    den = cv / dt + dS - c * D * Estar
    alpha = (cv * (Told - Tstar) / dt - S) / den
    beta = c * grey.sigE[0] / den
    g = c * D * Estar - dS
    eff = dataclasses.replace(
        grey,
        sigE=(grey.sigE[0] + g * beta / c)[None, :],
        emis=(S - g * alpha)[None, :],
    )
    sol = solve_level(eff, dx, c, dt)
    T = Tstar + alpha + beta * sol.E[0]
    floor = T < 0.5 * Tstar
    T = np.where(floor, 0.5 * Tstar, T)
    return GreyResult(T=T, sol=sol, sigE=grey.sigE[0].copy(), n_floor=int(np.count_nonzero(floor)))
