"""Time step of the MLQD method with multigrid in frequency (oracle).

TEST INFRASTRUCTURE ONLY.

Paper Alg. 3 (Sec. 4); Alg. 2 is its V-cycle case (Sec. 3.2, Fig. 1c).  One
backward-Euler step j:

  outer (transport) iterations s = 0, 1, ...:
    s > 0: opacities at T^(s), sweep every (group, direction), QD factors.
           (s = 0 reuses the factors of the previous step: no sweep.)
    inner cycles l = 1 .. lmax (stop early when the inner test passes):
      fine spectrum: solve the multigroup LOQD at T^(l,s)            -> E_g, F_g
      stage k = 0: restrict fine -> grey at T~[0] = T^(l,s), solve the grey
                   LOQD + MEB by one Newton iteration                  -> T~[1]
      stages k = 1..K along the schedule S (grid gamma_k):
                   restrict fine -> gamma at T~[k] (weights: this cycle's
                   fine solution), solve the coarse LOQD; restrict gamma ->
                   grey, one Newton iteration                          -> T~[k+1]
      T^(l+1,s) = T~[K+1]
    T^(s+1) = T after the last cycle.

Readings where the paper is silent or ambiguous (each is mirrored by the GPU
library; the design notes list them):
  * loop tests use the infinity norm over cells and continue until both the
    temperature and the grey energy density criteria hold;
  * the inner loop runs at most lmax cycles and stops earlier when converged;
    the inner test compares the cycle's final T and grey E with their values at
    the start of the cycle;
  * the outer test is first applied after s = 1 (every step sweeps at least
    once); it compares the T and grey E at the end of iteration s with those at
    its start; more than max_outer iterations is non-convergence;
  * the secant derivative D of the grey sigma_E uses the previous grey stage of
    the same time step (D = 0 at the first), is zeroed where the stage
    temperature moved by 1e-8 relative or less, and where c D E* would exceed
    half of c_v/dt + S';
  * the step carries T, the last sweep's intensity and factors, and the last
    fine-grid solution (E_g, F_g) as old-time values of the next step; coarse
    and grey old-time values are block sums of the fine ones.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

from . import opacity, planck
from .lo import Level, LOSolution, fine_level, grey_newton, solve_level
from .moments import Factors, energy_flux, factors
from .restrict import restrict
from .sweep import sweep

SECANT_REL = 1e-8


class NonConvergence(RuntimeError):
    pass


@dataclasses.dataclass
class Problem:
    x_edges: np.ndarray
    nu_edges: np.ndarray
    nu_center: np.ndarray
    mu: np.ndarray
    w: np.ndarray
    C_cell: np.ndarray
    inc_left: np.ndarray  # [G] isotropic incoming intensity at x = 0
    inc_right: np.ndarray  # [G] at x = X
    cv: float
    dt: float
    c: float
    aR: float
    opacity: int = 0  # 0: point law at the group centre; 1: group averages of the spectral law

    @property
    def dx(self):
        return np.diff(self.x_edges)

    @property
    def nx(self):
        return len(self.x_edges) - 1

    @property
    def G(self):
        return len(self.nu_center)

    def tables(self, T):
        kappa = planck.opacity(self.nu_center, self.C_cell, T)
        B = planck.planck_groups(self.nu_edges, T, self.aR, self.c)
        return kappa, B

    def coeffs(self, T, Egrey):
        """Group coefficients at the material temperature T (cell array) and
        the grey energy density Egrey of the same grey solve (radiation
        temperature of the spectral averages): (sigma_E, emission source
        sigma_B B, sigma_R), each [G, nx].  Point law: (kappa, kappa B, kappa)."""
        if self.opacity == 1:
            Tr = opacity.radiation_temperature(Egrey, self.aR)
            return opacity.spectral_tables(self.nu_edges, self.C_cell, T, Tr, self.aR, self.c)
        kappa, B = self.tables(T)
        return kappa, kappa * B, kappa

    def emission_dT(self, T):
        """S'(T) = d/dT sum_g 2 sigma_B,g B_g  -> [nx]"""
        if self.opacity == 1:
            return 2.0 * np.sum(opacity.emission_dT(self.nu_edges, self.C_cell, T, self.aR, self.c), axis=0)
        kappa, B = self.tables(T)
        dk = planck.opacity_dT(self.nu_center, self.C_cell, T)
        dB = planck.planck_groups_dT(self.nu_edges, T, self.aR, self.c)
        return np.sum(2.0 * (dk * B + kappa * dB), axis=0)


def problem_from_slab(slab) -> Problem:
    """Build the oracle's problem from an ``inputs.Slab`` (boundary Planck
    temperatures turned into incoming group intensities here)."""
    return Problem(
        x_edges=np.asarray(slab.x_edges, dtype=np.float64),
        nu_edges=np.asarray(slab.nu_edges, dtype=np.float64),
        nu_center=np.asarray(slab.nu_center, dtype=np.float64),
        mu=np.asarray(slab.mu, dtype=np.float64),
        w=np.asarray(slab.w, dtype=np.float64),
        C_cell=np.asarray(slab.C_cell, dtype=np.float64),
        inc_left=planck.boundary_intensity(slab.nu_edges, slab.T_left, slab.aR, slab.c),
        inc_right=planck.boundary_intensity(slab.nu_edges, slab.T_right, slab.aR, slab.c),
        cv=float(slab.cv), dt=float(slab.dt), c=float(slab.c), aR=float(slab.aR),
        opacity=int(getattr(slab, "opacity", 0)),
    )


@dataclasses.dataclass
class State:
    T: np.ndarray  # [nx]
    I: np.ndarray  # [G, M, nx, 2]
    E: np.ndarray  # [G, nx]   fine-grid solution of the last step
    F: np.ndarray  # [G, nx+1]
    Ebnd: np.ndarray  # [G, 2]
    fac: Factors  # factors of the last sweep
    Egrey: np.ndarray  # [nx] grey energy density of the last grey solve
    j: int = 0

    def copy(self):
        return State(T=self.T.copy(), I=self.I.copy(), E=self.E.copy(), F=self.F.copy(),
                     Ebnd=self.Ebnd.copy(), fac=dataclasses.replace(self.fac), Egrey=self.Egrey.copy(),
                     j=self.j)


@dataclasses.dataclass
class Stats:
    n_ti: int = 0  # transport sweeps
    n_c: int = 0  # cycles
    n_lo: int = 0  # group-wise low-order solves (grey counted 1)
    counts: List[List[int]] = dataclasses.field(default_factory=list)  # per step: cycles per outer iteration
    n_floor: int = 0
    dT_outer: List[float] = dataclasses.field(default_factory=list)
    dT_cycle: List[float] = dataclasses.field(default_factory=list)


def initial_state(pb: Problem, T0: float, M: Optional[int] = None) -> State:
    """I^0 = B_g(T0) in every corner and direction; E^0, F^0 its moments
    (F^0 = 0 at every edge); factors of I^0 with the boundary data."""
    nx, G = pb.nx, pb.G
    M = len(pb.mu)
    T = np.full(nx, float(T0))
    B0 = planck.planck_groups(pb.nu_edges, T, pb.aR, pb.c)  # [G, nx]
    I = np.broadcast_to(B0[:, None, :, None], (G, M, nx, 2)).copy()
    E, _ = energy_flux(pb.mu, pb.w, I, pb.c)
    fac = factors(pb.mu, pb.w, I, pb.inc_left, pb.inc_right, pb.c)
    Ebnd = np.stack([E[:, 0], E[:, -1]], axis=1)
    return State(T=T, I=I, E=E, F=np.zeros((G, nx + 1)), Ebnd=Ebnd, fac=fac,
                 Egrey=E.sum(axis=0), j=0)


CYCLE_V, CYCLE_W, CYCLE_F = 0, 1, 2


def schedule(n_levels: int, cycle: int) -> List[int]:
    """Grids (0-based indices into the hierarchy, fine = 0, grey = n_levels - 1)
    visited after each grey solve in one cycle (paper Sec. 4, Fig. 1): the
    V cycle (Alg. 2) visits none; the W cycle (three grids) the middle one; the
    F cycle every intermediate grid, from the coarsest non-grey one up to the
    second finest (Fig. 1 draws Gamma = 4, S = (3, 2); the low-order solve
    counts of Tables 1-2 fix S = (Gamma - 1, ..., 2) for the larger Gamma)."""
    if cycle == CYCLE_V or n_levels <= 2:
        return []
    if cycle == CYCLE_W:
        return [1]
    return list(range(n_levels - 2, 0, -1))


def _norm(x):
    return float(np.max(np.abs(x)))


def _converged(Tn, To, En, Eo, eps):
    return _norm(Tn - To) <= eps * _norm(Tn) and _norm(En - Eo) <= eps * _norm(En)


def _secant(Tst, sig, prev, Estar, dS, pb: Problem):
    if prev is None:
        return np.zeros_like(Tst)
    Tp, sp = prev
    dT = Tst - Tp
    ok = np.abs(dT) > SECANT_REL * np.abs(Tst)
    D = np.where(ok, (sig - sp) / np.where(ok, dT, 1.0), 0.0)
    bad = pb.c * D * Estar > 0.5 * (pb.cv / pb.dt + dS)
    return np.where(bad, 0.0, D)


def _with_boundary_data(fac: Factors, pb: Problem) -> Factors:
    """Phi = F^in - c C E^in with the current incoming intensities."""
    mu, w = pb.mu, pb.w
    pos, neg = mu > 0, mu < 0
    Ein_l = np.sum(w[pos]) * pb.inc_left / pb.c
    Fin_l = np.sum(w[pos] * mu[pos]) * pb.inc_left
    Ein_r = np.sum(w[neg]) * pb.inc_right / pb.c
    Fin_r = np.sum(w[neg] * mu[neg]) * pb.inc_right
    Phi = np.stack([Fin_l - pb.c * fac.C[:, 0] * Ein_l, Fin_r - pb.c * fac.C[:, 1] * Ein_r], axis=1)
    return dataclasses.replace(fac, Phi=Phi)


def step(pb: Problem, levels: List[int], schedule: List[int], lmax: int, eps: float, eps_inner: float,
         st: State, *, max_outer: int = 50, secant: bool = True, replay: Optional[List[int]] = None,
         stats: Optional[Stats] = None) -> State:
    """Advance ``st`` by one time step; returns the new state.

    ``replay``: cycles per outer iteration to execute instead of the
    convergence tests (e.g. [4, 3, 1]: s = 0 runs 4 cycles, s = 1 runs 3 and
    s = 2 runs 1, i.e. two sweeps)."""
    if stats is None:
        stats = Stats()
    dx, c, dt, cv = pb.dx, pb.c, pb.dt, pb.cv
    Told, Eold, Fold = st.T, st.E, st.F
    fac = _with_boundary_data(st.fac, pb)
    I = st.I
    T_s = Told.copy()
    E_s = st.Egrey.copy()
    prev = None
    counts = []
    fsol = None
    s = 0
    while True:
        if s > 0:
            sig, src, _ = pb.coeffs(T_s, E_s)
            I = sweep(pb.mu, pb.x_edges, sig, None, st.I, pb.inc_left, pb.inc_right, c, dt, source=src)
            fac = factors(pb.mu, pb.w, I, pb.inc_left, pb.inc_right, c)
            stats.n_ti += 1
        T_cur, E_cur = T_s, E_s
        ncyc = 0
        while True:
            ncyc += 1
            # fine spectrum at T^(l,s)
            sig, src, sR = pb.coeffs(T_cur, E_cur)
            fine = fine_level(sig, None, fac, Eold, Fold, dx, emis=2.0 * src, sigR=sR)
            fsol = solve_level(fine, dx, c, dt)
            stats.n_lo += levels[0]
            # stage k = 0: grey from the fine spectrum
            Tst = T_cur
            grey = restrict(fine, fsol, 1, dx, c)
            dS = pb.emission_dT(Tst)
            Estar = fsol.E.sum(axis=0)
            D = _secant(Tst, grey.sigE[0], prev, Estar, dS, pb) if secant else np.zeros_like(Tst)
            gr = grey_newton(grey, Tst, Told, grey.emis[0], dS, Estar, D, cv, dx, c, dt)
            stats.n_lo += 1
            stats.n_floor += gr.n_floor
            prev = (Tst, gr.sigE)
            Tt, Eg = gr.T, gr.sol.E[0]
            for gam in schedule:
                sig2, src2, sR2 = pb.coeffs(Tt, Eg)
                fine2 = fine_level(sig2, None, fac, Eold, Fold, dx, emis=2.0 * src2, sigR=sR2)
                lv = restrict(fine2, fsol, levels[gam], dx, c)
                csol = solve_level(lv, dx, c, dt)
                stats.n_lo += levels[gam]
                grey = restrict(lv, csol, 1, dx, c)
                dS = pb.emission_dT(Tt)
                Estar = csol.E.sum(axis=0)
                D = _secant(Tt, grey.sigE[0], prev, Estar, dS, pb) if secant else np.zeros_like(Tt)
                gr = grey_newton(grey, Tt, Told, grey.emis[0], dS, Estar, D, cv, dx, c, dt)
                stats.n_lo += 1
                stats.n_floor += gr.n_floor
                prev = (Tt, gr.sigE)
                Tt, Eg = gr.T, gr.sol.E[0]
            stats.n_c += 1
            stats.dT_cycle.append(_norm(Tt - T_cur))
            conv_in = _converged(Tt, T_cur, Eg, E_cur, eps_inner)
            T_cur, E_cur = Tt, Eg
            if replay is not None:
                if ncyc >= replay[s]:
                    break
            elif conv_in or ncyc >= lmax:
                break
        counts.append(ncyc)
        conv_out = s >= 1 and _converged(T_cur, T_s, E_cur, E_s, eps)
        stats.dT_outer.append(_norm(T_cur - T_s))
        T_s, E_s = T_cur, E_cur
        if replay is not None:
            if s + 1 >= len(replay):
                break
        elif conv_out:
            break
        s += 1
        if s > max_outer:
            raise NonConvergence(f"no convergence in {max_outer} transport iterations")
    stats.counts.append(counts)
    return State(T=T_s, I=I, E=fsol.E, F=fsol.F, Ebnd=fsol.Ebnd, fac=fac, Egrey=E_s, j=st.j + 1)


def run(pb: Problem, T0: float, levels, schedule, lmax, eps, eps_inner, nsteps, *, secant=True,
        replay=None, stats=None, state=None):
    st = initial_state(pb, T0) if state is None else state
    stats = Stats() if stats is None else stats
    for j in range(nsteps):
        st = step(pb, levels, schedule, lmax, eps, eps_inner, st, secant=secant,
                  replay=None if replay is None else replay[j], stats=stats)
    return st, stats


# ---------------------------------------------------------------------------
# Single-grid two-level QD (Alg. 1) for tiny problems: the multigroup LOQD and
# the multigroup MEB (Eq. eb-group) are solved together by a global nonlinear
# solve in T, independent of the grey / restriction machinery.
# ---------------------------------------------------------------------------

def alg1_step(pb: Problem, st: State, eps: float = 1e-13, max_outer: int = 200) -> State:
    from scipy.optimize import root

    dx, c, dt, cv = pb.dx, pb.c, pb.dt, pb.cv
    Told, Eold, Fold = st.T, st.E, st.F
    fac = _with_boundary_data(st.fac, pb)
    I = st.I
    T = Told.copy()

    # radiation temperature of the spectral averages: from the total energy
    # density of the previous outer iteration's solution (held during the
    # nonlinear solve); at the fixed point it is that of the solution itself
    Er = st.Egrey.copy()

    def lo_at(Tv, fac_):
        sig, src, sR = pb.coeffs(Tv, Er)
        sol = solve_level(fine_level(sig, None, fac_, Eold, Fold, dx, emis=2.0 * src, sigR=sR), dx, c, dt)
        return sig, src, sol

    def meb_residual(Tv, fac_):
        sig, src, sol = lo_at(Tv, fac_)
        return cv * (Tv - Told) / dt - np.sum(c * sig * sol.E - 2.0 * src, axis=0)

    sol = None
    for s in range(max_outer):
        if s > 0:
            sig, src, _ = pb.coeffs(T, Er)
            I = sweep(pb.mu, pb.x_edges, sig, None, st.I, pb.inc_left, pb.inc_right, c, dt, source=src)
            fac = factors(pb.mu, pb.w, I, pb.inc_left, pb.inc_right, c)
        r = root(meb_residual, T, args=(fac,), method="hybr", tol=1e-15)
        Tn = r.x
        _, _, sol = lo_at(Tn, fac)
        En = sol.E.sum(axis=0)
        done = s >= 1 and _norm(Tn - T) <= eps * _norm(Tn) and _norm(En - Er) <= eps * _norm(En)
        T, Er = Tn, En
        if done:
            break
    else:
        raise NonConvergence("alg1 did not converge")
    return State(T=T, I=I, E=sol.E, F=sol.F, Ebnd=sol.Ebnd, fac=fac, Egrey=sol.E.sum(axis=0), j=st.j + 1)
