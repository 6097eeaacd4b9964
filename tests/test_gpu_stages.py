"""GPU parity of each stage of the hot path against the CPU oracle, through the
C ABI: opacity/Planck tables, SCB sweep with its moments, QD factors, LO solves
on fine and coarse levels, restriction and the grey/MEB Newton update.

Sizes span several sweep passes (256 cells per wavefront pass), several
solver partitions (8 rows per thread) and ragged tails; degenerate cases cover
two cells, one group and two directions.
"""
import dataclasses

import numpy as np
import pytest

from oracle import lo, opacity, planck
from oracle.moments import Factors, factors
from oracle.restrict import restrict
from oracle.sweep import sweep
from paper_2011_05427_amd import binding, inputs

from gpu_util import assert_close, note, slab_case, to_dev, to_np

pytestmark = pytest.mark.gpu

K = binding


def _solver(slab, levels, cfg=None):
    if cfg is None:
        cfg = inputs.SolverCfg(levels=levels)
    return binding.Solver([slab], [levels], cfg)


@pytest.mark.parametrize("nx,ng", [(2, 1), (300, 130), (37, 64)])
def test_opacity_tables(nx, ng):
    note(f"opacity nx={nx} ng={ng}")
    slab, _ = slab_case(nx, ng, 2)
    rng = np.random.default_rng(nx + ng)
    T = 10 ** rng.uniform(-3, np.log10(1.5), nx)
    sv = _solver(slab, [ng, 1])
    kap, B, dS = sv.empty(K.TR_K_GI), sv.empty(K.TR_K_GI), sv.empty(K.TR_K_CELL)
    sv.opacity(to_dev(T), kap, B, dS)
    k_ref = planck.opacity(slab.nu_center, slab.C_cell, T)
    B_ref = planck.planck_groups(slab.nu_edges, T, slab.aR, slab.c)
    dk = planck.opacity_dT(slab.nu_center, slab.C_cell, T)
    dB = planck.planck_groups_dT(slab.nu_edges, T, slab.aR, slab.c)
    dS_ref = np.sum(2 * (dk * B_ref + k_ref * dB), axis=0)
    assert_close("kappa", to_np(kap, (ng, nx)), k_ref, 1e-13, atol_scale=0.0)
    got_B = to_np(B, (ng, nx))
    ok = np.abs(got_B - B_ref) <= 1e-12 * np.abs(B_ref) + 1e-300
    assert ok.all(), f"B mismatch at {np.argwhere(~ok)[0]}"
    assert_close("dS", to_np(dS), dS_ref, 1e-11)
    sv.close()


@pytest.mark.parametrize("nx,ng,lo_nu,hi_nu", [(13, 40, 1e-4, 10.0), (300, 6, 0.01, 100.0), (2, 1, 0.01, 100.0)])
def test_spectral_opacity_tables(nx, ng, lo_nu, hi_nu):
    """Group averages of the spectral opacity (sigma_E,g at the radiation
    temperature, emission sigma_B,g B_g = kappa B, Rosseland sigma_R,g) and
    dS against the oracle's quadratures of the definitions, over radiation
    temperatures from far below to far above the material temperature."""
    note(f"spectral opacity nx={nx} ng={ng} nu in [{lo_nu}, {hi_nu}]")
    slab = inputs.make_slab(nx, ng, 2, nu_lo=lo_nu, nu_hi=hi_nu, opacity=inputs.OPAC_SPECTRAL)
    rng = np.random.default_rng(nx + ng)
    T = 10 ** rng.uniform(-3, np.log10(1.5), nx)
    Tr = T * 10 ** rng.uniform(-2, 2.5, nx)
    Tr = np.clip(Tr, 1e-4, 3.0)
    Eg = slab.aR * Tr ** 4
    sv = _solver(slab, [ng, 1])
    kap, B, sR, dS = sv.empty(K.TR_K_GI), sv.empty(K.TR_K_GI), sv.empty(K.TR_K_GI), sv.empty(K.TR_K_CELL)
    sv.opacity(to_dev(T), kap, B, dS, Egrey=to_dev(Eg), sigR=sR)
    Tr_ref = opacity.radiation_temperature(Eg, slab.aR)
    sE_ref, src_ref, sR_ref = opacity.spectral_tables(slab.nu_edges, slab.C_cell, T, Tr_ref, slab.aR, slab.c)
    dS_ref = 2 * opacity.emission_dT(slab.nu_edges, slab.C_cell, T, slab.aR, slab.c).sum(axis=0)
    k = to_np(kap, (ng, nx))
    assert_close("sigma_E", k, sE_ref, 1e-12, atol_scale=0.0)
    assert_close("sigma_R", to_np(sR, (ng, nx)), sR_ref, 1e-12, atol_scale=0.0)
    src = k * to_np(B, (ng, nx))
    ok = np.abs(src - src_ref) <= 1e-12 * np.abs(src_ref) + 1e-300
    assert ok.all(), f"emission mismatch at {np.argwhere(~ok)[0]}"
    assert_close("dS", to_np(dS), dS_ref, 1e-12, atol_scale=0.0)
    sv.close()


@pytest.mark.parametrize("nx,ng,nmu", [(2, 3, 2), (50, 5, 8), (300, 4, 16), (700, 3, 32), (257, 2, 8)])
def test_sweep_and_moments(nx, ng, nmu):
    note(f"sweep nx={nx} ng={ng} nmu={nmu}")
    slab, _ = slab_case(nx, ng, nmu, T_left=1.0, T_right=0.7)
    rng = np.random.default_rng(3 * nx + ng)
    kap = 10 ** rng.uniform(-2, 4, (ng, nx))
    B = rng.uniform(0.0, 1.0, (ng, nx))
    Ip = rng.uniform(0.0, 1.0, (ng, nmu, nx, 2))
    sv = _solver(slab, [ng, 1])
    Io = sv.empty(K.TR_K_I)
    mom, bnd = sv.empty(K.TR_K_GI, 4), sv.empty(K.TR_K_G, 6)
    sv.sweep(to_dev(kap), to_dev(B), to_dev(Ip), Io, mom, bnd)
    f, fbnd, Cb, Phi = sv.empty(K.TR_K_GI), sv.empty(K.TR_K_G2), sv.empty(K.TR_K_G2), sv.empty(K.TR_K_G2)
    sv.moments(mom, bnd, f, fbnd, Cb, Phi)
    inc_l = planck.boundary_intensity(slab.nu_edges, 1.0, slab.aR, slab.c)
    inc_r = planck.boundary_intensity(slab.nu_edges, 0.7, slab.aR, slab.c)
    I_ref = sweep(slab.mu, slab.x_edges, kap, B, Ip, inc_l, inc_r, slab.c, slab.dt)
    fac = factors(slab.mu, slab.w, I_ref, inc_l, inc_r, slab.c)
    I_got = to_np(Io, I_ref.shape)
    for g in range(ng):
        assert_close(f"I[g={g}]", I_got[g], I_ref[g], 1e-12)
    assert_close("f", to_np(f, (ng, nx)), fac.f, 1e-12)
    assert_close("fbnd", to_np(fbnd, (ng, 2)), fac.f_bnd, 1e-12)
    assert_close("C", to_np(Cb, (ng, 2)), fac.C, 1e-12)
    assert_close("Phi", to_np(Phi, (ng, 2)), fac.Phi, 1e-12)
    sv.close()


def _random_factors(rng, ng, nx):
    return Factors(f=rng.uniform(0.25, 0.5, (ng, nx)), f_bnd=rng.uniform(0.25, 0.6, (ng, 2)),
                   C=np.stack([-rng.uniform(0.4, 0.6, ng), rng.uniform(0.4, 0.6, ng)], axis=1),
                   Phi=np.stack([rng.uniform(0, 2, ng), -rng.uniform(0, 0.1, ng)], axis=1))


@pytest.mark.parametrize("nx,ng,sepR", [(2, 1, False), (7, 3, False), (200, 2, False), (1000, 2, False),
                                        (2046, 1, False), (7, 3, True), (513, 2, True)])
def test_lo_fine(nx, ng, sepR):
    """sepR: a Rosseland table of its own (the group averages of the spectral
    opacity) instead of kappa for the edge opacities."""
    note(f"lo fine nx={nx} ng={ng} separate sigma_R={sepR}")
    slab, _ = slab_case(nx, ng, 2)
    rng = np.random.default_rng(nx * 7 + ng)
    kap = 10 ** rng.uniform(-2, 4, (ng, nx))
    B = rng.uniform(0.0, 1.0, (ng, nx))
    fac = _random_factors(rng, ng, nx)
    Eold = rng.uniform(0, 1, (ng, nx))
    Fold = rng.uniform(-0.5, 0.5, (ng, nx + 1))
    dx = np.diff(slab.x_edges)
    sR = kap * 10 ** rng.uniform(-1, 1, (ng, nx)) if sepR else None
    ref = lo.solve_level(lo.fine_level(kap, B, fac, Eold, Fold, dx, sigR=sR), dx, slab.c, slab.dt)
    sv = _solver(slab, [ng, 1])
    E, F, Eb = sv.empty(K.TR_K_GI), sv.empty(K.TR_K_GE), sv.empty(K.TR_K_G2)
    co = dict(kappa=to_dev(kap), B=to_dev(B), f=to_dev(fac.f), fbnd=to_dev(fac.f_bnd), C=to_dev(fac.C),
              Phi=to_dev(fac.Phi), Eold=to_dev(Eold), Fold=to_dev(Fold))
    if sepR:
        co["sigRc"] = to_dev(sR)
    sv.lo_solve(0, co, E, F, Eb)
    assert_close("E", to_np(E, (ng, nx)), ref.E, 1e-12)
    assert_close("Ebnd", to_np(Eb, (ng, 2)), ref.Ebnd, 1e-12)
    assert_close("F", to_np(F, (ng, nx + 1)), ref.F, 1e-11)
    sv.close()


def _random_level(rng, P, nx):
    return lo.Level(
        sigE=10 ** rng.uniform(-2, 3, (P, nx)), emis=rng.uniform(0, 5, (P, nx)),
        a=rng.uniform(0.2, 0.6, (P, nx + 1)), b=rng.uniform(0.2, 0.6, (P, nx + 1)),
        sigR=10 ** rng.uniform(-2, 3, (P, nx + 1)),
        C=np.stack([-rng.uniform(0.3, 0.7, P), rng.uniform(0.3, 0.7, P)], axis=1),
        Phi=np.stack([rng.uniform(0, 3, P), -rng.uniform(0, 0.1, P)], axis=1),
        Eold=rng.uniform(0, 2, (P, nx)), Fold=rng.uniform(-1, 1, (P, nx + 1)))


def _level_dev(lv):
    return dict(sigE=to_dev(lv.sigE), emis=to_dev(lv.emis), a=to_dev(lv.a), b=to_dev(lv.b), sigR=to_dev(lv.sigR),
                C=to_dev(lv.C), Phi=to_dev(lv.Phi), Eold=to_dev(lv.Eold), Fold=to_dev(lv.Fold))


@pytest.mark.parametrize("nx,P", [(9, 4), (513, 2)])
def test_lo_coarse(nx, P):
    note(f"lo coarse nx={nx} P={P}")
    ng = 4 * P
    slab, _ = slab_case(nx, ng, 2)
    rng = np.random.default_rng(nx + P)
    lv = _random_level(rng, P, nx)
    dx = np.diff(slab.x_edges)
    ref = lo.solve_level(lv, dx, slab.c, slab.dt)
    sv = _solver(slab, [ng, P, 1])
    E, F, Eb = sv.empty(K.TR_K_LEV_PI + 1), sv.empty(K.TR_K_LEV_PE + 1), sv.empty(K.TR_K_LEV_P2 + 1)
    sv.lo_solve(1, _level_dev(lv), E, F, Eb)
    assert_close("E", to_np(E, (P, nx)), ref.E, 1e-12)
    assert_close("Ebnd", to_np(Eb, (P, 2)), ref.Ebnd, 1e-12)
    assert_close("F", to_np(F, (P, nx + 1)), ref.F, 1e-11)
    sv.close()


def _level_out(sv, lev):
    pi, pe, p2 = K.TR_K_LEV_PI + lev, K.TR_K_LEV_PE + lev, K.TR_K_LEV_P2 + lev
    return dict(sigE=sv.empty(pi), emis=sv.empty(pi), a=sv.empty(pe), b=sv.empty(pe), sigR=sv.empty(pe),
                C=sv.empty(p2), Phi=sv.empty(p2), Eold=sv.empty(pi), Fold=sv.empty(pe), Esum=sv.empty(pi))


def _cmp_level(name, out, ref, P, nx, Esum_ref):
    for k in ("sigE", "emis", "Eold"):
        assert_close(f"{name}.{k}", to_np(out[k], (P, nx)), getattr(ref, k), 1e-12)
    for k in ("a", "b", "sigR", "Fold"):
        assert_close(f"{name}.{k}", to_np(out[k], (P, nx + 1)), getattr(ref, k), 1e-11)
    for k in ("C", "Phi"):
        assert_close(f"{name}.{k}", to_np(out[k], (P, 2)), getattr(ref, k), 1e-12)
    assert_close(f"{name}.Esum", to_np(out["Esum"], (P, nx)), Esum_ref, 1e-12)


@pytest.mark.parametrize("ng,P,nx,sepR", [(16, 4, 11, False), (256, 2, 9, False), (128, 1, 300, False),
                                          (260, 2, 5, False), (16, 4, 11, True), (256, 2, 9, True)])
def test_restriction(ng, P, nx, sepR):
    note(f"restrict ng={ng} P={P} nx={nx} separate sigma_R={sepR}")
    levels = [ng, P, 1] if P > 1 else [ng, 1]
    slab, _ = slab_case(nx, ng, 2)
    rng = np.random.default_rng(ng + P + nx)
    dx = np.diff(slab.x_edges)
    kap = 10 ** rng.uniform(-2, 4, (ng, nx))
    B = rng.uniform(0, 1, (ng, nx))
    fac = _random_factors(rng, ng, nx)
    Eold = rng.uniform(0, 1, (ng, nx))
    Fold = rng.uniform(-0.5, 0.5, (ng, nx + 1))
    sR = kap * 10 ** rng.uniform(-1, 1, (ng, nx)) if sepR else None
    fine = lo.fine_level(kap, B, fac, Eold, Fold, dx, sigR=sR)
    fs = lo.solve_level(fine, dx, slab.c, slab.dt)
    sv = _solver(slab, levels)
    co = dict(kappa=to_dev(kap), B=to_dev(B), f=to_dev(fac.f), fbnd=to_dev(fac.f_bnd), C=to_dev(fac.C),
              Phi=to_dev(fac.Phi), Eold=to_dev(Eold), Fold=to_dev(Fold))
    if sepR:
        co["sigRc"] = to_dev(sR)
    sol = dict(E=to_dev(fs.E), F=to_dev(fs.F), Ebnd=to_dev(fs.Ebnd))
    lev = 1
    out = _level_out(sv, lev)
    sv.restrict(0, lev, co, sol, out)
    ref = restrict(fine, fs, P, dx, slab.c)
    r = ng // P
    _cmp_level("fine->1", out, ref, P, nx, fs.E.reshape(P, r, nx).sum(axis=1))
    if P > 1:
        # level 1 -> grey with the level-1 solution
        cs = lo.solve_level(ref, dx, slab.c, slab.dt)
        co1 = _level_dev(ref)
        sol1 = dict(E=to_dev(cs.E), F=to_dev(cs.F), Ebnd=to_dev(cs.Ebnd))
        outg = _level_out(sv, 2)
        sv.restrict(1, 2, co1, sol1, outg)
        refg = restrict(ref, cs, 1, dx, slab.c)
        _cmp_level("1->grey", outg, refg, 1, nx, cs.E.sum(axis=0, keepdims=True))
    sv.close()


@pytest.mark.parametrize("nx", [3, 64, 1500])
def test_grey_newton(nx):
    note(f"grey nx={nx}")
    slab, _ = slab_case(nx, 4, 2)
    rng = np.random.default_rng(nx)
    dx = np.diff(slab.x_edges)
    grey = _random_level(rng, 1, nx)
    Told = rng.uniform(0.1, 0.5, nx)
    Tstar = Told * rng.uniform(1.0, 1.3, nx)
    dS = rng.uniform(1.0, 10.0, nx)
    Estar = rng.uniform(0.1, 1.0, nx)
    D = rng.uniform(-1.0, 1.0, nx)
    ref = lo.grey_newton(grey, Tstar, Told, grey.emis[0], dS, Estar, D, slab.cv, dx, slab.c, slab.dt)
    sv = _solver(slab, [4, 1])
    E, F, Eb = sv.empty(K.TR_K_LEV_PI + 1), sv.empty(K.TR_K_LEV_PE + 1), sv.empty(K.TR_K_LEV_P2 + 1)
    Tout = sv.empty(K.TR_K_CELL)
    sv.grey_solve(_level_dev(grey), to_dev(Tstar), to_dev(Told), to_dev(dS), to_dev(Estar), to_dev(D), Tout,
                  E, F, Eb)
    assert_close("T", to_np(Tout), ref.T, 1e-12, atol_scale=0.0)
    assert_close("E", to_np(E, (1, nx)), ref.sol.E, 1e-12)
    assert_close("F", to_np(F, (1, nx + 1)), ref.sol.F, 1e-11)
    sv.close()
