"""Parity at the large workload's full size (2000 cells, S32 Gauss-Legendre,
4096 groups, F cycle on 4096,1024,256,64,16,1) in the launch configuration the
benchmark times.  The oracle cannot run whole steps of this size in a test, so
(1) the opacity tables, the first transport sweep of the initial state and its
QD factors are compared with the oracle on a sample of groups (every group's
sweep is independent given the tables), and (2) a full converged time step is
checked against the discrete energy balance, a property that holds at any
size: the change of radiation plus material energy equals the net boundary
inflow over the step, to the convergence tolerance."""
import numpy as np
import pytest

from oracle import planck
from oracle.moments import factors
from oracle.sweep import sweep
from paper_2011_05427_amd import binding, inputs, tuning

from gpu_util import assert_close, note, to_np

pytestmark = pytest.mark.gpu

SAMPLE = [0, 1, 777, 2047, 3000, 4095]


def test_large_hierarchy_replay_matches_oracle():
    """The large workload's frequency hierarchy and cycle (F on
    4096,1024,256,64,16,1 with S32 Gauss-Legendre) on 12 cells, two replayed
    steps against the oracle at 1e-10 (every state array)."""
    from test_gpu_step import _compare_state, _oracle_run

    slabs, cfg, _ = inputs.config_large()
    slab = inputs.make_slab(12, 4096, 32)
    note(f"large hierarchy replay nx=12 ng=4096 nmu=32 levels={cfg.levels} lmax={cfg.lmax}")
    states, stats = _oracle_run(slab, cfg, cfg.levels, 2)
    sv = binding.Solver([slab], [cfg.levels], cfg)
    st = sv.new_state()
    sv.state_init(st, slab.T0)
    for j in range(2):
        note(f"  step {j} replay {stats.counts[j]}")
        gs = sv.step(st, replay=[stats.counts[j]])
        assert list(gs[0].cycles[:len(stats.counts[j])]) == stats.counts[j]
        _compare_state(f"large hierarchy step {j}", sv, st, states[j + 1])
    sv.close()


@pytest.mark.parametrize("levels,cycle", [([256, 16, 1], inputs.CYCLE_W), ([256, 64, 16, 1], inputs.CYCLE_F)])
def test_wide_slab_few_coarse_groups_replay(levels, cycle):
    """A wide slab (520 cells: 9 edge tiles) restricted to 16 coarse groups
    and to the grey group, where the restriction takes the chunk pass for r
    = 16 instead of the single pass (stage restriction fine -> 16 with its dS
    partials, coarse -> grey adding them), two replayed steps at 1e-10."""
    import dataclasses

    from test_gpu_step import _compare_state, _oracle_run

    _, cfg0, _ = inputs.config_large()
    cfg = dataclasses.replace(cfg0, cycle=cycle, lmax=1)
    slab = inputs.make_slab(520, 256, 8)
    note(f"wide slab replay nx=520 ng=256 nmu=8 levels={levels} cycle={'VWF'[cycle]}")
    states, stats = _oracle_run(slab, cfg, levels, 2)
    sv = binding.Solver([slab], [levels], cfg)
    st = sv.new_state()
    sv.state_init(st, slab.T0)
    for j in range(2):
        gs = sv.step(st, replay=[stats.counts[j]])
        assert list(gs[0].cycles[:len(stats.counts[j])]) == stats.counts[j]
        _compare_state(f"wide slab {levels} step {j}", sv, st, states[j + 1])
    sv.close()


def test_sixteen_tile_slab_chunk_widths_replay():
    """A slab of 960 cells (16 edge tiles), where the chunk pass starts at 16
    finer groups per wavefront (or r / 8): the fine -> grey restriction (r =
    256) and the stage restriction fine -> 4 groups (r = 64) take the wider
    chunks; F cycle on 256,16,4,1, two replayed steps at 1e-10."""
    import dataclasses

    from test_gpu_step import _compare_state, _oracle_run

    _, cfg0, _ = inputs.config_large()
    cfg = dataclasses.replace(cfg0, cycle=inputs.CYCLE_F, lmax=1)
    levels = [256, 16, 4, 1]
    slab = inputs.make_slab(960, 256, 8)
    note(f"16-tile slab replay nx=960 ng=256 nmu=8 levels={levels} cycle=F")
    states, stats = _oracle_run(slab, cfg, levels, 2)
    sv = binding.Solver([slab], [levels], cfg)
    st = sv.new_state()
    sv.state_init(st, slab.T0)
    for j in range(2):
        gs = sv.step(st, replay=[stats.counts[j]])
        assert list(gs[0].cycles[:len(stats.counts[j])]) == stats.counts[j]
        _compare_state(f"16-tile slab step {j}", sv, st, states[j + 1])
    sv.close()


def test_large_workload_sampled_sweep_and_energy_balance():
    import torch

    slabs, cfg, _ = inputs.config_large()
    slab = slabs[0]
    G, M, nx = slab.ng, slab.nmu, slab.nx
    note(f"large workload nx={nx} ng={G} nmu={M}: sampled sweep groups {SAMPLE}, one step energy balance")
    sv = binding.Solver([slab], [cfg.levels], cfg)
    st = sv.new_state()
    sv.state_init(st, slab.T0)
    # the sweep runs with the tile the autotuner picks for this size (as timed)
    tuning.tune(sv, st, reps=2, path=None)
    K, S, _ = sv.get_tiles()
    note(f"  autotuned tile for nx > 1024: K={K[5]} split={S[5]}")
    T0 = to_np(st["T"]).copy()
    # (1) stage parity on sampled groups
    kap, B = sv.empty(binding.TR_K_GI), sv.empty(binding.TR_K_GI)
    sv.opacity(st["T"], kap, B)
    Io = torch.empty_like(st["I_prev"])
    mom, bnd = sv.empty(binding.TR_K_GI, 4), sv.empty(binding.TR_K_G, 6)
    sv.sweep(kap, B, st["I_prev"], Io, mom, bnd)
    f, fbnd, Cb, Phi = (sv.empty(binding.TR_K_GI), sv.empty(binding.TR_K_G2), sv.empty(binding.TR_K_G2),
                        sv.empty(binding.TR_K_G2))
    sv.moments(mom, bnd, f, fbnd, Cb, Phi)
    idx = torch.as_tensor(SAMPLE, device="cuda")
    Ip = st["I_prev"].view(G, M, nx, 2).index_select(0, idx).cpu().numpy()
    Ig = Io.view(G, M, nx, 2).index_select(0, idx).cpu().numpy()
    k_ref = planck.opacity(slab.nu_center, slab.C_cell, T0)[SAMPLE]
    B_ref = planck.planck_groups(slab.nu_edges, T0, slab.aR, slab.c)[SAMPLE]
    assert_close("kappa", to_np(kap, (G, nx))[SAMPLE], k_ref, 1e-12)
    assert_close("B", to_np(B, (G, nx))[SAMPLE], B_ref, 1e-12)
    inc_l = planck.boundary_intensity(slab.nu_edges, slab.T_left, slab.aR, slab.c)[SAMPLE]
    inc_r = np.zeros(len(SAMPLE))
    I_ref = sweep(slab.mu, slab.x_edges, k_ref, B_ref, Ip, inc_l, inc_r, slab.c, slab.dt)
    for q, g in enumerate(SAMPLE):
        assert_close(f"I[g={g}]", Ig[q], I_ref[q], 1e-12)
    fac = factors(slab.mu, slab.w, I_ref, inc_l, inc_r, slab.c)
    phi_ok = I_ref.sum(axis=(1, 3)) > 1e-280
    fg = to_np(f, (G, nx))[SAMPLE]
    assert_close("f", np.where(phi_ok, fg, 0), np.where(phi_ok, fac.f, 0), 1e-12)
    assert_close("C", to_np(Cb, (G, 2))[SAMPLE], fac.C, 1e-12)
    assert_close("Phi", to_np(Phi, (G, 2))[SAMPLE], fac.Phi, 1e-12)
    del Io, mom, bnd
    # (2) one converged step: discrete energy balance
    E0 = to_np(st["E"], (G, nx)).sum(axis=0)
    stats = sv.step(st)
    assert stats[0].n_ti >= 1 and stats[0].n_floor == 0
    T1 = to_np(st["T"])
    E1 = to_np(st["E"], (G, nx)).sum(axis=0)
    F1 = to_np(st["F"], (G, nx + 1)).sum(axis=0)
    dx = np.diff(slab.x_edges)
    lhs = np.sum(dx * ((E1 - E0) + slab.cv * (T1 - T0)))
    rhs = -slab.dt * (F1[-1] - F1[0])
    scale = np.sum(dx * (E1 + slab.cv * T1))
    note(f"  energy balance residual {abs(lhs - rhs) / scale:.3e} of the total energy")
    assert abs(lhs - rhs) < 1e-8 * scale
    sv.close()
