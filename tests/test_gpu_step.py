"""GPU parity of whole time steps (paper Alg. 3) against the CPU oracle.

Replay mode: the oracle runs free and records its cycles per transport
iteration; the GPU executes the same counts, so the two follow the same path
and must agree to 1e-10 relative (FP64).  Free-running GPU steps must reach
the oracle's converged solution within the convergence tolerance.
"""
import numpy as np
import pytest

from oracle import mlqd
from paper_2011_05427_amd import binding, inputs

from gpu_util import assert_close, note, rel_err, to_np

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _oracle_run(slab, cfg, levels, nsteps):
    pb = mlqd.problem_from_slab(slab)
    st = mlqd.initial_state(pb, slab.T0)
    stats = mlqd.Stats()
    states = [st]
    for _ in range(nsteps):
        st = mlqd.step(pb, levels, _sched(cfg, levels), cfg.lmax, cfg.eps, cfg.eps_inner, st, stats=stats)
        states.append(st)
    return states, stats


def _sched(cfg, levels):
    return mlqd.schedule(len(levels), cfg.cycle)


def _compare_state(tag, sv, st, ref, slab_idx=0):
    s = sv.slabs[slab_idx]
    nx, ng, M = s.nx, s.ng, s.nmu
    oc = sv.layout(binding.TR_K_CELL, slab_idx)[0]
    ogi = sv.layout(binding.TR_K_GI, slab_idx)[0]
    oge = sv.layout(binding.TR_K_GE, slab_idx)[0]
    og2 = sv.layout(binding.TR_K_G2, slab_idx)[0]
    oI = sv.layout(binding.TR_K_I, slab_idx)[0]
    T = to_np(st["T"])[oc:oc + nx]
    assert_close(f"{tag} T", T, ref.T, TOL, atol_scale=0.0)
    E = to_np(st["E"])[ogi:ogi + ng * nx].reshape(ng, nx)
    assert_close(f"{tag} E", E, ref.E, TOL)
    F = to_np(st["F"])[oge:oge + ng * (nx + 1)].reshape(ng, nx + 1)
    assert_close(f"{tag} F", F, ref.F, TOL * 10)
    Eb = to_np(st["Ebnd"])[og2:og2 + 2 * ng].reshape(ng, 2)
    assert_close(f"{tag} Ebnd", Eb, ref.Ebnd, TOL)
    I = to_np(st["I_prev"])[oI:oI + ng * M * nx * 2].reshape(ng, M, nx, 2)
    assert_close(f"{tag} I", I, ref.I, TOL)
    Eg = to_np(st["Egrey"])[oc:oc + nx]
    assert_close(f"{tag} Egrey", Eg, ref.Egrey, TOL)
    f = to_np(st["f"])[ogi:ogi + ng * nx].reshape(ng, nx)
    phi_ok = ref.I.sum(axis=(1, 3)) > 1e-280  # factors of underflowed groups are defaults
    assert_close(f"{tag} f", np.where(phi_ok, f, 0), np.where(phi_ok, ref.fac.f, 0), TOL)
    C = to_np(st["C"])[og2:og2 + 2 * ng].reshape(ng, 2)
    assert_close(f"{tag} C", C, ref.fac.C, TOL)


@pytest.mark.parametrize("case", ["small_V", "W3", "F4", "W_r32", "vacuum_both", "two_cells_S2", "max_cells",
                                  "thin", "thick", "spectral_V", "spectral_W", "spectral_F"])
def test_step_replay(case):
    if case.startswith("spectral"):  # the paper's group averages of the spectral opacity
        slab = inputs.make_slab(20, 16, 8, dt=0.004, nu_lo=1e-3, nu_hi=30.0, opacity=inputs.OPAC_SPECTRAL)
        cyc = {"V": inputs.CYCLE_V, "W": inputs.CYCLE_W, "F": inputs.CYCLE_F}[case[-1]]
        levels = {"V": [16, 1], "W": [16, 4, 1], "F": [16, 8, 2, 1]}[case[-1]]
        cfg = inputs.SolverCfg(levels=levels, cycle=cyc, lmax=2)
        nsteps = 2
    elif case == "small_V":
        slabs, cfg, nsteps = inputs.config_small()
        slab, levels = slabs[0], cfg.levels
        nsteps = 2
    elif case == "W3":
        slab = inputs.make_slab(40, 32, 8, dt=0.004)
        levels = [32, 4, 1]
        cfg = inputs.SolverCfg(levels=levels, cycle=inputs.CYCLE_W, lmax=2)
        nsteps = 3
    elif case == "F4":
        slab = inputs.make_slab(70, 64, 16, dt=0.002)
        levels = [64, 16, 4, 1]
        cfg = inputs.SolverCfg(levels=levels, cycle=inputs.CYCLE_F, lmax=2)
        nsteps = 2
    elif case == "W_r32":  # stage level of 32 fine groups per coarse group (two-pass stage restriction)
        slab = inputs.make_slab(70, 64, 8, dt=0.004)
        levels = [64, 2, 1]
        cfg = inputs.SolverCfg(levels=levels, cycle=inputs.CYCLE_W, lmax=2)
        nsteps = 2
    elif case == "vacuum_both":
        slab = inputs.make_slab(20, 8, 4, T_left=0.0, T_right=0.0, T0=0.05)
        levels = [8, 1]
        cfg = inputs.SolverCfg(levels=levels, cycle=inputs.CYCLE_V, lmax=3)
        nsteps = 2
    elif case == "two_cells_S2":  # smallest slab, two groups, two directions
        slab = inputs.make_slab(2, 2, 2)
        levels = [2, 1]
        cfg = inputs.SolverCfg(levels=levels, cycle=inputs.CYCLE_V, lmax=4)
        nsteps = 2
    elif case == "max_cells":  # the largest slab the LO block solver takes (2046 cells)
        slab = inputs.make_slab(2046, 4, 2)
        levels = [4, 1]
        cfg = inputs.SolverCfg(levels=levels, cycle=inputs.CYCLE_V, lmax=4)
        nsteps = 1
    elif case == "thin":  # optically thin everywhere
        slab = inputs.make_slab(30, 16, 8, C1=0.01, C2=0.001)
        levels = [16, 4, 1]
        cfg = inputs.SolverCfg(levels=levels, cycle=inputs.CYCLE_W, lmax=2)
        nsteps = 2
    else:  # optically thick everywhere (diffusive, near-isotropic factors)
        slab = inputs.make_slab(30, 16, 8, C1=3.0e4, C2=1.0e4)
        levels = [16, 4, 1]
        cfg = inputs.SolverCfg(levels=levels, cycle=inputs.CYCLE_W, lmax=2)
        nsteps = 2
    note(f"step replay {case} nx={slab.nx} ng={slab.ng} nmu={slab.nmu} levels={levels}")
    states, stats = _oracle_run(slab, cfg, levels, nsteps)
    sv = binding.Solver([slab], [levels], cfg)
    st = sv.new_state()
    sv.state_init(st, slab.T0)
    _compare_state(f"{case} init", sv, st, states[0])
    for j in range(nsteps):
        note(f"  step {j} replay {stats.counts[j]}")
        gs = sv.step(st, replay=[stats.counts[j]])
        assert list(gs[0].cycles[:len(stats.counts[j])]) == stats.counts[j]
        _compare_state(f"{case} step {j}", sv, st, states[j + 1])
    sv.close()


def test_step_free_running_matches_oracle():
    slabs, cfg, _ = inputs.config_small()
    slab = slabs[0]
    cfg = inputs.SolverCfg(levels=cfg.levels, cycle=cfg.cycle, lmax=cfg.lmax, eps=1e-12, eps_inner=1e-13)
    note("free-running small")
    states, stats = _oracle_run(slab, cfg, cfg.levels, 2)
    sv = binding.Solver([slab], [cfg.levels], cfg)
    st = sv.new_state()
    sv.state_init(st, slab.T0)
    tot = binding.TrStats * 1
    acc = tot()
    for j in range(2):
        sv.step(st, stats=acc)
    T = to_np(st["T"])
    assert rel_err(T, states[-1].T) < 1e-10
    E = to_np(st["E"]).reshape(slab.ng, slab.nx)
    assert rel_err(E, states[-1].E) < 1e-10
    assert acc[0].n_ti == stats.n_ti and acc[0].n_c == stats.n_c and acc[0].n_lo == stats.n_lo
    sv.close()


def test_batch_of_uneven_slabs_replay():
    """Three slabs of different sizes in one context (pooled layout, per-slab
    convergence), each against its own oracle run."""
    slabs = [inputs.make_slab(30, 16, 8, C1=5.0, C2=40.0, T_left=0.8),
             inputs.make_slab(77, 64, 16, C1=60.0, C2=2.0, T_left=1.3),
             inputs.make_slab(12, 128, 8, C1=1.5, C2=9.0, T_left=0.6)]
    levels = [[s.ng, s.ng // 8, 1] for s in slabs]
    cfg = inputs.SolverCfg(levels=[0, 0, 1], cycle=inputs.CYCLE_W, lmax=2)
    refs = [_oracle_run(s, cfg, lv, 2) for s, lv in zip(slabs, levels)]
    note("batch of 3 slabs")
    sv = binding.Solver(slabs, levels, cfg)
    st = sv.new_state()
    sv.state_init(st, 0.001)
    for j in range(2):
        sv.step(st, replay=[r[1].counts[j] for r in refs])
        for k, (states, _) in enumerate(refs):
            _compare_state(f"batch slab {k} step {j}", sv, st, states[j + 1], slab_idx=k)
    sv.close()


def test_paper_scale_one_step_replay():
    """Full-size paper-scale workload (200 cells, S16, 512 groups, V cycle on
    512,128,32,8,1), first time step."""
    slabs, cfg, _ = inputs.config_paper_scale()
    slab = slabs[0]
    note("paper-scale step 0")
    states, stats = _oracle_run(slab, cfg, cfg.levels, 1)
    sv = binding.Solver([slab], [cfg.levels], cfg)
    st = sv.new_state()
    sv.state_init(st, slab.T0)
    sv.step(st, replay=[stats.counts[0]])
    _compare_state("paper-scale step 0", sv, st, states[1])
    sv.close()


def test_graph_replay_equals_eager_launches():
    """tr_step replays captured graphs of a transport iteration (default) or
    launches eagerly (timing mode); over several steps, with eager work and
    synchronisations between replays, both give bitwise identical states."""
    slab = inputs.make_slab(40, 32, 8, dt=0.004)
    levels = [32, 4, 1]
    cfg = inputs.SolverCfg(levels=levels, cycle=inputs.CYCLE_W, lmax=2)
    note("graph vs eager, W cycle, 4 steps")
    outs = []
    for timing in (False, True):
        sv = binding.Solver([slab], [levels], cfg, timing=timing)
        st = sv.new_state()
        sv.state_init(st, slab.T0)
        for _ in range(4):
            sv.step(st)
        outs.append({k: to_np(v).copy() for k, v in st.items()})
        sv.close()
    for k in outs[0]:
        assert np.array_equal(outs[0][k], outs[1][k]), k


@pytest.mark.gpu
def test_timed_sweep_launches_equal_graph_replay():
    """With sweep timing on, tr_step launches the sweeps outside its graphs
    with start / end events; the states stay bitwise identical to the plain
    graph replay, and the sweep kernel time is reported for every launch."""
    slab = inputs.make_slab(40, 32, 8, dt=0.004)
    levels = [32, 4, 1]
    cfg = inputs.SolverCfg(levels=levels, cycle=inputs.CYCLE_W, lmax=2)
    note("graph replay vs timed sweep launches, W cycle, 4 steps (timing on in steps 1 and 3)")
    outs = []
    for mode in (0, 1):
        sv = binding.Solver([slab], [levels], cfg)
        st = sv.new_state()
        sv.state_init(st, slab.T0)
        for k in range(4):
            sv.set_sweep_timing(mode == 1 and k % 2 == 1)
            stats = sv.step(st)
            if mode == 1 and k % 2 == 1:
                assert stats[0].n_launch[binding.T_SWEEP] == stats[0].n_ti > 0
                assert stats[0].t_ms[binding.T_SWEEP] > 0.0
            else:
                assert stats[0].n_launch[binding.T_SWEEP] == 0
        outs.append({k: to_np(v).copy() for k, v in st.items()})
        sv.close()
    for k in outs[0]:
        assert np.array_equal(outs[0][k], outs[1][k]), k


@pytest.mark.gpu
def test_steps_on_a_side_stream_equal_the_default_stream():
    """tr_step and tr_run run on the caller's stream (the library only
    captures its graphs on a stream of its own): the same steps queued on a
    side stream give bitwise the state they give on the default stream, with
    the same counters."""
    import torch

    slab = inputs.make_slab(40, 32, 8, dt=0.004)
    levels = [32, 4, 1]
    cfg = inputs.SolverCfg(levels=levels, cycle=inputs.CYCLE_V, lmax=2)
    note("V cycle, 1 tr_step + 3 steps of tr_run, default stream vs a side stream")
    outs, counts = [], []
    for side in (False, True):
        sv = binding.Solver([slab], [levels], cfg)
        st = sv.new_state()
        sv.state_init(st, slab.T0)
        torch.cuda.synchronize()
        stream = torch.cuda.Stream() if side else torch.cuda.current_stream()
        with torch.cuda.stream(stream):
            a = sv.step(st)
            b = sv.run(st, 3)
        stream.synchronize()
        counts.append((a[0].n_ti, a[0].n_c, b[0].n_ti, b[0].n_c))
        outs.append({k: to_np(v).copy() for k, v in st.items()})
        sv.close()
    assert counts[0] == counts[1] and counts[0][2] > 0
    for k in outs[0]:
        assert np.array_equal(outs[0][k], outs[1][k]), k


@pytest.mark.gpu
@pytest.mark.parametrize("cycle,levels", [
    (inputs.CYCLE_V, [8, 1]),
    (inputs.CYCLE_W, [8, 4, 1]),
    (inputs.CYCLE_F, [8, 4, 2, 1]),
])
def test_steps_reach_the_single_grid_solution(cycle, levels):
    """Paper Alg. 1 solves the multigroup LOQD equations and the energy
    balance as one nonlinear system on the fine frequency grid (the oracle:
    a global root find in T around the multigroup LO solve).  At tight
    tolerances the multigrid steps on the GPU converge to the same solution,
    for every cycle shape."""
    slab = inputs.make_slab(6, 8, 4, dt=0.004, T0=0.01, C1=4.0, C2=1.0)
    pb = mlqd.problem_from_slab(slab)
    ref = mlqd.initial_state(pb, slab.T0)
    for _ in range(2):
        ref = mlqd.alg1_step(pb, ref, eps=1e-14)
    cfg = inputs.SolverCfg(levels=levels, cycle=cycle, lmax=4, eps=1e-13, eps_inner=1e-14, max_outer=60)
    note(f"cycle {cycle} levels {levels}: 2 GPU steps against 2 single-grid oracle steps")
    sv = binding.Solver([slab], [levels], cfg)
    st = sv.new_state()
    sv.state_init(st, slab.T0)
    for _ in range(2):
        sv.step(st)
    T = to_np(st["T"])
    E = to_np(st["E"]).reshape(slab.ng, slab.nx)
    np.testing.assert_allclose(T, ref.T, rtol=1e-10)
    np.testing.assert_allclose(E, ref.E, rtol=1e-9, atol=1e-12 * ref.E.max())
    sv.close()
