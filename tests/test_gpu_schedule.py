"""Per-step cycle and lmax (tr_set_schedule) on the GPU.

The oracle runs a sequence of time steps whose cycle (V / W / F over one grid
hierarchy, paper Alg. 3) and lmax change from step to step; the GPU context
switches its schedule the same way and replays the oracle's cycle counts:
every state after every step agrees to 1e-10 and the LO solve counts are
equal.  Graph replay and eager launches stay bitwise identical across the
switches, and the stage-adaptive controller reaches the fixed schedule's
solution.
"""
import numpy as np
import pytest

from oracle import mlqd
from paper_2011_05427_amd import binding, inputs, tuning

from gpu_util import note, rel_err, to_np
from test_gpu_step import _compare_state

pytestmark = pytest.mark.gpu

V, W, F = inputs.CYCLE_V, inputs.CYCLE_W, inputs.CYCLE_F


def _sched(levels, cycle):
    return mlqd.schedule(len(levels), cycle)


def test_schedule_changes_replay_the_oracle():
    slab = inputs.make_slab(70, 64, 16, dt=0.002)
    levels = [64, 16, 4, 1]
    plan = [(V, 1), (W, 2), (F, 1), (F, 3), (V, 4), (W, 1)]
    base = inputs.SolverCfg(levels=levels, cycle=V, lmax=4)
    pb = mlqd.problem_from_slab(slab)
    ost = mlqd.initial_state(pb, slab.T0)
    sv = binding.Solver([slab], [levels], base)
    st = sv.new_state()
    sv.state_init(st, slab.T0)
    for j, (cyc, lmax) in enumerate(plan):
        stats = mlqd.Stats()
        ost = mlqd.step(pb, levels, _sched(levels, cyc), lmax, base.eps, base.eps_inner, ost, stats=stats)
        note(f"step {j}: cycle {'VWF'[cyc]} lmax {lmax} replay {stats.counts[0]}")
        sv.set_schedule(cyc, lmax)
        gs = sv.step(st, replay=[stats.counts[0]])
        assert list(gs[0].cycles[:len(stats.counts[0])]) == stats.counts[0]
        assert gs[0].n_lo == stats.n_lo and gs[0].n_c == stats.n_c
        _compare_state(f"schedule step {j}", sv, st, ost)
    sv.close()


def test_schedule_switches_graph_replay_equals_eager():
    slab = inputs.make_slab(40, 32, 8, dt=0.004)
    levels = [32, 8, 2, 1]
    plan = [(V, 1), (W, 2), (V, 1), (F, 2), (W, 2), (V, 4)]
    note("graph vs eager across schedule switches")
    outs = []
    for timing in (False, True):
        sv = binding.Solver([slab], [levels], inputs.SolverCfg(levels=levels, cycle=V, lmax=4), timing=timing)
        st = sv.new_state()
        sv.state_init(st, slab.T0)
        for cyc, lmax in plan:
            sv.set_schedule(cyc, lmax)
            sv.step(st)
        outs.append({k: to_np(v).copy() for k, v in st.items()})
        sv.close()
    for k in outs[0]:
        assert np.array_equal(outs[0][k], outs[1][k]), k


def test_invalid_schedules_are_rejected():
    slab = inputs.make_slab(10, 8, 4)
    sv = binding.Solver([slab], [[8, 1]], inputs.SolverCfg(levels=[8, 1]))
    for cyc, lmax in ((3, 1), (-1, 1), (V, 0), (V, 65)):
        with pytest.raises(binding.TrError):
            sv.set_schedule(cyc, lmax)
    sv.close()


def test_stage_adaptive_run_reaches_the_fixed_schedule_solution():
    slab = inputs.make_slab(60, 64, 8, dt=0.004)
    levels = [64, 8, 1]
    cands = [(W, 1), (W, 2), (V, 1), (W, 4)]
    note("stage-adaptive controller, 8 steps, against fixed W lmax 4")
    res = []
    for adaptive in (False, True):
        sv = binding.Solver([slab], [levels], inputs.SolverCfg(levels=levels, cycle=W, lmax=4))
        st = sv.new_state()
        sv.state_init(st, slab.T0)
        ctl = tuning.StageSchedule(cands, probe=3)
        for _ in range(8):
            if adaptive:
                ctl.step(sv, st)
            else:
                sv.step(st)
        res.append((to_np(st["T"]).copy(), to_np(st["E"]).copy()))
        if adaptive:
            assert len(ctl.history) == 8
            assert {c for c, _ in ctl.history[:4]} == set(cands)
        sv.close()
    assert rel_err(res[1][0], res[0][0]) < 1e-8
    assert rel_err(res[1][1], res[0][1]) < 1e-8


def test_batch_schedule_changes_replay_each_slab():
    """Three uneven slabs in one context switch schedule together; each slab
    replays its own oracle run (its LO solve count follows its own grids)."""
    slabs = [inputs.make_slab(30, 16, 8, C1=5.0, C2=40.0, T_left=0.8),
             inputs.make_slab(50, 64, 16, C1=60.0, C2=2.0, T_left=1.3),
             inputs.make_slab(12, 128, 8, C1=1.5, C2=9.0, T_left=0.6)]
    levels = [[s.ng, s.ng // 8, 1] for s in slabs]
    plan = [(W, 2), (V, 1), (W, 1), (V, 3)]
    base = inputs.SolverCfg(levels=[0, 0, 1], cycle=W, lmax=2)
    pbs = [mlqd.problem_from_slab(s) for s in slabs]
    osts = [mlqd.initial_state(pb, s.T0) for pb, s in zip(pbs, slabs)]
    sv = binding.Solver(slabs, levels, base)
    st = sv.new_state()
    sv.state_init(st, 0.001)
    for j, (cyc, lmax) in enumerate(plan):
        counts, nlo = [], []
        for k in range(len(slabs)):
            stats = mlqd.Stats()
            osts[k] = mlqd.step(pbs[k], levels[k], _sched(levels[k], cyc), lmax, base.eps, base.eps_inner, osts[k],
                                stats=stats)
            counts.append(stats.counts[0])
            nlo.append(stats.n_lo)
        note(f"batch step {j}: cycle {'VWF'[cyc]} lmax {lmax}")
        sv.set_schedule(cyc, lmax)
        gs = sv.step(st, replay=counts)
        for k in range(len(slabs)):
            assert gs[k].n_lo == nlo[k], (j, k)
            _compare_state(f"batch schedule step {j} slab {k}", sv, st, osts[k], slab_idx=k)
    sv.close()


def test_grid_hierarchy_per_step_replays_the_oracle():
    """tr_set_grids: the grids visited after each grey solve chosen step by
    step (sub-hierarchies of the context's 64,32,16,8,4,1: two-grid, W through
    one grid, F over two or four grids), each step replayed against the
    oracle's step with the same schedule at 1e-10, with equal low-order solve
    counts."""
    from test_gpu_step import _compare_state

    slab = inputs.make_slab(40, 64, 8, dt=0.004)
    levels = [64, 32, 16, 8, 4, 1]
    cfg = inputs.SolverCfg(levels=levels, cycle=inputs.CYCLE_F, lmax=2)
    plan = [((), 2), ((2,), 1), ((4, 2), 2), ((3, 1), 1), ((1,), 2), ((4, 3, 2, 1), 1)]
    pb = mlqd.problem_from_slab(slab)
    ost = mlqd.initial_state(pb, slab.T0)
    sv = binding.Solver([slab], [levels], cfg)
    st = sv.new_state()
    sv.state_init(st, slab.T0)
    for j, (grids, lmax) in enumerate(plan):
        stats = mlqd.Stats()
        ost = mlqd.step(pb, levels, list(grids), lmax, cfg.eps, cfg.eps_inner, ost, stats=stats)
        note(f"grids {grids} lmax {lmax}: counts {stats.counts[0]}")
        sv.set_grids(grids, lmax)
        gs = sv.step(st, replay=[stats.counts[0]])
        assert gs[0].n_lo == stats.n_lo
        _compare_state(f"grids {grids} step {j}", sv, st, ost)
    with pytest.raises(binding.TrError):
        sv.set_grids((5,), 1)
    with pytest.raises(binding.TrError):
        sv.set_grids((2, 2), 1)
    sv.close()
