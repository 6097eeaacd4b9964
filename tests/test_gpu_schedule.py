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
    return inputs.SolverCfg(levels=levels, cycle=cycle).schedule()


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
