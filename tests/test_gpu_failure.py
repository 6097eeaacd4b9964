"""Failure paths and reproducibility of tr_step on the GPU.  Each failure is
forced from the host (every kernel still runs to its normal end): too few
transport iterations allowed, a non-finite temperature in the state, and a
closure whose every prediction is rejected.  Two runs are bitwise identical,
and a run resumed from a copy of its state in a fresh context equals the
uninterrupted run bitwise."""
import numpy as np
import pytest
import torch

from oracle import mlqd
from paper_2011_05427_amd import binding, inputs

from gpu_util import note, to_np

pytestmark = pytest.mark.gpu

TR_ENOCONV, TR_ENAN = -4, -5
LEVELS = [16, 4, 1]


def _slab():
    return inputs.make_slab(30, 16, 8, dt=0.004)


def _solver(slab, **kw):
    cfg = inputs.SolverCfg(levels=LEVELS, cycle=inputs.CYCLE_W, lmax=2, **kw)
    sv = binding.Solver([slab], [LEVELS], cfg)
    st = sv.new_state()
    sv.state_init(st, slab.T0)
    return sv, st


def test_too_few_transport_iterations_is_enoconv():
    slab = _slab()
    pb = mlqd.problem_from_slab(slab)
    note("max_outer = 1")
    with pytest.raises(mlqd.NonConvergence):
        mlqd.step(pb, LEVELS, [1], 2, 1e-10, 1e-11, mlqd.initial_state(pb, slab.T0), max_outer=1)
    sv, st = _solver(slab, max_outer=1)
    with pytest.raises(binding.TrError) as err:
        sv.step(st)
    assert err.value.code == TR_ENOCONV
    sv.close()


def test_non_finite_temperature_is_enan():
    slab = _slab()
    sv, st = _solver(slab)
    sv.step(st)
    note("NaN in one cell of T")
    T = st["T"]
    T[7] = float("nan")
    torch.cuda.synchronize()
    with pytest.raises(binding.TrError) as err:
        sv.step(st)
    assert err.value.code == TR_ENAN
    sv.close()


def test_rejected_closure_predictions_leave_the_plain_step():
    """Weights of NaN make every predicted factor non-finite: each is rejected
    (the previous factor stays), so the step equals the plain one bitwise."""
    slab = _slab()
    outs = []
    for closure in (False, True):
        sv, st = _solver(slab)
        acc = (binding.TrStats * 1)()
        if closure:
            net = binding.Mlp(np.full(binding.load().tr_mlp_nparam(), np.nan, dtype=np.float32))
            sv.set_closure(net, np.zeros(7, np.float32), np.ones(7, np.float32))
        for _ in range(2):
            sv.step(st, stats=acc)
        if closure:
            assert acc[0].n_seeded == 0 and acc[0].n_fallback == 2 * slab.ng * slab.nx
        outs.append({k: to_np(v).copy() for k, v in st.items()})
        sv.close()
    for k in outs[0]:
        assert np.array_equal(outs[0][k], outs[1][k]), k


def test_two_runs_and_a_resumed_run_are_bitwise_identical():
    slab = _slab()
    note("4 steps twice; 2 + 2 steps with the state copied to the host between contexts")
    runs = []
    for _ in range(2):
        sv, st = _solver(slab)
        for _ in range(4):
            sv.step(st)
        runs.append({k: to_np(v).copy() for k, v in st.items()})
        sv.close()
    for k in runs[0]:
        assert np.array_equal(runs[0][k], runs[1][k]), k
    sv, st = _solver(slab)
    for _ in range(2):
        sv.step(st)
    ckpt = {k: v.cpu().clone() for k, v in st.items()}
    sv.close()
    sv, st = _solver(slab)
    for k, v in ckpt.items():
        st[k].copy_(v.to(st[k].device))
    torch.cuda.synchronize()
    for _ in range(2):
        sv.step(st)
    res = {k: to_np(v).copy() for k, v in st.items()}
    sv.close()
    for k in runs[0]:
        assert np.array_equal(res[k], runs[0][k]), k


def test_run_equals_single_steps():
    """tr_run of n steps (no return to the caller between steps) leaves the
    same state and counters as n calls of tr_step, bitwise, for an odd and an
    even n."""
    slab = _slab()
    for n in (3, 4):
        outs = []
        for multi in (False, True):
            sv, st = _solver(slab)
            acc = (binding.TrStats * 1)()
            if multi:
                sv.run(st, n, stats=acc)
            else:
                for _ in range(n):
                    sv.step(st, stats=acc)
            outs.append(({k: to_np(v).copy() for k, v in st.items()}, (acc[0].n_ti, acc[0].n_c, acc[0].n_lo)))
            sv.close()
        assert outs[0][1] == outs[1][1]
        for k in outs[0][0]:
            assert np.array_equal(outs[0][0][k], outs[1][0][k]), (n, k)
