"""GPU parity on the paper's Fleck-Cummings set-up (10 cells, 256 groups,
double S8, eps = 1e-6, the group averages of the spectral opacity): steps of
three of the Tables 1-2 algorithms replayed against the oracle (1e-10), one
with the point opacity law, and free-running steps reaching the oracle's
iteration counts."""
import pytest

from oracle import mlqd
from paper_2011_05427_amd import binding, inputs

from gpu_util import note, rel_err, to_np
from test_gpu_step import _compare_state

pytestmark = pytest.mark.gpu

ROWS = [(0.02, [256, 32, 1], inputs.CYCLE_W, 2), (0.02, [256, 32, 16, 4, 1], inputs.CYCLE_F, 2),
        (0.04, [256, 1], inputs.CYCLE_V, 6)]


@pytest.mark.parametrize("row,opac", [(0, inputs.OPAC_SPECTRAL), (1, inputs.OPAC_SPECTRAL),
                                      (2, inputs.OPAC_SPECTRAL), (1, inputs.OPAC_POINT)])
def test_fc_steps_replay_the_oracle(row, opac):
    dt, levels, cyc, lmax = ROWS[row]
    slabs, cfg, _ = inputs.config_fc(dt, levels, cyc, lmax, opacity=opac)
    s = slabs[0]
    note(f"FC dt={dt} grids={levels} cycle={'VWF'[cyc]} lmax={lmax} opacity={'point spectral'.split()[opac]}")
    pb = mlqd.problem_from_slab(s)
    ost = mlqd.initial_state(pb, s.T0)
    sv = binding.Solver(slabs, [levels], cfg)
    st = sv.new_state()
    sv.state_init(st, s.T0)
    for j in range(2):
        stats = mlqd.Stats()
        ost = mlqd.step(pb, levels, mlqd.schedule(len(levels), cfg.cycle), lmax, cfg.eps, cfg.eps_inner, ost, stats=stats)
        gs = sv.step(st, replay=[stats.counts[0]])
        assert gs[0].n_lo == stats.n_lo
        _compare_state(f"FC row {row} opacity {opac} step {j}", sv, st, ost)
    sv.close()


def test_fc_free_running_counts_match_the_oracle():
    dt, levels, cyc, lmax = ROWS[1]
    slabs, cfg, _ = inputs.config_fc(dt, levels, cyc, lmax)
    s = slabs[0]
    note("FC free run, F cycle, spectral opacities, 3 steps")
    pb = mlqd.problem_from_slab(s)
    ost = mlqd.initial_state(pb, s.T0)
    stats = mlqd.Stats()
    sv = binding.Solver(slabs, [levels], cfg)
    st = sv.new_state()
    sv.state_init(st, s.T0)
    acc = (binding.TrStats * 1)()
    for _ in range(3):
        ost = mlqd.step(pb, levels, mlqd.schedule(len(levels), cfg.cycle), lmax, cfg.eps, cfg.eps_inner, ost, stats=stats)
        sv.step(st, stats=acc)
    assert (acc[0].n_ti, acc[0].n_c, acc[0].n_lo) == (stats.n_ti, stats.n_c, stats.n_lo)
    assert rel_err(to_np(st["T"]), ost.T) < 1e-10
    sv.close()
