"""The Fleck-Cummings set-up of the paper's Sec. 6 (inputs.fc_slab): the
group grid, the double S8 rule and the material constants it states, and one
oracle step on it."""
import numpy as np
import pytest

from oracle import mlqd
from paper_2011_05427_amd import inputs


def test_fc_grid_quadrature_and_constants():
    s = inputs.fc_slab(0.02)
    assert (s.nx, s.ng, s.nmu) == (10, 256, 16)
    assert np.allclose(np.diff(s.x_edges), 0.4) and s.x_edges[-1] == pytest.approx(4.0)
    # 254 groups log-spaced between 1e-4 and 10 keV, end groups to 0 and inf
    e = s.nu_edges
    assert e[0] == 0.0 and np.isinf(e[-1])
    assert e[1] == pytest.approx(1e-4, rel=1e-12) and e[255] == pytest.approx(10.0, rel=1e-12)
    ratio = e[2:256] / e[1:255]
    assert np.allclose(ratio, (1e5) ** (1 / 254), rtol=1e-12)
    # double S8: 8-point Gauss rule on each half range (exact to degree 15 there)
    pos = s.mu > 0
    assert pos.sum() == 8 and np.allclose(s.mu, -s.mu[::-1])
    for k in range(16):
        assert np.sum(s.w[pos] * s.mu[pos] ** k) == pytest.approx(1.0 / (k + 1), rel=1e-13)
    assert s.cv == pytest.approx(0.5917 * inputs.A_RAD) and s.T0 == 1e-3 and s.T_left == 1.0
    assert np.all(s.C_cell == 27.0)
    for dt, n in zip(inputs.FC_DT, (150, 75)):
        _, cfg, nsteps = inputs.config_fc(dt)
        assert nsteps == n and cfg.eps == 1e-6 and cfg.eps_inner == 1e-7


def test_fc_first_step_heats_from_the_left():
    slabs, cfg, _ = inputs.config_fc(0.02, [256, 32, 1], inputs.CYCLE_W, 2)
    s = slabs[0]
    pb = mlqd.problem_from_slab(s)
    st = mlqd.initial_state(pb, s.T0)
    stats = mlqd.Stats()
    new = mlqd.step(pb, cfg.levels, mlqd.schedule(len(cfg.levels), cfg.cycle), cfg.lmax, cfg.eps, cfg.eps_inner, st, stats=stats)
    # radiation enters at x = 0: temperature falls off monotonically into the slab
    assert np.all(np.diff(new.T) < 0) and new.T[0] > 0.05 and new.T.min() >= s.T0
    assert all(1 <= c <= cfg.lmax for c in stats.counts[0])
