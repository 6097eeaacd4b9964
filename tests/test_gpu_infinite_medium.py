"""T7 on the GPU: a spatially uniform slab whose boundaries receive the 0-D
solution reproduces the 0-D backward-Euler step (per-group energy balance
and the scalar material energy balance, solved here by root finding on the
CPU, independent of both the oracle's and the library's solvers)."""
import dataclasses

import numpy as np
import pytest
import torch

from oracle import mlqd, planck
from oracle.moments import factors
from paper_2011_05427_amd import binding, inputs

from gpu_util import note, to_np
from test_oracle_step import _zero_d

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("cycle", [inputs.CYCLE_V, inputs.CYCLE_W])
def test_uniform_medium_matches_zero_d_on_the_gpu(cycle):
    slab = inputs.make_slab(6, 8, 8, C1=5.0, C2=5.0, dt=0.01)
    pb = mlqd.problem_from_slab(slab)
    T_old = 0.3
    E_old = 2 * planck.planck_groups(pb.nu_edges, np.array([0.5]), pb.aR, pb.c)[:, 0] / pb.c
    T1, E1 = _zero_d(pb, T_old, E_old, pb.dt)
    inc = pb.c * E1 / 2
    pb = dataclasses.replace(pb, inc_left=inc, inc_right=inc)
    G, nx, M = pb.G, pb.nx, len(pb.mu)
    I = np.broadcast_to((pb.c * E_old / 2)[:, None, None, None], (G, M, nx, 2)).copy()
    fac = factors(pb.mu, pb.w, I, pb.inc_left, pb.inc_right, pb.c)
    levels = [8, 1] if cycle == inputs.CYCLE_V else [8, 2, 1]
    note(f"uniform medium, cycle {'VWF'[cycle]}")
    cfg = inputs.SolverCfg(levels=levels, cycle=cycle, lmax=3, eps=1e-13, eps_inner=1e-14)
    sv = binding.Solver([slab], [levels], cfg)
    sv.set_incoming(0, inc, inc)
    st = sv.new_state()
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64).ravel()).to("cuda")
    st["T"].copy_(dev(np.full(nx, T_old)))
    st["I_prev"].copy_(dev(I))
    st["E"].copy_(dev(np.broadcast_to(E_old[:, None], (G, nx))))
    st["F"].zero_()
    st["Ebnd"].copy_(dev(np.stack([E_old, E_old], axis=1)))
    st["f"].copy_(dev(fac.f))
    st["fbnd"].copy_(dev(fac.f_bnd))
    st["C"].copy_(dev(fac.C))
    st["Egrey"].copy_(dev(np.full(nx, E_old.sum())))
    torch.cuda.synchronize()
    sv.step(st)
    T = to_np(st["T"])
    E = to_np(st["E"]).reshape(G, nx)
    F = to_np(st["F"]).reshape(G, nx + 1)
    np.testing.assert_allclose(T, T1, rtol=1e-11)
    np.testing.assert_allclose(E, np.broadcast_to(E1[:, None], E.shape), rtol=1e-10, atol=1e-12 * E1.max())
    assert np.max(np.abs(F.sum(axis=0))) < 1e-9 * pb.c * E1.sum()
    sv.close()
