"""Binary32 storage of the corner intensities: the sweep still computes in
binary64, so its output equals the oracle's on the float-rounded input up to
the final rounding, its moments equal the binary64 moments, and whole steps
converge to within the stated error of the binary64 run."""
import numpy as np
import pytest

from oracle import planck
from oracle.moments import factors
from oracle.sweep import sweep
from paper_2011_05427_amd import binding, inputs

from gpu_util import assert_close, note, rel_err, to_dev, to_np

pytestmark = pytest.mark.gpu


def test_fp32_storage_sweep():
    note("fp32-storage sweep")
    import torch

    slab = inputs.make_slab(300, 3, 16, T_left=1.0, T_right=0.5)
    cfg = inputs.SolverCfg(levels=[3, 1], precision=1)
    sv = binding.Solver([slab], [[3, 1]], cfg)
    rng = np.random.default_rng(9)
    kap = 10 ** rng.uniform(-2, 4, (3, 300))
    B = rng.uniform(0, 1, (3, 300))
    Ip = rng.uniform(0, 1, (3, 16, 300, 2)).astype(np.float32)
    Io = torch.zeros(Ip.size, dtype=torch.float32, device="cuda")
    mom, bnd = sv.empty(binding.TR_K_GI, 4), sv.empty(binding.TR_K_G, 6)
    sv.sweep(to_dev(kap), to_dev(B), torch.as_tensor(Ip.ravel()).to("cuda"), Io, mom, bnd)
    f, fb, Cb, Phi = (sv.empty(binding.TR_K_GI), sv.empty(binding.TR_K_G2), sv.empty(binding.TR_K_G2),
                      sv.empty(binding.TR_K_G2))
    sv.moments(mom, bnd, f, fb, Cb, Phi)
    il = planck.boundary_intensity(slab.nu_edges, 1.0, slab.aR, slab.c)
    ir = planck.boundary_intensity(slab.nu_edges, 0.5, slab.aR, slab.c)
    ref = sweep(slab.mu, slab.x_edges, kap, B, Ip.astype(np.float64), il, ir, slab.c, slab.dt)
    got = to_np(Io).reshape(ref.shape).astype(np.float64)
    np.testing.assert_allclose(got, ref.astype(np.float32).astype(np.float64), rtol=2.5e-7, atol=1e-37)
    fac = factors(slab.mu, slab.w, ref, il, ir, slab.c)
    assert_close("f", to_np(f, (3, 300)), fac.f, 1e-12)
    assert_close("C", to_np(Cb, (3, 2)), fac.C, 1e-12)
    sv.close()


def test_fp32_storage_steps_error_vs_fp64():
    slab = inputs.make_slab(70, 64, 16, dt=0.002)
    levels = [64, 16, 4, 1]
    out = {}
    for prec in (0, 1):
        note(f"F-cycle steps, precision {prec}")
        cfg = inputs.SolverCfg(levels=levels, cycle=inputs.CYCLE_F, lmax=2, precision=prec)
        sv = binding.Solver([slab], [levels], cfg)
        st = sv.new_state()
        sv.state_init(st, slab.T0)
        acc = (binding.TrStats * 1)()
        for _ in range(5):
            sv.step(st, stats=acc)
        out[prec] = (to_np(st["T"]).copy(), to_np(st["E"]).copy(), acc[0].n_ti)
        sv.close()
    eT = rel_err(out[1][0], out[0][0])
    eE = rel_err(out[1][1], out[0][1])
    print(f"fp32 storage vs fp64 after 5 steps: T {eT:.2e}, E {eE:.2e}; sweeps {out[1][2]} vs {out[0][2]}",
          flush=True)
    assert eT < 1e-5 and eE < 1e-5
