"""GPU parity of the learned closure's MFMA kernels against the FP64 reference
(same bfloat16 rounding points, float32 accumulation on the GPU): forward
outputs and gradients per parameter tensor to relative Frobenius error 1e-2
and cosine 0.9999, one Adam step, closure inputs and training targets; then
training on the solver's own steps and a learned run that must converge to
the plain method's answer."""
import numpy as np
import pytest

from oracle import mlp, mlqd, planck
from paper_2011_05427_amd import binding, closure, inputs

from gpu_util import note, rel_err, to_dev, to_np

pytestmark = pytest.mark.gpu


def _f32(a):
    import torch

    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32)).to("cuda")


def _cos(a, b):
    a, b = np.ravel(a), np.ravel(b)
    return float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b) + 1e-300))


def _data(n, seed):
    rng = np.random.default_rng(seed)
    X = np.zeros((n, 8))
    X[:, :mlp.NIN] = rng.normal(0, 1, (n, mlp.NIN))
    Y = np.stack([rng.uniform(0.2, 0.6, n), rng.normal(0, 0.2, n)], axis=1)
    return X, Y


@pytest.mark.parametrize("n", [1, 77, 1000])
def test_forward_matches_reference(n):
    note(f"mlp forward n={n}")
    theta = mlp.init_params(3)
    X, _ = _data(n, n)
    net = binding.Mlp(theta)
    out = to_np(net.forward(_f32(X))).reshape(n, 2)
    ref, _ = mlp.forward(theta, X[:, :mlp.NIN], bf16=True)
    assert rel_err(out, ref) < 1e-2
    assert _cos(out[:, 1], ref[:, 1]) > 0.9999 or n == 1
    assert np.max(np.abs(out[:, 0] - ref[:, 0])) < 1e-2


@pytest.mark.parametrize("n", [64, 333])
def test_gradients_match_reference(n):
    note(f"mlp grad n={n}")
    theta = mlp.init_params(4)
    X, Y = _data(n, 10 + n)
    net = binding.Mlp(theta)
    g, loss = net.grad(_f32(X), _f32(Y))
    g = to_np(g).astype(np.float64)
    lref, gref = mlp.loss_and_grad(theta, X[:, :mlp.NIN], Y, bf16=True)
    assert abs(float(to_np(loss)[0]) - lref) <= 1e-3 * lref
    o = 0
    for name, shp in mlp.SHAPES:
        k = int(np.prod(shp))
        a, b = g[o:o + k], gref[o:o + k]
        if name == "W1":  # padded input rows carry no gradient
            a, b = a[:mlp.NIN * mlp.NH], b[:mlp.NIN * mlp.NH]
        assert rel_err(a, b) < 1e-2, name
        assert _cos(a, b) > 0.9999, name
        o += k


def test_adam_step_matches_reference():
    theta = mlp.init_params(5)
    rng = np.random.default_rng(1)
    grad = rng.normal(0, 1e-2, theta.size)
    net = binding.Mlp(theta)
    for _ in range(3):
        net.adam(_f32(grad), 1e-3)
    th, m, v = theta.copy(), np.zeros_like(theta), np.zeros_like(theta)
    for t in range(1, 4):
        th, m, v = mlp.adam_step(th, m, v, grad, t)
    assert np.max(np.abs(to_np(net.params) - th)) < 1e-6


def test_features_and_targets_match_reference():
    slab = inputs.make_slab(37, 24, 4, T_left=0.9)
    levels = [24, 6, 1]
    sv = binding.Solver([slab], [levels], inputs.SolverCfg(levels=levels))
    rng = np.random.default_rng(2)
    T = 10 ** rng.uniform(-3, 0, slab.nx)
    Tp = T * rng.uniform(0.7, 1.3, slab.nx)
    kap = planck.opacity(slab.nu_center, slab.C_cell, T)
    fp = rng.uniform(0.2, 0.6, (24, slab.nx))
    mean, std = rng.normal(0, 1, mlp.NIN), rng.uniform(0.5, 2, mlp.NIN)
    for T_prev in (None, Tp):
        X = sv.empty(binding.TR_K_GI, 8).float()
        sv.mlp_features(to_dev(T), None if T_prev is None else to_dev(T_prev), to_dev(kap), to_dev(fp), mean, std, X)
        ref = mlp.standardise(mlp.features(T, slab.nu_center, kap, np.diff(slab.x_edges), slab.T_left, fp, T_prev),
                              mean, std)
        got = to_np(X).reshape(-1, 8)
        np.testing.assert_allclose(got[:, :mlp.NIN], ref, rtol=1e-5, atol=1e-5)
        assert np.all(got[:, mlp.NIN:] == 0)
    f = fp + rng.uniform(-0.08, 0.08, (24, slab.nx))
    En = 10 ** rng.uniform(-5, 0, (24, slab.nx))
    Ep = 10 ** rng.uniform(-5, 0, (24, slab.nx))
    Y = sv.empty(binding.TR_K_GI, 2).float()
    sv.closure_targets(to_dev(f), to_dev(fp), to_dev(En), to_dev(Ep), 4, Y)
    np.testing.assert_allclose(to_np(Y).reshape(-1, 2), mlp.targets(f, fp, En, Ep, 4), rtol=2e-6, atol=1e-6)
    sv.close()


@pytest.mark.parametrize("with_prev", [False, True])
def test_fused_seeding_matches_three_call_path(with_prev):
    """tr_closure_seed (inputs, network and seeding in one kernel; the
    weights are the A operand and the activations stay in registers between
    layers) against the three-call path over a two-slab context with ragged
    256-sample items: tr_mlp_features, tr_mlp_forward, then the seeding
    formula f + 0.05 (2 s - 1) kept inside (0, 1).  Both run the network in
    bfloat16 with float32 accumulation, in different orders (the products'
    sums differ in the last float32 bits): seeded factors agree to 1e-5."""
    import torch

    slabs = [inputs.make_slab(37, 24, 4, T_left=0.9), inputs.make_slab(53, 40, 8, C1=9.0)]
    levels = [[24, 6, 1], [40, 10, 1]]
    sv = binding.Solver(slabs, levels, inputs.SolverCfg(levels=levels[0]))
    note(f"fused seeding, 2 slabs, T_prev={'yes' if with_prev else 'no'}")
    rng = np.random.default_rng(11)
    theta = mlp.init_params(6)
    net = binding.Mlp(theta)
    mean, std = rng.normal(0, 1, mlp.NIN), rng.uniform(0.5, 2, mlp.NIN)
    T = np.concatenate([10 ** rng.uniform(-3, 0, s.nx) for s in slabs])
    Tp = T * rng.uniform(0.7, 1.3, T.size)
    kap = np.concatenate([planck.opacity(s.nu_center, s.C_cell, T[o:o + s.nx]).ravel()
                          for s, o in zip(slabs, sv.offsets(binding.TR_K_CELL))])
    f = rng.uniform(0.02, 0.98, sv.total(binding.TR_K_GI))
    f[:40] = rng.uniform(0.0, 0.03, 40)  # seeds that may leave (0, 1) are kept
    T_prev = to_dev(Tp) if with_prev else None
    X = sv.empty(binding.TR_K_GI, 8).float()
    sv.mlp_features(to_dev(T), T_prev, to_dev(kap), to_dev(f), mean, std, X)
    out = to_np(net.forward(X.reshape(-1, 8))).reshape(-1, 2).astype(np.float64)
    cand = f + 0.05 * (2.0 * out[:, 0] - 1.0)
    inside = (cand > 0.0) & (cand < 1.0)
    ref = np.where(inside, cand, f)
    sv.set_closure(net, mean, std)
    fd = to_dev(f)
    counts = torch.zeros(2, dtype=torch.int64, device="cuda")
    sv.closure_seed(to_dev(T), T_prev, to_dev(kap), fd, counts)
    got = to_np(fd)
    c = to_np(counts)
    print(f"fused seeding: seeded {c[0]} kept {c[1]} of {f.size}; max |f - ref| {np.max(np.abs(got - ref)):.2e}",
          flush=True)
    assert int(c[0]) + int(c[1]) == f.size
    assert abs(int(c[1]) - int(np.sum(~inside))) <= 2
    assert np.max(np.abs(got - ref)) < 1e-5
    sv.set_closure(None)
    with pytest.raises(binding.TrError):
        sv.closure_seed(to_dev(T), T_prev, to_dev(kap), fd, counts)  # no closure attached
    sv.close()


def test_training_and_learned_steps_converge_to_plain():
    """The closure trained on one slab's plain steps seeds a held-out slab
    (other opacity constants and boundary temperature, 32 directions, where a
    sweep costs most relative to inference): the learned steps reach the
    plain solution to 1e-10 (the plain sweeps decide convergence), and the
    test reports what the network gains or costs in sweeps and ms per step.
    The seeding saves at most a fraction of a sweep per step here (exact
    seeds save about a quarter of the sweeps), so the assertion on the gain
    is only that seeding costs at most one extra sweep per step."""
    import time

    import torch

    levels = [32, 8, 1]
    cfg = inputs.SolverCfg(levels=levels, cycle=inputs.CYCLE_W, lmax=2, eps=1e-12, eps_inner=1e-13)
    train_slab = inputs.make_slab(50, 32, 32, dt=0.004)
    test_slab = inputs.make_slab(60, 32, 32, dt=0.004, C1=20.0, C2=4.0, T_left=0.9)
    note("closure: data and training on one slab, learned vs plain on a held-out slab")
    ds = closure.generate(train_slab, cfg, levels, nsteps=8, n_samples=8 * 32 * 50, seed=0)
    net, losses = closure.train(ds, epochs=30, batch=256, lr=2e-3, seed=0)
    print("closure losses", losses[0], losses[-1], flush=True)
    assert losses[-1] < 0.5 * losses[0]
    nsteps = 8
    runs = {}
    for learned in (False, True):
        sv = binding.Solver([test_slab], [levels], cfg)
        if learned:
            sv.set_closure(net, ds.mean, ds.std)
        st = sv.new_state()
        sv.state_init(st, test_slab.T0)
        sv.step(st)  # graphs
        sv.state_init(st, test_slab.T0)
        acc = (binding.TrStats * 1)()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(nsteps):
            sv.step(st, stats=acc)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / nsteps
        runs[learned] = (to_np(st["T"]).copy(), to_np(st["E"]).copy(), acc[0].n_ti, acc[0].n_seeded,
                         acc[0].n_fallback, ms, acc[0].n_c)
        sv.close()
    p, q = runs[False], runs[True]
    print(f"closure gain on the held-out slab: sweeps plain {p[2]} learned {q[2]} ({p[2] - q[2]:+d}), "
          f"cycles {p[6]} / {q[6]}, ms/step plain {p[5]:.3f} learned {q[5]:.3f} (speedup {p[5] / q[5]:.2f}), "
          f"seeded {q[3]} fallback {q[4]}", flush=True)
    assert q[3] > 0
    assert q[2] <= p[2] + nsteps
    assert rel_err(q[0], p[0]) < 1e-10
    assert rel_err(q[1], p[1]) < 1e-10


@pytest.mark.parametrize("with_r", [False, True])
def test_prolong_matches_oracle(with_r):
    """tr_prolong on a batch of two slabs (levels G, G/8, 1), every coarse level,
    against the oracle prolongation; includes a cell whose block is empty."""
    from oracle.prolong import prolong

    slabs = [inputs.make_slab(37, 32, 8), inputs.make_slab(70, 64, 8, C1=5.0)]
    levels = [[s.ng, s.ng // 8, 1] for s in slabs]
    cfg = inputs.SolverCfg(levels=[0, 0, 1], cycle=inputs.CYCLE_W, lmax=2)
    note(f"prolong, r={'closure output' if with_r else 'none'}")
    sv = binding.Solver(slabs, levels, cfg)
    rng = np.random.default_rng(11)
    n_gi = sv.total(binding.TR_K_GI)
    Eprev = 10.0 ** rng.uniform(-9, 1, size=n_gi)
    o1 = sv.layout(binding.TR_K_GI, 1)[0]
    Eprev[o1 + 5 * 70 + 3: o1 + 5 * 70 + 4] = 0.0  # one cell of one fine group
    Eprev_blk = Eprev.copy()
    for g in range(8):  # block 0 of level 1 in cell 11 of slab 1: empty
        Eprev_blk[o1 + g * 70 + 11] = 0.0
    r = rng.uniform(-2, 2, size=(n_gi, 2)).astype(np.float32) if with_r else None
    for lev in (1, 2):
        n_pi = sv.total(binding.TR_K_LEV_PI + lev)
        Ec = 10.0 ** rng.uniform(-4, 0, size=n_pi)
        out = sv.empty(binding.TR_K_GI)
        rd = None
        if r is not None:
            import torch

            rd = torch.as_tensor(np.ascontiguousarray(r).ravel()).to("cuda")  # float32 [gi][2]
        sv.prolong(lev, to_dev(Ec), to_dev(Eprev_blk), rd, out)
        got = to_np(out)
        for k, s in enumerate(slabs):
            og = sv.layout(binding.TR_K_GI, k)[0]
            op = sv.layout(binding.TR_K_LEV_PI + lev, k)[0]
            npl = levels[k][lev]
            Ep = Ec[op:op + npl * s.nx].reshape(npl, s.nx)
            Epr = Eprev_blk[og:og + s.ng * s.nx].reshape(s.ng, s.nx)
            rr = None if r is None else r[og:og + s.ng * s.nx, 1].astype(np.float64).reshape(s.ng, s.nx)
            want = prolong(Ep, Epr, rr)
            have = got[og:og + s.ng * s.nx].reshape(s.ng, s.nx)
            assert rel_err(have, want) < 1e-13, (lev, k, rel_err(have, want))
    sv.close()
