"""Batched path (many uneven slabs per launch) and its tiles: every sweep tile
agrees with the oracle; a slab solved inside a batch equals the same slab
solved alone bit for bit; sampled slabs of a batch match their own oracle
runs; the autotuner keeps a valid tile per bucket."""
import numpy as np
import pytest

from oracle import mlqd, planck
from oracle.moments import factors
from oracle.sweep import sweep
from paper_2011_05427_amd import binding, inputs, tuning

from gpu_util import assert_close, note, to_dev, to_np

pytestmark = pytest.mark.gpu


TILES = [(K, S, 16) for K in (1, 2, 4, 8) for S in (1, 2, 4)] + [(2, 2, 6), (4, 4, 6), (1, 4, 2), (8, 2, 2)]


# (K, split, nmu, nx): several passes of 64 K cells per wavefront with a
# partial last pass, up to the large workload's 2000 cells and 32 directions
MULTI_PASS = [(8, 1, 32, 1300), (8, 2, 32, 1300), (8, 4, 32, 1300), (4, 4, 32, 1100), (8, 4, 32, 2000),
              (8, 2, 16, 1100), (2, 1, 8, 1100)]


@pytest.mark.parametrize("K,S,nmu", TILES)
def test_every_sweep_tile_matches_oracle(K, S, nmu):
    """Every tile (K cells per lane, S wavefronts sharing a group's half range)
    against the oracle sweep, incl. direction counts that S does not divide
    (wavefronts with one or no direction)."""
    _tile_case(K, S, nmu, 300)


@pytest.mark.parametrize("K,S,nmu,nx", MULTI_PASS)
def test_multi_pass_sweep_tiles_match_oracle(K, S, nmu, nx):
    """Tiles whose wavefronts cross the slab in several passes (the carry of
    the inflow from one pass to the next), incl. the tile the autotuner picks
    for slabs above 1024 cells."""
    _tile_case(K, S, nmu, nx)


def _tile_case(K, S, nmu, nx):
    note(f"sweep tile K={K} split={S} nmu={nmu} nx={nx}")
    slab = inputs.make_slab(nx, 3, nmu, T_left=1.0, T_right=0.5)
    sv = binding.Solver([slab], [[3, 1]], inputs.SolverCfg(levels=[3, 1]))
    sv.set_tiles([K] * 6, [S] * 6)
    assert sv.get_tiles()[:2] == ([K] * 6, [S] * 6)
    rng = np.random.default_rng(K + 10 * S + nmu + nx)
    kap = 10 ** rng.uniform(-2, 4, (3, nx))
    # the first group optically thin everywhere: its inflow crosses every pass
    kap[0] = 10 ** rng.uniform(-3, -1, nx)
    B = rng.uniform(0, 1, (3, nx))
    Ip = rng.uniform(0, 1, (3, nmu, nx, 2))
    Io = sv.empty(binding.TR_K_I)
    mom, bnd = sv.empty(binding.TR_K_GI, 4), sv.empty(binding.TR_K_G, 6)
    sv.sweep(to_dev(kap), to_dev(B), to_dev(Ip), Io, mom, bnd)
    f, fb, Cb, Phi = (sv.empty(binding.TR_K_GI), sv.empty(binding.TR_K_G2), sv.empty(binding.TR_K_G2),
                      sv.empty(binding.TR_K_G2))
    sv.moments(mom, bnd, f, fb, Cb, Phi)
    il = planck.boundary_intensity(slab.nu_edges, 1.0, slab.aR, slab.c)
    ir = planck.boundary_intensity(slab.nu_edges, 0.5, slab.aR, slab.c)
    ref = sweep(slab.mu, slab.x_edges, kap, B, Ip, il, ir, slab.c, slab.dt)
    fac = factors(slab.mu, slab.w, ref, il, ir, slab.c)
    got = to_np(Io, ref.shape)
    for g in range(3):
        assert_close(f"I g={g}", got[g], ref[g], 1e-12)
    assert_close("f", to_np(f, (3, nx)), fac.f, 1e-12)
    assert_close("C", to_np(Cb, (3, 2)), fac.C, 1e-12)
    sv.close()


def _batch(n):
    slabs, cfg, _ = inputs.config_batch(n)
    levels = [inputs.levels_for(s, cfg) for s in slabs]
    return slabs, levels, cfg


def _slab_view(sv, st, k):
    s = sv.slabs[k]
    oc = sv.layout(binding.TR_K_CELL, k)[0]
    ogi = sv.layout(binding.TR_K_GI, k)[0]
    oI = sv.layout(binding.TR_K_I, k)[0]
    return (to_np(st["T"])[oc:oc + s.nx].copy(), to_np(st["E"])[ogi:ogi + s.ng * s.nx].copy(),
            to_np(st["I_prev"])[oI:oI + s.ng * s.nmu * s.nx * 2].copy())


def test_batched_equals_individual():
    slabs, levels, cfg = _batch(20)
    note("batch of 20 slabs from the uneven-batch distribution, one free-running step")
    sv = binding.Solver(slabs, levels, cfg)
    st = sv.new_state()
    sv.state_init(st, 0.001)
    sv.step(st)
    batched = {k: _slab_view(sv, st, k) for k in (0, 7, 13)}
    sv.close()
    for k, ref in batched.items():
        one = binding.Solver([slabs[k]], [levels[k]], cfg)
        s1 = one.new_state()
        one.state_init(s1, 0.001)
        one.step(s1)
        got = _slab_view(one, s1, 0)
        one.close()
        for a, b, name in zip(got, ref, ("T", "E", "I")):
            assert np.array_equal(a, b), (k, name)


def test_wide_slab_in_a_batch_equals_alone():
    """A 1000-cell slab (16 edge tiles: the chunk widths of the restriction
    follow the slab alone) beside a small one: one free-running F-cycle step
    of each inside the batch equals the step of the slab alone bit for bit."""
    import dataclasses

    _, cfg0, _ = inputs.config_large()
    cfg = dataclasses.replace(cfg0, cycle=inputs.CYCLE_F, lmax=1)
    slabs = [inputs.make_slab(1000, 256, 4), inputs.make_slab(100, 64, 4, C1=10.0, T_left=0.8)]
    levels = [[256, 16, 4, 1], [64, 16, 4, 1]]
    note("wide slab (1000 cells, 256 groups) and a small one, batched vs alone, one F step")
    sv = binding.Solver(slabs, levels, cfg)
    st = sv.new_state()
    sv.state_init(st, 0.001)
    sv.step(st)
    batched = {k: _slab_view(sv, st, k) for k in range(2)}
    sv.close()
    for k, ref in batched.items():
        one = binding.Solver([slabs[k]], [levels[k]], cfg)
        s1 = one.new_state()
        one.state_init(s1, 0.001)
        one.step(s1)
        got = _slab_view(one, s1, 0)
        one.close()
        for a, b, name in zip(got, ref, ("T", "E", "I")):
            assert np.array_equal(a, b), (k, name)


def test_batch_sampled_slabs_match_oracle():
    slabs, levels, cfg = _batch(20)
    small = sorted(range(20), key=lambda k: slabs[k].ng * slabs[k].nx * slabs[k].nmu)[:2]
    refs = {}
    for k in small:
        pb = mlqd.problem_from_slab(slabs[k])
        st0 = mlqd.initial_state(pb, 0.001)
        stats = mlqd.Stats()
        sched = mlqd.schedule(len(levels[k]), cfg.cycle)
        refs[k] = (mlqd.step(pb, levels[k], sched, cfg.lmax, cfg.eps, cfg.eps_inner, st0, stats=stats),
                   stats.counts[0])
    note(f"batch of 20, replay on slabs {small}")
    sv = binding.Solver(slabs, levels, cfg)
    tuning.tune(sv, _init(sv), reps=1, path=None)
    st = _init(sv)
    replay = [refs[k][1] if k in refs else [0] for k in range(20)]
    sv.step(st, replay=replay)
    for k, (ref, _) in refs.items():
        T, E, I = _slab_view(sv, st, k)
        assert_close(f"slab {k} T", T, ref.T, 1e-10, atol_scale=0.0)
        assert_close(f"slab {k} E", E.reshape(ref.E.shape), ref.E, 1e-10)
        assert_close(f"slab {k} I", I.reshape(ref.I.shape), ref.I, 1e-10)
    K, S, items = sv.get_tiles()
    assert all(k in (1, 2, 4, 8) for k in K)
    assert all(k in (1, 2, 4) for k in S)
    assert sum(items) == sum(s.ng for s in slabs)
    sv.close()


def _bucket_cover(instances):
    """Indices of batch instances that cover every populated slab-size bucket
    of the sweep (nx <= 64, 128, 256, 512) and every group count, the
    1024-group slabs among them: per bucket the instance with the most
    groups, plus the smallest and the largest slab of the batch."""
    bounds = [64, 128, 256, 512]
    pick = set()
    for lo, hi in zip([0] + bounds[:-1], bounds):
        inb = [k for k, d in enumerate(instances) if lo < d["nx"] <= hi]
        if inb:
            pick.add(max(inb, key=lambda k: (instances[k]["ng"], instances[k]["nx"])))
    for G in (64, 128, 256, 512, 1024):
        ing = [k for k, d in enumerate(instances) if d["ng"] == G]
        if ing and not any(instances[k]["ng"] == G for k in pick):
            pick.add(min(ing, key=lambda k: instances[k]["nx"]))
    cost = lambda k: instances[k]["nx"] * instances[k]["ng"] * instances[k]["nmu"]
    pick.add(min(range(len(instances)), key=cost))
    pick.add(max(range(len(instances)), key=cost))
    return sorted(pick)


def test_batch_replay_covers_every_bucket_and_group_count():
    """One replayed step of slabs that cover every populated size bucket and
    every group count of the uneven-batch distribution (incl. 1024 groups and
    the largest slab), solved together in one batch with the autotuned tiles,
    each against its own oracle run at 1e-10."""
    inst = inputs.batch_instances(256)
    ks = _bucket_cover(inst)
    slabs, cfg, _ = inputs.config_batch(256)
    slabs = [slabs[k] for k in ks]
    levels = [inputs.levels_for(s, cfg) for s in slabs]
    assert {s.ng for s in slabs} == {64, 128, 256, 512, 1024}
    assert len({min(4, max(0, (s.nx - 1).bit_length() - 6)) for s in slabs}) == 4
    refs = []
    for s, lv in zip(slabs, levels):
        pb = mlqd.problem_from_slab(s)
        stats = mlqd.Stats()
        ref = mlqd.step(pb, lv, mlqd.schedule(len(lv), cfg.cycle), cfg.lmax, cfg.eps, cfg.eps_inner,
                        mlqd.initial_state(pb, 0.001), stats=stats)
        refs.append((ref, stats.counts[0]))
    note(f"batch of instances {ks}: nx={[s.nx for s in slabs]} ng={[s.ng for s in slabs]}, one replayed step")
    sv = binding.Solver(slabs, levels, cfg)
    tuning.tune(sv, _init(sv), reps=1, path=None)
    note(f"  tiles {sv.get_tiles()}")
    st = _init(sv)
    stats = sv.step(st, replay=[c for _, c in refs])
    for k, (ref, counts) in enumerate(refs):
        assert list(stats[k].cycles[:len(counts)]) == counts
        T, E, I = _slab_view(sv, st, k)
        assert_close(f"slab {ks[k]} T", T, ref.T, 1e-10, atol_scale=0.0)
        assert_close(f"slab {ks[k]} E", E.reshape(ref.E.shape), ref.E, 1e-10)
        assert_close(f"slab {ks[k]} I", I.reshape(ref.I.shape), ref.I, 1e-10)
    sv.close()


def _init(sv):
    st = sv.new_state()
    sv.state_init(st, 0.001)
    return st


def test_batch_of_point_and_spectral_slabs_replays_the_oracle():
    """A context mixing the point opacity law and the spectral group averages
    (a sigma_R table of its own for the whole context): one replayed W-cycle
    step per slab against its own oracle run at 1e-10."""
    slabs = [inputs.make_slab(30, 16, 8, dt=0.004, nu_lo=1e-3, nu_hi=30.0, opacity=inputs.OPAC_SPECTRAL),
             inputs.make_slab(45, 32, 8, dt=0.004),
             inputs.make_slab(20, 16, 4, dt=0.004, C1=5.0, C2=0.5, opacity=inputs.OPAC_SPECTRAL)]
    levels = [[s.ng, s.ng // 8, 1] for s in slabs]
    cfg = inputs.SolverCfg(levels=[0, 0, 1], cycle=inputs.CYCLE_W, lmax=2)
    refs = []
    for s, lv in zip(slabs, levels):
        pb = mlqd.problem_from_slab(s)
        stats = mlqd.Stats()
        ref = mlqd.step(pb, lv, mlqd.schedule(3, cfg.cycle), cfg.lmax, cfg.eps, cfg.eps_inner,
                        mlqd.initial_state(pb, 0.001), stats=stats)
        refs.append((ref, stats.counts[0]))
    note("mixed point / spectral batch of 3 slabs, one replayed W step")
    sv = binding.Solver(slabs, levels, cfg)
    st = _init(sv)
    sv.step(st, replay=[c for _, c in refs])
    for k, (ref, _) in enumerate(refs):
        T, E, I = _slab_view(sv, st, k)
        assert_close(f"slab {k} T", T, ref.T, 1e-10, atol_scale=0.0)
        assert_close(f"slab {k} E", E.reshape(ref.E.shape), ref.E, 1e-10)
        assert_close(f"slab {k} I", I.reshape(ref.I.shape), ref.I, 1e-10)
    sv.close()
